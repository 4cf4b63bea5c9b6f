// Philox4x64-10 counter-based generator for the GPU path (Salmon, Moraes, Dror,
// Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11).
//
// The random samples R_f of the method (initial loading, the free-flight times
// of Eq. (5), the null-collision selection following Eq. (6), the impact
// parameter and azimuth of Eq. (10), the sputter yield and emission laws) are
// drawn from counter = (particle id, step or event index, tag, aux) under
// key = (seed, stream), tag = species * 256 + purpose, so a particle's numbers do
// not depend on which thread or slot handles it.
//
// One call gives four 64-bit words; word w yields two uniforms in (0, 1):
//   hi(w) = ((w >> 41) + 0.5) 2^-23,   lo(w) = (((w >> 9) & (2^23 - 1)) + 0.5) 2^-23,
// in the order hi(w0), lo(w0), hi(w1), ..., lo(w3).  Each value is exact in FP32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {

enum : uint32_t { SP_E = 0, SP_I = 1, SP_AL = 2, SP_YIELD = 3 };
enum : uint32_t { PU_INIT = 1, PU_SKIP = 2, PU_COLL = 3, PU_ION = 5,
                  PU_CHILD = 6, PU_TP_SRC = 16, PU_TP_EVT = 17, PU_YIELD = 32 };

__host__ __device__ constexpr uint64_t rng_tag(uint32_t species, uint32_t purpose) {
  return (uint64_t)species * 256u + purpose;
}

struct Words4 { uint64_t w0, w1, w2, w3; };

// The 128-bit product a * b from four 32 x 32 -> 64 multiply-adds
// (v_mad_u64_u32): t and u absorb the carries of the middle partial products,
// and none of the sums can overflow 64 bits.
__device__ __forceinline__ void mulhilo64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
  const uint64_t a0 = (uint32_t)a, a1 = a >> 32, b0 = (uint32_t)b, b1 = b >> 32;
  const uint64_t p00 = a0 * b0;
  const uint64_t t = a0 * b1 + (p00 >> 32);
  const uint64_t u = a1 * b0 + (uint32_t)t;
  lo = (u << 32) | (uint32_t)p00;
  hi = a1 * b1 + (t >> 32) + (u >> 32);
}

__device__ __forceinline__ Words4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                uint64_t k0, uint64_t k1) {
  const uint64_t MA = 0xD2E7470EE14C6C93ull, MB = 0xCA5A826395121157ull;
  const uint64_t KA = 0x9E3779B97F4A7C15ull, KB = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t pa_hi, pa_lo, pb_hi, pb_lo;
    mulhilo64(MA, c0, pa_hi, pa_lo);
    mulhilo64(MB, c2, pb_hi, pb_lo);
    const uint64_t n0 = pb_hi ^ c1 ^ k0;
    const uint64_t n2 = pa_hi ^ c3 ^ k1;
    c0 = n0; c1 = pb_lo; c2 = n2; c3 = pa_lo;
    k0 += KA; k1 += KB;
  }
  return Words4{c0, c1, c2, c3};
}

template <typename R>
__device__ __forceinline__ R u_hi(uint64_t w) {
  return ((R)(uint32_t)(w >> 41) + (R)0.5) * (R)1.1920928955078125e-07;   // 2^-23
}
template <typename R>
__device__ __forceinline__ R u_lo(uint64_t w) {
  return ((R)(uint32_t)((w >> 9) & 0x7FFFFFu) + (R)0.5) * (R)1.1920928955078125e-07;
}

// The 8 uniforms of one call.
template <typename R>
struct Uniforms8 {
  R u[8];
  __device__ __forceinline__ explicit Uniforms8(const Words4& w) {
    u[0] = u_hi<R>(w.w0); u[1] = u_lo<R>(w.w0);
    u[2] = u_hi<R>(w.w1); u[3] = u_lo<R>(w.w1);
    u[4] = u_hi<R>(w.w2); u[5] = u_lo<R>(w.w2);
    u[6] = u_hi<R>(w.w3); u[7] = u_lo<R>(w.w3);
  }
  __device__ __forceinline__ R operator[](int i) const { return u[i]; }
};

template <typename R>
__device__ __forceinline__ Uniforms8<R> draw8(uint64_t id, uint64_t index, uint64_t tag,
                                              uint64_t key0, uint64_t key1, uint64_t aux = 0) {
  return Uniforms8<R>(philox4x64_10(id, index, tag, aux, key0, key1));
}

}  // namespace pm
