// PIC/MCC kernels for gfx950 (Sec. IV.A, Fig. 4 of arXiv:1607.04069).
//
// One time step is two launches.  k_step (the push) stages the field of step l
// in LDS and advances the cell-sorted particles of its tiles: gather, leapfrog
// push of Eqs. (3)-(4), wall absorption, and the deposit of the new positions
// into an LDS tile of the next step's charge (linear weighting, integer units of
// 2^-32 particle, so the sum is exact and independent of order); a particle
// whose null-collision examination falls on this step is appended to a
// candidate list instead of being touched further.  k_mcc (the collisions) walks
// the candidate lists: selection of Eq. (6), kinematics, births, the next
// waiting time; its last workgroup to finish solves Poisson's equation for step
// l+1, accumulates the diagnostics and publishes the step counter.  Every K
// steps a counting sort by cell compacts the slots.  An RF cycle is the chain of
// these launches captured in a HIP graph; the _batch forms run many independent
// cases in the same launches from per-case work lists.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <stdint.h>

#include "philox.h"
#include "pm_internal.h"

namespace pm {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ float dsqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double dsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float dlog(float x) { return logf(x); }
__device__ __forceinline__ double dlog(double x) { return log(x); }
__device__ __forceinline__ float dacos(float x) { return acosf(x); }
__device__ __forceinline__ double dacos(double x) { return acos(x); }
__device__ __forceinline__ void dsincospi(float x, float* s, float* c) { sincospif(x, s, c); }
__device__ __forceinline__ void dsincospi(double x, double* s, double* c) { sincospi(x, s, c); }

template <typename R>
struct Pair { R a, b; };

// rint((xt - j) 2^32): the charge share of node j+1 in units of 2^-32 particle
__device__ __forceinline__ uint64_t frac_fixed(float f) {
  return (uint64_t)__float2uint_rn(f * 4294967296.0f);
}
__device__ __forceinline__ uint64_t frac_fixed(double f) {
  return (uint64_t)rint(f * 4294967296.0);
}

// Box-Muller pair from two uniforms
template <typename R>
__device__ __forceinline__ void box_muller(R ua, R ub, R& n0, R& n1) {
  const R r = dsqrt((R)-2 * dlog(ua));
  R s, c;
  dsincospi((R)2 * ub, &s, &c);
  n0 = r * c;
  n1 = r * s;
}

// Isotropic unit vector of the VHS scattering law: b/b_max = sqrt(Ua),
// chi = 2 arccos(b/b_max) gives cos chi = 2 Ua - 1; psi = 2 pi Ub.
template <typename R>
__device__ __forceinline__ void iso_dir(R ua, R ub, R& nx, R& ny, R& nz) {
  const R cc = (R)2 * ua - (R)1;
  const R sc = dsqrt(fmax((R)0, (R)1 - cc * cc));
  R sp, cp;
  dsincospi((R)2 * ub, &sp, &cp);
  nx = cc;
  ny = sc * cp;
  nz = sc * sp;
}

// Next examination after step `step`: geometric waiting time of the per-step
// checks R_f <= P_c,tot, G = ceil(ln u / ln(1 - P)) >= 1, as evaluated in FP64,
// cut at kWaitCap steps (the law has no memory, so a cut wait is simply drawn
// afresh at the cut).  Returns the 16-bit examination code.  The ratio is first
// taken in FP32 (u has 24 significant bits, so it is exact in FP32); its error
// stays below 1e-6 relative, so unless it lies that close to an integer its
// ceiling is the FP64 one, and only then is FP64 used.  A species without
// collisions is never examined (its code is not read).
__device__ __forceinline__ uint16_t next_candidate(double u, int64_t step, double log1m_p) {
  if (log1m_p == 0.0) return 0;
  const float rf = logf((float)u) / (float)log1m_p;
  double ratio = (double)rf;
  if (!(fabsf(rf - rintf(rf)) > 1e-6f * fmaxf(rf, 1.0f))) ratio = log(u) / log1m_p;
  const double G = fmax(ceil(ratio), 1.0);
  const bool cut = !(G <= (double)kWaitCap);
  const int64_t nx = step + (cut ? (int64_t)kWaitCap : (int64_t)G);
  return (uint16_t)(((uint32_t)nx & 0x7FFFu) | (cut ? kRedraw : 0u));
}

template <typename R>
__device__ __forceinline__ R ln_x_over_x(R eps, double eth, double sigma0) {
  const R x = eps / (R)eth;
  return x > (R)1 ? (R)sigma0 * dlog(x) / x : (R)0;
}

// Source voltage at t_l: the fundamental and its harmonic (Sec. III).
__device__ __forceinline__ double drive_voltage(const CaseConst& c, int64_t step) {
  const int64_t ph = step % c.Nt;
  const double wt = 6.283185307179586 * (double)ph / (double)c.Nt;
  return c.V0 * cos(wt + c.phase) + c.V2 * cos(2.0 * wt + c.phase2);
}

__device__ __forceinline__ void add128(uint64_t* acc, int64_t v) {
  const uint64_t lo = acc[0];
  const uint64_t nlo = lo + (uint64_t)v;
  acc[0] = nlo;
  acc[1] += (uint64_t)(nlo < lo) + (v < 0 ? ~0ull : 0ull);
}

// Inclusive scan over a 64-lane wavefront (fixed combination order).
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  return v;
}

// Inclusive scan over the 256 threads of a workgroup; *total receives the sum.
// s_w is 4 entries of LDS.  The combination order is fixed, so FP64 results are
// reproducible run to run.
template <typename T>
__device__ __forceinline__ T block_incl_scan(T v, T* s_w, T* total) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const T x = wave_incl_scan(v, lane);
  if (lane == 63) s_w[w] = x;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kBlock / 64; ++i) {
    if (i < w) off += s_w[i];
    tot += s_w[i];
  }
  __syncthreads();
  if (total) *total = tot;
  return x + off;
}

// Wait until every memory operation this thread issued has been performed.
// Cross-workgroup data inside a launch is only ever touched through device-scope
// atomics (performed at the coherent level) and read back with device-scope
// atomic loads, so completing the atomics is all the last workgroup needs; a
// device-scope fence would also write back the whole L2 of this XCD for the
// plain particle stores, which only the next launch reads.
__device__ __forceinline__ void complete_memory_ops() { __builtin_amdgcn_s_waitcnt(0); }

// ------------------------------------------------------------------ field solve
// Second-order finite-difference Poisson equation on nodes 0..N with
// Phi_0 = V and Phi_N = 0 ('EM Field Solver' of Sec. IV.A).  With
// D_m = Phi_{m+1} - Phi_m the interior equations read D_m - D_{m-1} = -c q_m,
// c = e w dx / (2^32 eps0), so D_m = D_0 - c S_m with S_m = q_1 + ... + q_m and
// Phi_N = 0 fixes D_0 = (c sum_{m=1}^{N-1} S_m - V) / N.  For integer q the
// prefix sums are exact; the only rounding is in the final FP64 products.
// E_m = -(D_m + D_{m-1}) / (2 dx) inside, half-cell Gauss forms at the walls.
// With circ_den > 0 the driven electrode sits behind the blocking capacitor and
// Phi_0 is unknown: its surface charge by Gauss over the half cell,
// eps0 (Phi_0 - Phi_1) / dx - rho_0 dx / 2 = (eps0 / L) Phi_0 - qs (T / N + q_0)
// with qs = e w / 2^32, must equal circ_num - cb Phi_0 (what the circuit and the
// absorbed particles delivered), so Phi_0 = (circ_num + qs (T / N + q_0)) /
// circ_den with circ_den = eps0 / L + cb.  *V0_out receives the Phi_0 used.
// Runs on one workgroup; sq holds q_0..q_N in LDS; writes E to sE (LDS).
constexpr int kMaxPer = (kMaxCells + kBlock - 1) / kBlock;   // interior nodes per thread

template <typename QT, typename Load>
__device__ void solve_field(const CaseConst& c, Load qload, double V, double* sE,
                            QT* s_wq, double* s_wd, double* sD, double* phi_out, double circ_num = 0.0,
                            double circ_den = 0.0, double* V0_out = nullptr) {
  const int N = c.N, tid = threadIdx.x;
  const int M = N - 1;
  const int per = (M + kBlock - 1) / kBlock;
  const int b = 1 + tid * per;
  const int e = min(b + per, N);
  QT q[kMaxPer];
  QT loc = 0;
#pragma unroll
  for (int t = 0; t < kMaxPer; ++t) {
    q[t] = (t < per && b + t < e) ? qload(b + t) : (QT)0;
    loc += q[t];
  }
  QT S_all;
  const QT S_before = block_incl_scan<QT>(loc, s_wq, &S_all) - loc;   // S_{b-1}; S_{N-1}
  double tl = 0.0;
  {
    QT S = S_before;
#pragma unroll
    for (int t = 0; t < kMaxPer; ++t) { S += q[t]; if (t < per && b + t < e) tl += (double)S; }
  }
  double T;
  block_incl_scan<double>(tl, s_wd, &T);
  const double cp = c.c_phi, dx = c.dx;
  if (circ_den > 0.0)
    V = (circ_num + c.e_w * 2.3283064365386963e-10 * (T / (double)N + (double)qload(0))) / circ_den;
  if (V0_out && tid == 0) *V0_out = V;
  const double D0 = (cp * T - V) / (double)N;
  {
    QT Sp = S_before;
#pragma unroll
    for (int t = 0; t < kMaxPer; ++t) {
      if (!(t < per && b + t < e)) break;
      const int m = b + t;
      const QT Sm = Sp + q[t];
      const double Dm = D0 - cp * (double)Sm;
      const double Dm1 = D0 - cp * (double)Sp;
      sE[m] = -(Dm + Dm1) / (2.0 * dx);
      if (sD) sD[m] = Dm;
      Sp = Sm;
    }
  }
  if (tid == 0) {
    sE[0] = -(D0 + cp * (double)qload(0)) / dx;
    const double DN1 = D0 - cp * (double)S_all;
    sE[N] = (-DN1 + cp * (double)qload(N)) / dx;
    if (sD) sD[0] = D0;
  }
  __syncthreads();
  if (phi_out) {
    // Phi_m = V + D_0 + ... + D_{m-1}: fixed-order FP64 scan of D over m = 0..N-1
    const int per2 = (N + kBlock - 1) / kBlock;
    const int b2 = tid * per2, e2 = min(b2 + per2, N);
    double l2 = 0.0;
    for (int m = b2; m < e2; ++m) l2 += sD[m];
    double run = V + (block_incl_scan<double>(l2, s_wd, nullptr) - l2);
    if (tid == 0) phi_out[0] = V;
    for (int m = b2; m < e2; ++m) { run += sD[m]; phi_out[m + 1] = m + 1 == N ? 0.0 : run; }
    __syncthreads();
  }
}

// Store (E'_j, E'_{j+1} - E'_j) per cell with E' = E (-e/m_e) dt^2 / dx, the
// electron's velocity change in cells per step; a species s multiplies the
// interpolated value by kpush[s] / kpush[0] (1 for electrons).
template <typename R>
__device__ void publish_field(const CaseConst& c, const double* sE, Pair<R>* Epair, double* E64) {
  const int N = c.N;
  for (int j = threadIdx.x; j < N; j += kBlock) {
    const double e0 = sE[j], e1 = sE[j + 1];
    Pair<R> pr;
    pr.a = (R)(c.kpush[0] * e0);
    pr.b = (R)(c.kpush[0] * (e1 - e0));
    Epair[j] = pr;
  }
  if (E64)
    for (int m = threadIdx.x; m <= N; m += kBlock) E64[m] = sE[m];
}

// LDS working set of the field solve, carved from a raw buffer of
// field_lds_bytes(N) (the step epilogue reuses the step's dead tiles).
struct FieldLds {
  double* E;
  double* D;
  int64_t* wq;
  double* wd;
};
__device__ __forceinline__ FieldLds carve_field(unsigned char* p, int N) {
  FieldLds v;
  v.E = reinterpret_cast<double*>(p);
  v.D = v.E + N + 1;
  v.wq = reinterpret_cast<int64_t*>(v.D + N + 1);
  v.wd = reinterpret_cast<double*>(v.wq + 8);
  return v;
}

// Solve from the charge buffer of step `step` and publish E for that step.
template <typename R>
__device__ __forceinline__ void field_for_step(const KArgs<R>& A, int64_t step, bool atomic_q, double* phi_out,
                               FieldLds& L) {
  const CaseConst& c = A.c;
  const int nodes = c.N + 1;
  const int64_t* Q = A.g.Q + qbuf_index(step, 0) * 2 * nodes;
  const bool self = !(c.flags & 1u);
  auto qload = [&](int m) -> int64_t {
    if (!self) return 0;
    if (atomic_q)
      return __hip_atomic_load(&Q[nodes + m], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
             __hip_atomic_load(&Q[m], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return Q[nodes + m] - Q[m];
  };
  // the driven electrode behind the blocking capacitor, once its reference
  // surface charge is known (the capacitor is uncharged at the first solve)
  Ctrl* C = A.ctrl;
  const double Vs = drive_voltage(c, step);
  double num = 0.0, den = 0.0;
  if (c.cb > 0.0 && C->circ_ready) {
    const int64_t n_net = atomic_q ? __hip_atomic_load(&C->n_abs_net, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                   : C->n_abs_net;
    num = C->sigma_init + c.cb * Vs + c.e_w * (double)n_net;
    den = c.cgap + c.cb;
  }
  double V0 = Vs;
  solve_field<int64_t>(c, qload, Vs, L.E, L.wq, L.wd, L.D, phi_out, num, den, &V0);
  publish_field<R>(c, L.E, reinterpret_cast<Pair<R>*>(A.g.Epair), A.g.E64);
  if (threadIdx.x == 0) {
    C->phi0 = V0;
    if (c.cb > 0.0 && !C->circ_ready) {
      C->sigma_init = c.eps0 * L.E[0];
      C->circ_ready = 1u;
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------------ loading
// Uniform positions and Maxwellian velocities (Box-Muller), Sec. IV.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_load(KArgs<R> A, int64_t np_e, int64_t np_i,
                                                 double sig_e, double sig_i) {
  const CaseConst& c = A.c;
  const int64_t gi = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int s = blockIdx.y;
  const int64_t n = s ? np_i : np_e;
  if (gi >= n) return;
  const uint64_t id = (uint64_t)gi;
  const Uniforms8<R> U = draw8<R>(id, 0, rng_tag(s, PU_INIT), c.seed, c.case_id);
  const R sig = (R)((s ? sig_i : sig_e) * c.inv_v_scale);
  R n0, n1, n2, n3;
  box_muller<R>(U[1], U[2], n0, n1);
  box_muller<R>(U[3], U[4], n2, n3);
  A.p.xt[s][0][gi] = (R)c.N * U[0];
  A.p.ux[s][0][gi] = sig * n0;
  A.p.cold[s][0][gi] = Cold<R>{sig * n1, sig * n2, id};
  const Uniforms8<double> Us = draw8<double>(id, ~0ull, rng_tag(s, PU_SKIP), c.seed, c.case_id);
  A.p.next[s][0][gi] = next_candidate(Us[0], -1, c.log1m_p[s]);
}

// Charge of every live particle into the read buffer of the current step, with
// per-cell counts for the sort (set-up path; plain global atomics).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_deposit_all(KArgs<R> A) {
  const CaseConst& c = A.c;
  const Ctrl* C = A.ctrl;
  const int s = blockIdx.y;
  const int64_t n = C->n_range[s];
  const uint32_t buf = C->buf;
  const int nodes = c.N + 1;
  int64_t* Q = A.g.Q + qbuf_index(C->step, 0) * 2 * nodes + s * nodes;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock) {
    const R x = A.p.xt[s][buf][k];
    if (!(x >= (R)0)) continue;
    const int j = (int)x;
    const uint64_t W = frac_fixed(x - (R)j);
    atomicAdd((unsigned long long*)&Q[j], (unsigned long long)((1ull << 32) - W));
    atomicAdd((unsigned long long*)&Q[j + 1], (unsigned long long)W);
    atomicAdd(&A.g.cell_count[s * c.N + j], 1u);
  }
}

// 128-bit accumulator (lo, hi) shared by many threads: the carry out of each
// atomic add to the low word is known from the value it returned, so the two
// words together always hold the exact sum modulo 2^128.
__device__ __forceinline__ void atomic_add128(uint64_t* acc, int64_t v) {
  const uint64_t a = (uint64_t)v;
  const uint64_t old = atomicAdd((unsigned long long*)&acc[0], (unsigned long long)a);
  const uint64_t hi = (uint64_t)(old + a < old) + (v < 0 ? ~0ull : 0ull);
  if (hi) atomicAdd((unsigned long long*)&acc[1], (unsigned long long)hi);
}

// Particle flux sample of the state that step l starts from (positions x^(l),
// velocities v_x^(l-1/2) after the collisions of step l-1): each live particle
// adds u (1 - f) and u f to the nodes j and j+1 of its cell by the same linear
// weighting as the charge, u in 2^-40 cells per step (an ion's thermal u is
// near 1e-4, so a coarser unit would round it at the 1e-6 level), int64 fixed
// point so that the sums do not depend on the order (the two shares add up to
// round(u 2^40) exactly; kFluxFlushSlots slots stay below 2^63 for |u| < 2^9
// cells per step).  The push takes the samples (step_block with kFlux): a
// workgroup sums its slots in an LDS tile and adds the touched nodes to the
// 128-bit sums of the step's phase bin at least every kFluxFlushSlots slots.
constexpr int64_t kFluxFlushSlots = 16384;

// round(v 2^sh) for v < 2^57 (halves away from zero; 0 once the shift passes 63)
__device__ __forceinline__ long long shift_round(uint64_t v, int sh) {
  if (sh >= 0) return (long long)(v << sh);
  const int r = -sh;
  if (r > 63) return 0;
  return (long long)((v + (1ull << (r - 1))) >> r);
}

// A particle's two flux shares (node j, node j+1) in 2^-40 cells per step.  In
// FP32 the velocity is m 2^(e-150) exactly, so both shares are integer products
// and shifts of the mantissa (the double-precision products and conversions
// this replaces cost as much as the loads); FP64 rounds the products once.
template <typename R>
__device__ __forceinline__ void flux_shares(R x, int j, R u, long long& a0, long long& a1) {
  const uint64_t W = frac_fixed(x - (R)j);                 // weight of node j+1, 2^-32 units
  if constexpr (sizeof(R) == 4) {
    const uint32_t bits = __float_as_uint(u);
    const int ex = (int)((bits >> 23) & 0xFFu);
    a0 = a1 = 0;
    if (ex == 0 || ex > 148) return;                      // |u| < 2^-126 (below the unit) or >= 2^22
    const uint64_t m = (uint64_t)((bits & 0x7FFFFFu) | 0x800000u);
    long long cu = shift_round(m, ex - 110);               // m 2^(e-150) 2^40
    long long c1 = shift_round(m * W, ex - 142);           // m 2^(e-150) W 2^-32 2^40
    if (bits >> 31) {
      cu = -cu;
      c1 = -c1;
    }
    a0 = cu - c1;
    a1 = c1;
  } else {
    const double ud = (double)u;
    const long long cu = (long long)rint(ud * 1099511627776.0);      // 2^40
    a1 = (long long)rint(ud * (double)W * 256.0);                     // W in 2^-32, times 2^8
    a0 = cu - a1;
  }
}

// Exclusive scan of the per-cell counts into sort offsets (one workgroup).
__device__ void scan_cells(const CaseConst& c, GridPtrs g, Ctrl* C, int64_t* s_w) {
  const int N = c.N, tid = threadIdx.x;
  const int per = (N + kBlock - 1) / kBlock;
  const int b = tid * per, e = min(b + per, N);
  for (int s = 0; s < 2; ++s) {
    uint32_t* cnt = g.cell_count + s * N;
    uint32_t* off = g.cell_off + s * N;
    uint32_t k[kMaxPer];
    int64_t loc = 0;
#pragma unroll
    for (int t = 0; t < kMaxPer; ++t) {
      k[t] = (t < per && b + t < e) ? __hip_atomic_load(&cnt[b + t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
      loc += k[t];
    }
    int64_t tot;
    int64_t run = block_incl_scan<int64_t>(loc, s_w, &tot) - loc;
#pragma unroll
    for (int t = 0; t < kMaxPer; ++t) {
      if (!(t < per && b + t < e)) break;
      off[b + t] = (uint32_t)run;
      run += k[t];
      cnt[b + t] = 0;
    }
    if (tid == 0) C->n_live[s] = tot;
    // the count is whole: the banks' live deltas of the step are in it
    if (tid < kBanks) bank_of(g, tid)->n_live[s] = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_scan_cells(CaseConst c, GridPtrs g, Ctrl* C) {
  __shared__ int64_t s_w[8];
  scan_cells(c, g, C, s_w);
}

// Counting-sort scatter by cell into the other buffer; drops dead slots.
// Each workgroup ranks a chunk of 2048 slots in LDS, reserves its share of
// every touched cell with one global atomic, and copies its particles.
constexpr int kSortPer = 8;
template <typename R>
__device__ __forceinline__ void sort_block(const KArgs<R>& A, int bid, int nblk, unsigned char* smem) {
  const CaseConst& c = A.c;
  const int N = c.N, tid = threadIdx.x;
  uint32_t* lh = reinterpret_cast<uint32_t*>(smem);     // [2][N] chunk histogram
  uint32_t* lb = lh + 2 * N;                              // [2][N] chunk base in cell
  __shared__ int s_last;
  Ctrl* C = A.ctrl;
  const uint32_t buf = C->buf;
  const int64_t n0 = C->n_range[0], n1 = C->n_range[1];
  const int64_t chunk = (int64_t)kBlock * kSortPer;
  // chunks never straddle the species boundary, so array pointers are uniform
  const int64_t ch0 = (n0 + chunk - 1) / chunk, ch1 = (n1 + chunk - 1) / chunk;
  for (int64_t cix = bid; cix < ch0 + ch1; cix += nblk) {
    const int s = cix >= ch0;
    const int64_t base = (s ? cix - ch0 : cix) * chunk;
    const int64_t ns = s ? n1 : n0;
    for (int i = tid; i < 2 * N; i += kBlock) lh[i] = 0;
    __syncthreads();
    int cell[kSortPer];
    uint32_t rank[kSortPer];
    const R PM_GLOBAL* __restrict__ xs = A.p.xt[s][buf];
#pragma unroll
    for (int q = 0; q < kSortPer; ++q) {
      const int64_t k = base + q * kBlock + tid;
      cell[q] = -1;
      if (k < ns) {
        const R x = xs[k];
        if (x >= (R)0) {
          cell[q] = s * N + (int)x;
          rank[q] = atomicAdd(&lh[cell[q]], 1u);
        }
      }
    }
    __syncthreads();
    for (int i = tid; i < 2 * N; i += kBlock)
      if (lh[i]) lb[i] = atomicAdd(&A.g.cell_count[i], lh[i]) + A.g.cell_off[i];
    __syncthreads();
    const uint32_t o = buf ^ 1u;
#pragma unroll
    for (int q = 0; q < kSortPer; ++q) {
      if (cell[q] < 0) continue;
      const int64_t k = base + q * kBlock + tid;
      const int64_t d = (int64_t)lb[cell[q]] + rank[q];
      A.p.xt[s][o][d] = xs[k];
      A.p.ux[s][o][d] = A.p.ux[s][buf][k];
      A.p.cold[s][o][d] = A.p.cold[s][buf][k];
      A.p.next[s][o][d] = A.p.next[s][buf][k];
    }
    __syncthreads();
  }
  complete_memory_ops();
  __syncthreads();
  if (tid == 0)
    s_last = nblk == 1 ||      // a lone workgroup is the last without the round trip
             __hip_atomic_fetch_add(&C->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (uint32_t)nblk - 1;
  __syncthreads();
  if (!s_last) return;
  for (int i = tid; i < 2 * N; i += kBlock) A.g.cell_count[i] = 0;
  if (tid == 0) {
    C->buf = buf ^ 1u;
    for (int s = 0; s < 2; ++s) {
      const int64_t nl = __hip_atomic_load(&C->n_live[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      C->n_range[s] = nl;
      C->n_alloc[s] = nl;
    }
    C->done = 0;
  }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_sort_scatter(KArgs<R> A) {
  extern __shared__ __align__(16) unsigned char smem[];
  sort_block<R>(A, blockIdx.x, gridDim.x, smem);
}

// Many cases in one launch: work[b] = case << 16 | workgroup within the case.
// The case table is read through the constant address space: those loads are
// scalar and known not to change during the launch, so the compiler re-reads
// a field where it is needed instead of holding every field of the table in
// registers (as it does for a kernel argument).
template <typename R>
__device__ inline const KArgs<R>& case_of(uintptr_t table, uint32_t ci) {
  using CP = const KArgs<R> __attribute__((address_space(4)))*;
  return *(const KArgs<R>*)((CP)table + ci);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_sort_batch(uintptr_t cases,
                                                       const uint32_t* __restrict__ work,
                                                       const uint32_t* __restrict__ nblocks) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t w = work[blockIdx.x];
  if (w == kIdleWork) return;
  sort_block<R>(case_of<R>(cases, w >> 16), (int)(w & 0xFFFFu), (int)nblocks[w >> 16], smem);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_field(KArgs<R> A, int want_phi) {
  extern __shared__ __align__(16) unsigned char smem[];
  FieldLds L = carve_field(smem, A.c.N);
  field_for_step<R>(A, A.ctrl->step, false, want_phi ? A.g.phi64 : nullptr, L);
}

// ------------------------------------------------------------------ the step
// One time step is two launches.  The push kernel (k_step) gathers, pushes,
// applies the walls and deposits every particle of its range, and lists the
// null-collision candidates; the collision kernel (k_mcc) runs the candidates
// (Eq. (6) and the selection rule), deposits the births, and its last workgroup
// solves the field of the next step.  Splitting the two keeps the long,
// register-hungry collision path out of the streaming loop, whose occupancy
// then hides the memory latency of the particle stream.
enum { CN_LIVE = 0, CN_CAND = 1, CN_EL = 3, CN_EXC = 4, CN_ION = 5, CN_CX = 6, CN_OVER = 7,
       CN_ABS = 9, CN_BIRTH = 13, CN_N = 16 };

// Ions absorbed by a wall are tallied (impact energy and angle) after the
// workgroup's loop, from an LDS list of their slots; in the meantime the slot
// holds x = -3 (target) or -4 (substrate) and v_x^(l+1/2), and a list that
// overflows is recovered by a rescan of the range for those marks.
constexpr int kWallCap = 256;
constexpr float kMarkTarget = -3.0f, kMarkSubstrate = -4.0f;

// Candidates found by a push workgroup wait in LDS, with the x^(l+1) and
// v_x^(l+1/2) the push gave them, and go to the case's per-species candidate
// list in global memory in blocks: one global atomic per flush, so that the
// list's counter sees a few thousand atomics per step however large the case.
// A candidate that finds the LDS list full appends itself directly.
template <typename R>
constexpr int kCandCap = sizeof(R) == 4 ? 704 : 512;

template <typename R>
struct StepShared {
  uint32_t cnt[CN_N];
  uint32_t qn;
  uint32_t qbase;
  uint32_t wn;
  uint32_t q[kCandCap<R>];    // slot indices of this species' candidates
  XU<R> qxu[kCandCap<R>];     // and their new x and v_x
  uint32_t wall[kWallCap];    // slot indices of absorbed ions
};

struct MccShared {
  uint32_t cnt[CN_N];
  int last;
};

// Candidates a collision lane loads together before computing them.
constexpr int kMccBatch = 2;

// Impact energy and angle of an ion absorbed at electrode el (Sec. IV.A 'Wall
// Interaction'): the 1 eV energy and 0.25 degree angle histograms and the
// energy sum.  un, uy, uz: its velocity in cells per step.
template <typename R>
__device__ void tally_ion(const KArgs<R>& A, int el, R un, R uy, R uz) {
  const CaseConst& c = A.c;
  const double u2 = (double)un * un + (double)uy * uy + (double)uz * uz;
  const R E = (R)(c.ion_e_factor * u2);
  const R ct = (R)(fabs((double)un) / sqrt(u2));
  const R th = dacos(fmin(ct, (R)1)) * (R)57.29577951308232;
  const int eb = (int)fmin((double)E, (double)(c.n_ebins - 1));
  const int ab = (int)fmin((double)th / 0.25, (double)(kAngleBins - 1));
  atomicAdd((unsigned long long*)&A.g.iedf[el * c.n_ebins + eb], 1ull);
  atomicAdd((unsigned long long*)&A.g.iadf[el * kAngleBins + ab], 1ull);
  const int ne4 = (c.n_ebins + kIeadEGroup - 1) / kIeadEGroup;
  atomicAdd((unsigned long long*)&A.g.iead[((int64_t)el * ne4 + eb / kIeadEGroup) * kIeadABins + ab / 4], 1ull);
  atomicAdd((unsigned long long*)&A.ctrl->ion_e_fx[el], (unsigned long long)(int64_t)rint((double)E * 1048576.0));
}

// Tally the marked ions of the workgroup's tiles t0, t0 + stride, ... of the ion
// slots [g_lo, g_hi) of the numbering (uniform call): from the LDS list, or by a
// rescan of those tiles when it overflowed; each slot ends dead (x = -1).
template <typename R, int64_t kTile>
__device__ __forceinline__ void tally_ion_walls(const KArgs<R>& A, uint32_t buf, int64_t t0, int64_t stride,
                                                int64_t g_lo, int64_t g_hi, StepShared<R>& sh) {
  __syncthreads();
  const uint32_t n = sh.wn;
  R PM_GLOBAL* xs = A.p.xt[1][buf];
  if (n <= (uint32_t)kWallCap) {
    for (uint32_t i = threadIdx.x; i < n; i += kBlock) {
      const int64_t k = sh.wall[i];
      const Cold<R> cr = A.p.cold[1][buf][k];
      tally_ion<R>(A, xs[k] == (R)kMarkTarget ? 0 : 1, A.p.ux[1][buf][k], cr.uy, cr.uz);
      xs[k] = (R)-1;
    }
  } else {
    for (int64_t t = t0; t * kTile < g_hi; t += stride) {
      const int64_t k_hi = min((t + 1) * kTile, g_hi) - g_lo;
      for (int64_t k = max(t * kTile, g_lo) - g_lo + threadIdx.x; k < k_hi; k += kBlock) {
        const R x = xs[k];
        if (x == (R)kMarkTarget || x == (R)kMarkSubstrate) {
          const Cold<R> cr = A.p.cold[1][buf][k];
          tally_ion<R>(A, x == (R)kMarkTarget ? 0 : 1, A.p.ux[1][buf][k], cr.uy, cr.uz);
          xs[k] = (R)-1;
        }
      }
    }
  }
  __syncthreads();
}

// Add the step's counters of one workgroup to its counter bank (the net charge
// absorbed at the driven electrode, read by the next field solve, goes to the
// control block itself; few workgroups have any).
__device__ __forceinline__ void flush_counters(Ctrl* C, CtrBank* B, const uint32_t* cn) {
  if (cn[CN_LIVE]) atomicAdd((unsigned long long*)&B->particle_steps, (unsigned long long)cn[CN_LIVE]);
  if (cn[CN_CAND]) atomicAdd((unsigned long long*)&B->candidates[0], (unsigned long long)cn[CN_CAND]);
  if (cn[CN_CAND + 1]) atomicAdd((unsigned long long*)&B->candidates[1], (unsigned long long)cn[CN_CAND + 1]);
  if (cn[CN_EL]) atomicAdd((unsigned long long*)&B->collisions[0], (unsigned long long)cn[CN_EL]);
  if (cn[CN_EXC]) atomicAdd((unsigned long long*)&B->collisions[1], (unsigned long long)cn[CN_EXC]);
  if (cn[CN_ION]) atomicAdd((unsigned long long*)&B->collisions[2], (unsigned long long)cn[CN_ION]);
  if (cn[CN_CX]) atomicAdd((unsigned long long*)&B->collisions[4], (unsigned long long)cn[CN_CX]);
  if (cn[CN_OVER]) atomicAdd((unsigned long long*)&B->overflow[0], (unsigned long long)cn[CN_OVER]);
  if (cn[CN_OVER + 1]) atomicAdd((unsigned long long*)&B->overflow[1], (unsigned long long)cn[CN_OVER + 1]);
  for (int q = 0; q < 4; ++q)
    if (cn[CN_ABS + q]) atomicAdd((unsigned long long*)&B->absorbed[q >> 1][q & 1], (unsigned long long)cn[CN_ABS + q]);
  const int64_t net0 = (int64_t)cn[CN_ABS + 2] - (int64_t)cn[CN_ABS];   // Ar+ minus e at electrode 0
  if (net0) atomicAdd((unsigned long long*)&C->n_abs_net, (unsigned long long)net0);
  const uint64_t nb = (uint64_t)cn[CN_BIRTH] + cn[CN_BIRTH + 1];
  if (nb) atomicAdd((unsigned long long*)&B->births, (unsigned long long)nb);
  for (int s = 0; s < 2; ++s) {
    const int64_t d = (int64_t)cn[CN_BIRTH + s] - (int64_t)cn[CN_ABS + 2 * s] - (int64_t)cn[CN_ABS + 2 * s + 1];
    if (d) atomicAdd((unsigned long long*)&B->n_live[s], (unsigned long long)d);
  }
}

// Add a super-particle at x (cells) to the global charge of species s for the
// next step (a birth), and to the cell histogram of the next sort.
template <typename R>
__device__ __forceinline__ void deposit_global(int64_t* Qs, uint32_t* cell_count, R x) {
  const int j = (int)x;
  const uint64_t W = frac_fixed(x - (R)j);
  atomicAdd((unsigned long long*)&Qs[j], (unsigned long long)((1ull << 32) - W));
  atomicAdd((unsigned long long*)&Qs[j + 1], (unsigned long long)W);
  if (cell_count) atomicAdd(&cell_count[j], 1u);
}

// Null-collision Monte Carlo collision of a candidate at step l (Eq. (6) and
// the selection rule of Sec. IV.A).  xn is x^(l+1) and un v_x^(l+1/2) in cell
// units, both as the push left them.  Qn: the charge buffer of step l+1.  One
// Philox draw gives all of the candidate's uniforms: U0 selects the process,
// U1-U2 (and U3-U4 for ionisation) the electron directions or U1-U4 the ion's
// Maxwellian partner, U7 the waiting time to its next candidate.  An entry
// marked redraw is an examination at a cut wait: it takes only the fresh wait.
template <typename R>
__device__ __forceinline__ void mcc_candidate(const KArgs<R>& A, int s, int64_t k, bool redraw, uint32_t buf,
                                              int64_t l, R xn, R un, R uy, R uz, uint64_t id, int64_t* Qn,
                                              uint32_t* cell_count, uint32_t* cnt) {
  const CaseConst& c = A.c;
  Ctrl* C = A.ctrl;
  const int nodes = c.N + 1;
  const R vs = (R)c.v_scale, ivs = (R)c.inv_v_scale;
  R vx = un * vs, vy = uy * vs, vz = uz * vs;
  const Uniforms8<R> U = draw8<R>(id, (uint64_t)l, rng_tag(s, PU_COLL), c.seed, c.case_id);
  if (redraw) {                            // a cut wait: only a fresh wait, from U7
    A.p.next[s][buf][k] = next_candidate((double)U[7], l, c.log1m_p[s]);
    return;
  }
  const R ng = (R)c.n_gas;
  const R numax = (R)c.nu_max[s];
  bool real = false;
  if (s == 0) {
    const R g2 = vx * vx + vy * vy + vz * vz;
    const R g = dsqrt(g2);
    const R eps = (R)c.half_mr_over_e[0] * g2;
    const R S1 = ng * (R)c.sigma_el * g;
    const R S2 = S1 + ng * ln_x_over_x(eps, c.eth_exc, c.sigma0_exc) * g;
    const R S3 = S2 + ng * ln_x_over_x(eps, c.eth_ion, c.sigma0_ion) * g;
    const R r = U[0] * numax;
    if (S3 > numax) atomicAdd(&cnt[CN_OVER + 0], 1u);
    real = r < S3;
    if (r < S2) {
      // elastic or excitation: isotropic in the CM frame, gas at rest
      const bool exc = !(r < S1);
      atomicAdd(&cnt[exc ? CN_EXC : CN_EL], 1u);
      const R gp = exc ? dsqrt(fmax(g2 - (R)c.two_eexc_over_mr, (R)0)) : g;
      R nx, ny, nz;
      iso_dir<R>(U[1], U[2], nx, ny, nz);
      const R mr = (R)c.m_ratio_e, Mr = (R)c.M_ratio_e;
      vx = mr * vx + Mr * gp * nx;
      vy = mr * vy + Mr * gp * ny;
      vz = mr * vz + Mr * gp * nz;
    } else if (r < S3) {
      atomicAdd(&cnt[CN_ION], 1u);
      const R Ek = fmax((R)0.5 * (eps - (R)c.eth_ion), (R)0);
      const R sp = dsqrt(Ek) * (R)c.v_e_per_sqrt_ev;
      R nx, ny, nz;
      iso_dir<R>(U[1], U[2], nx, ny, nz);
      vx = sp * nx; vy = sp * ny; vz = sp * nz;
      R mx, my, mz;
      iso_dir<R>(U[3], U[4], mx, my, mz);
      const Uniforms8<R> Ui = draw8<R>(id, (uint64_t)l, rng_tag(0, PU_ION), c.seed, c.case_id);
      R g0, g1, g2n, g3;
      box_muller<R>(Ui[0], Ui[1], g0, g1);
      box_muller<R>(Ui[2], Ui[3], g2n, g3);
      const R sg = (R)c.sig_gas;
      const Words4 ch = philox4x64_10(id, (uint64_t)l, rng_tag(0, PU_CHILD), 0, c.seed, c.case_id);
      const uint64_t cid[2] = {ch.w0, ch.w1};
      const R cvx[2] = {sp * mx, sg * g0}, cvy[2] = {sp * my, sg * g1}, cvz[2] = {sp * mz, sg * g2n};
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const unsigned long long slot = atomicAdd((unsigned long long*)&C->n_alloc[t], 1ull);
        if ((int64_t)slot >= c.capacity[t]) { atomicOr(&C->status, ST_CAPACITY); continue; }
        const Uniforms8<double> Us = draw8<double>(cid[t], (uint64_t)l, rng_tag(t, PU_SKIP), c.seed, c.case_id);
        A.p.xt[t][buf][slot] = xn;
        A.p.ux[t][buf][slot] = cvx[t] * ivs;
        A.p.cold[t][buf][slot] = Cold<R>{cvy[t] * ivs, cvz[t] * ivs, cid[t]};
        A.p.next[t][buf][slot] = next_candidate(Us[0], l, c.log1m_p[t]);
        deposit_global<R>(Qn + t * nodes, cell_count ? cell_count + t * c.N : nullptr, xn);
        atomicAdd(&cnt[CN_BIRTH + t], 1u);
      }
    }
  } else {
    // Ar+: Maxwellian partner; resonant charge exchange hands over its velocity
    R g0, g1, g2n, g3;
    box_muller<R>(U[1], U[2], g0, g1);
    box_muller<R>(U[3], U[4], g2n, g3);
    const R sg = (R)c.sig_gas;
    const R bx = sg * g0, by = sg * g1, bz = sg * g2n;
    const R gx = vx - bx, gy = vy - by, gz = vz - bz;
    const R g = dsqrt(gx * gx + gy * gy + gz * gz);
    const R S1 = ng * (R)c.sigma_cx * g;
    if (S1 > numax) atomicAdd(&cnt[CN_OVER + 1], 1u);
    real = U[0] * numax < S1;
    if (real) {
      atomicAdd(&cnt[CN_CX], 1u);
      vx = bx; vy = by; vz = bz;
    }
  }
  A.p.next[s][buf][k] = next_candidate((double)U[7], l, c.log1m_p[s]);
  if (real) {                              // a null collision leaves the velocity as it was
    A.p.ux[s][buf][k] = vx * ivs;
    Cold<R> PM_GLOBAL& cr = A.p.cold[s][buf][k];         // uy and uz only; the id stays
    cr.uy = vy * ivs;
    cr.uz = vz * ivs;
  }
}

// Sum of a 32-bit value over the 64 lanes of a wavefront, returned as a scalar:
// an inclusive scan by DPP row shifts (1, 2, 4, 8 within rows of 16) and row
// broadcasts (lane 15 into the next row, lane 31 into the upper half), all in
// registers, then lane 63.  Every lane must be active.
__device__ __forceinline__ uint32_t dpp_wave_sum(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true);   // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true);   // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true);   // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true);   // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// Deposit the packed values (count << 48) + W of a wavefront into the LDS tile
// (key = cell, < 0 for none).  Cell-sorted particles put long runs of lanes into
// one cell (slow ions fill whole wavefronts), which would serialise 64 atomics
// on one LDS address.  Mode 0: an atomic per lane.  Mode 1: a wavefront in one
// cell is summed by DPP and one lane adds it; mixed wavefronts use per-lane
// atomics.  Must be called by all lanes.
__device__ __forceinline__ void wave_deposit(unsigned long long* sDep, int key, unsigned long long val,
                                             int mode) {
  if (mode == 0) {
    if (key >= 0) atomicAdd(&sDep[key], val);
    return;
  }
  const int lane = (int)__lane_id();
  const unsigned long long act = __ballot(key >= 0);
  if (act == 0) return;
  const int first = __ffsll((long long)act) - 1;
  const int k0 = __builtin_amdgcn_readlane(key, first);
  if (__ballot(key == k0) == act) {
    // W = hi * 2^16 + lo, and the count rides above the low sum
    // (64 * 2^16 < 2^23), so two 32-bit sums never overflow
    const uint64_t W = key >= 0 ? (val & ((1ull << 48) - 1)) : 0ull;
    const uint32_t a = dpp_wave_sum(key >= 0 ? (uint32_t)(W & 0xFFFFu) + (1u << 23) : 0u);
    const uint32_t b = dpp_wave_sum((uint32_t)(W >> 16));
    if (lane == first)
      atomicAdd(&sDep[k0], ((unsigned long long)(a >> 23) << 48) + ((unsigned long long)b << 16) +
                               (unsigned long long)(a & 0x7FFFFFu));
  } else if (key >= 0) {
    atomicAdd(&sDep[key], val);
  }
}

// Add the LDS charge tile of one species (count << 48 | sum of W per cell) to
// the global charge Qs of step l+1 -- one pair of 64-bit atomics per touched
// cell -- and the counts to the cell histogram of the next sort; clear it.
__device__ __forceinline__ void flush_tile(unsigned long long* sDep, int64_t* Qs, int N, uint32_t* cell_count) {
  for (int i = threadIdx.x; i < N; i += kBlock) {
    const uint64_t v = sDep[i];
    if (v) {
      const uint64_t cnt = v >> 48, sw = v & ((1ull << 48) - 1);
      atomicAdd((unsigned long long*)&Qs[i], (unsigned long long)((cnt << 32) - sw));
      if (sw) atomicAdd((unsigned long long*)&Qs[i + 1], (unsigned long long)sw);
      if (cell_count) atomicAdd(&cell_count[i], (uint32_t)cnt);
      sDep[i] = 0ull;
    }
  }
}

// Add the LDS flux tile (int64 sums per node) to the 128-bit sums F and clear it.
__device__ __forceinline__ void flush_flux(long long* sFlux, uint64_t* F, int nodes) {
  for (int i = threadIdx.x; i < nodes; i += kBlock) {
    const long long v = sFlux[i];
    if (v != 0) {
      atomic_add128(&F[2 * i], (int64_t)v);
      sFlux[i] = 0;
    }
  }
}

// Append the LDS candidate list to the global list of species s (uniform call).
template <typename R>
__device__ __forceinline__ void flush_candidates(Ctrl* C, uint32_t* list, XU<R>* list_xu, int s,
                                                 StepShared<R>& sh) {
  __syncthreads();
  const uint32_t n = min(sh.qn, (uint32_t)kCandCap<R>);
  if (n) {
    if (threadIdx.x == 0) sh.qbase = atomicAdd(&C->n_cand[s], n);
    __syncthreads();
    const uint32_t base = sh.qbase;
    for (uint32_t i = threadIdx.x; i < n; i += kBlock) {
      list[base + i] = sh.q[i];
      list_xu[base + i] = sh.qxu[i];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) sh.qn = 0;
  __syncthreads();
}

__device__ __forceinline__ uint64_t wall_clock() { return __builtin_amdgcn_s_memrealtime(); }

// Advance one particle by one step: gather, push, wall.  Returns its new cell
// (-1 if the slot is dead or was absorbed) and the packed deposit in *val; x
// and u become the values to store (x^(l+1) and v_x^(l+1/2), or for an absorbed
// particle its mark; a dead slot keeps its values).
template <typename R>
__device__ __forceinline__ int advance(const KArgs<R>& A, int s, int64_t k, R& x, R& u, const Pair<R>* sEp,
                                       uint32_t* cnt, uint32_t* wn, uint32_t* wall, uint32_t& live,
                                       unsigned long long* val) {
  const CaseConst& c = A.c;
  const int N = c.N;
  if (!(x >= (R)0)) {                       // dead slot (or a NaN: flagged)
    if (x != x) {
      atomicOr(&A.ctrl->status, ST_NUMERIC);
      x = (R)-1;
    }
    return -1;
  }
  ++live;
  const int j = (int)x;
  const R w = x - (R)j;
  const Pair<R> e = sEp[j];
  const R acc = e.a + w * e.b;              // electron velocity change, cells per step
  const R un = u + (s ? acc * (R)c.ion_over_e : acc);    // v^(l+1/2) = v^(l-1/2) + (q/m) E dt
  const R xn = x + un;                      // x^(l+1) = x^(l) + v^(l+1/2) dt
  u = un;
  if (!(xn >= (R)0 && xn < (R)N)) {
    x = (R)-1;                                             // either way the slot is dead
    if (xn != xn) {
      atomicOr(&A.ctrl->status, ST_NUMERIC);               // a NaN leaves the case failed
    } else {
      const int el = xn < (R)0 ? 0 : 1;
      atomicAdd(&cnt[CN_ABS + 2 * s + el], 1u);
      if (s == 1) {                                        // tallied after the loop
        x = el ? (R)kMarkSubstrate : (R)kMarkTarget;
        const uint32_t w = atomicAdd(wn, 1u);
        if (w < (uint32_t)kWallCap) wall[w] = (uint32_t)k;
      }
    }
    return -1;
  }
  x = xn;
  const int jn = (int)xn;
  *val = (1ull << 48) + frac_fixed(xn - (R)jn);
  return jn;
}

template <typename T>
using Vec4 = T __attribute__((ext_vector_type(4)));

// The push workgroup bid of nblk (the first nwork share the slots).  With
// kFlux it also samples the particle flux profiles of the step (Fig. 8): the
// state it loads is the one a step starts from (x^(l), v_x^(l-1/2)), so each
// live particle adds its linear-weighting shares of u_x to an LDS tile of
// int64 sums before it is advanced, and the tile is added to the step's
// 128-bit sums of its RF phase bin when the species' walk ends.
template <typename R, int kUnroll, bool kFlux>
__device__ __forceinline__ void step_block(const KArgs<R>& A, int bid, int nblk, int nwork, int count_cells,
                                           unsigned char* smem, StepShared<R>& sh) {
  const CaseConst& c = A.c;
  const int N = c.N, nodes = N + 1, tid = threadIdx.x;
  Pair<R>* sEp = reinterpret_cast<Pair<R>*>(smem);                               // [N]
  unsigned long long* sDep = reinterpret_cast<unsigned long long*>(sEp + N);      // [N], one species
  long long* sFlux = reinterpret_cast<long long*>(sDep + N);                      // [N + 1], with kFlux
  Ctrl* C = A.ctrl;
  const int64_t l = C->step;
  const uint32_t buf = C->buf;
  const int64_t n0 = C->n_range[0], n1 = C->n_range[1];
  // The live slots are cut into tiles of kTile (one pass of the workgroup) and
  // the first nwork workgroups take every nwork-th tile: at any moment the
  // workgroups stream neighbouring tiles, which keeps HBM busier than one long
  // chunk per workgroup.  Workgroups without tiles only take their share of the
  // charge-buffer rotation.
  // Slots are numbered electrons [0, n0), then ions from n0p = n0 rounded up to
  // a whole tile, so that no tile holds both species (a workgroup with the last
  // electron tile and the first ion tile would walk two tiles' worth of fixed
  // cost and end last); tiles are multiples of 4 slots, so every tile of either
  // species starts on a 16-byte boundary (vector loads).
  constexpr int64_t kTile = (int64_t)kBlock * kUnroll;
  const int64_t n0p = (n0 + kTile - 1) / kTile * kTile;
  const int64_t T = n0p + n1;
  const bool idle = bid >= nwork || (int64_t)bid * kTile >= T;

  uint64_t* prof = c.prof ? A.g.prof + 8 * (int64_t)bid : nullptr;
  if (prof && tid == 0) prof[0] = wall_clock();
  if (!idle) {
    const Pair<R>* Eg = reinterpret_cast<const Pair<R>*>(A.g.Epair);
    for (int i = tid; i < N; i += kBlock) sEp[i] = Eg[i];
    for (int i = tid; i < N; i += kBlock) sDep[i] = 0ull;
    if (kFlux)
      for (int i = tid; i <= N; i += kBlock) sFlux[i] = 0;
  }
  if (tid < CN_N) sh.cnt[tid] = 0;
  if (tid == 0) {
    sh.qn = 0;
    sh.wn = 0;
  }
  {
    // clear the charge buffer of step l+2 (last read by step l-1), and add the
    // charge of step l (final since the previous launch) to the averaging sums
    // (and to the sums of its RF phase bin when phase-resolved sums are kept)
    int64_t* Qc = A.g.Q + qbuf_index(l, 2) * 2 * nodes;
    const int64_t* Qa = A.g.Q + qbuf_index(l, 0) * 2 * nodes;
    const int pb = c.n_phase > 0 ? phase_bin(c, l) : -1;
    uint64_t* Sp = pb >= 0 ? A.g.sumQp + (int64_t)pb * 4 * nodes : nullptr;
    for (int64_t i = (int64_t)bid * kBlock + tid; i < 2 * nodes; i += (int64_t)nblk * kBlock) {
      Qc[i] = 0;
      add128(&A.g.sumQ[2 * i], Qa[i]);
      if (Sp) add128(&Sp[2 * i], Qa[i]);
    }
    if (bid == 0 && tid == 0) {
      C->v_sum += C->phi0;                 // the driven electrode's potential at t_l
      C->avg_steps += 1;
      if (pb >= 0) {
        A.g.phase_v[pb] += C->phi0;
        A.g.phase_n[pb] += 1;
      }
      if (kFlux) A.g.flux_n[pb >= 0 ? pb : 0] += 1;   // one flux sample of this step
    }
  }
  if (idle) return;
  __syncthreads();
  if (prof && tid == 0) prof[1] = wall_clock();

  int64_t* Qn = A.g.Q + qbuf_index(l, 1) * 2 * nodes;
  const int fbin = kFlux && c.n_phase > 0 ? phase_bin(c, l) : 0;
  const int lane = (int)__lane_id();
  uint32_t live = 0;
  // The range is walked one species at a time so that the species index (and
  // with it every array pointer) is uniform: a per-lane species would fetch
  // each pointer with a vector load and serialise the stream.  The trip count
  // is uniform over the workgroup so every lane joins the wavefront-wide
  // deposit; lanes past the range carry no particle.
  // Each lane takes kUnroll / 4 groups of 4 consecutive slots, loaded and stored
  // as 16-byte vectors; a wavefront covers 256 consecutive slots per group.
  constexpr int kVec = kUnroll / 4;
  for (int s = 0; s < 2; ++s) {
    // species s holds slots [g_lo, g_hi) of the numbering; its first tile of
    // this workgroup is the first t >= g_lo / kTile with t = bid (mod nwork)
    const int64_t g_lo = s ? n0p : 0, g_hi = s ? T : n0;
    const int64_t tf = g_lo / kTile;
    const int64_t t0 = tf + (((int64_t)bid - tf) % nwork + nwork) % nwork;
    if (g_lo >= g_hi || t0 * kTile >= g_hi) continue;
    R PM_GLOBAL* __restrict__ xs = A.p.xt[s][buf];
    R PM_GLOBAL* __restrict__ us = A.p.ux[s][buf];
    uint32_t ncand = 0;                      // real candidates listed by this wavefront
    const uint16_t PM_GLOBAL* __restrict__ ns = A.p.next[s][buf];
    const bool coll = c.log1m_p[s] != 0.0;   // the species has a schedule at all
    const uint32_t l15 = (uint32_t)l & 0x7FFFu;
    uint32_t* list = A.g.cand + (s ? c.capacity[0] : 0);
    XU<R>* list_xu = reinterpret_cast<XU<R>*>(A.g.cand_xu) + (s ? c.capacity[0] : 0);
    // slots deposited into the LDS tile since it was last flushed: a cell's
    // count must stay below 2^16 (and, with kFlux, slots in the flux tile)
    int64_t used = 0, fused = 0;
    for (int64_t t = t0; t * kTile < g_hi; t += nwork) {
      const int64_t k_hi = min((t + 1) * kTile, g_hi) - g_lo;          // species-local slot bound
      const int64_t base = max(t * kTile, g_lo) - g_lo + 4 * tid;
      R x[kUnroll], u[kUnroll];
      uint32_t nx[kUnroll];
#pragma unroll
      for (int v = 0; v < kVec; ++v) {
        const int64_t k0 = base + (int64_t)v * (4 * kBlock);
        if (k0 + 3 < k_hi) {
          // the particle stream is read and written once per step: keep it out of the L2
          const Vec4<R> xv = __builtin_nontemporal_load((const Vec4<R> PM_GLOBAL*)(xs + k0));
          const Vec4<R> uv = __builtin_nontemporal_load((const Vec4<R> PM_GLOBAL*)(us + k0));
          const Vec4<uint16_t> nv = __builtin_nontemporal_load((const Vec4<uint16_t> PM_GLOBAL*)(ns + k0));
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            x[4 * v + j] = xv[j];
            u[4 * v + j] = uv[j];
            nx[4 * v + j] = nv[j];
          }
        } else {
          // past the range a lane carries a dead slot
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const bool in = k0 + j < k_hi;
            x[4 * v + j] = in ? xs[k0 + j] : (R)-1;
            u[4 * v + j] = in ? us[k0 + j] : (R)0;
            nx[4 * v + j] = in ? ns[k0 + j] : 0u;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
        const int64_t k = base + (int64_t)(q >> 2) * (4 * kBlock) + (q & 3);
        if (kFlux && x[q] >= (R)0 && x[q] < (R)N) {          // a live slot's flux sample
          const int j = (int)x[q];
          long long a0, a1;
          flux_shares<R>(x[q], j, u[q], a0, a1);
          atomicAdd((unsigned long long*)&sFlux[j], (unsigned long long)a0);
          atomicAdd((unsigned long long*)&sFlux[j + 1], (unsigned long long)a1);
        }
        unsigned long long val = 0;
        const int key = advance<R>(A, s, k, x[q], u[q], sEp, sh.cnt, &sh.wn, sh.wall, live, &val);
        wave_deposit(sDep, key, val, c.dep_mode);
        // due for examination at this step; the list entry carries the redraw bit
        const bool cd = coll && key >= 0 && (nx[q] & 0x7FFFu) == l15;
        const uint32_t entry = (uint32_t)k | ((nx[q] & kRedraw) << 16);
        const uint64_t m = __ballot(cd);
        if (m) {
          // the wavefront's candidates take consecutive places in the LDS list
          uint32_t wbase = 0;
          if (lane == 0) wbase = atomicAdd(&sh.qn, (uint32_t)__popcll(m));
          wbase = __builtin_amdgcn_readfirstlane(wbase);
          if (cd) {
            const uint32_t pos = wbase + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            if (pos < (uint32_t)kCandCap<R>) {
              sh.q[pos] = entry;
              sh.qxu[pos] = XU<R>{x[q], u[q]};
            } else {                                                   // LDS list full
              const uint32_t g = atomicAdd(&C->n_cand[s], 1u);
              list[g] = entry;
              list_xu[g] = XU<R>{x[q], u[q]};
            }
          }
          ncand += (uint32_t)__popcll(__ballot(cd && !(nx[q] & kRedraw)));
        }
      }
#pragma unroll
      for (int v = 0; v < kVec; ++v) {
        const int64_t k0 = base + (int64_t)v * (4 * kBlock);
        if (k0 + 3 < k_hi) {
          Vec4<R> xv, uv;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            xv[j] = x[4 * v + j];
            uv[j] = u[4 * v + j];
          }
          __builtin_nontemporal_store(xv, (Vec4<R> PM_GLOBAL*)(xs + k0));
          __builtin_nontemporal_store(uv, (Vec4<R> PM_GLOBAL*)(us + k0));
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (k0 + j < k_hi) {
              xs[k0 + j] = x[4 * v + j];
              us[k0 + j] = u[4 * v + j];
            }
        }
      }
      __syncthreads();
      if (sh.qn >= (uint32_t)kCandCap<R> / 2) flush_candidates<R>(C, list, list_xu, s, sh);
      used += kTile;
      if (used + kTile > kMaxSlotsPerBlock) {
        flush_tile(sDep, Qn + s * nodes, N, count_cells ? A.g.cell_count + s * N : nullptr);
        __syncthreads();
        used = 0;
      }
      if (kFlux) {
        fused += kTile;
        if (fused >= kFluxFlushSlots) {
          flush_flux(sFlux, A.g.sumF + ((int64_t)fbin * 2 + s) * 2 * nodes, nodes);
          __syncthreads();
          fused = 0;
        }
      }
    }
    if (prof && tid == 0) prof[2] = wall_clock();
    if (lane == 0 && ncand) atomicAdd(&sh.cnt[CN_CAND + s], ncand);
    if (s == 1) tally_ion_walls<R, kTile>(A, buf, t0, nwork, g_lo, g_hi, sh);
    flush_candidates<R>(C, list, list_xu, s, sh);      // ends with a barrier
    if (prof && tid == 0) prof[3] = wall_clock();
    flush_tile(sDep, Qn + s * nodes, N, count_cells ? A.g.cell_count + s * N : nullptr);
    if (kFlux) flush_flux(sFlux, A.g.sumF + ((int64_t)fbin * 2 + s) * 2 * nodes, nodes);
    __syncthreads();
  }
  // live count: one LDS atomic per wavefront
  const uint32_t wl = dpp_wave_sum(live);
  if (lane == 0) atomicAdd(&sh.cnt[CN_LIVE], wl);
  __syncthreads();
  if (tid == 0) flush_counters(C, bank_of(A.g, bid), sh.cnt);
  if (prof && tid == 0) prof[4] = wall_clock();
}

template <typename R>
__device__ __forceinline__ void step_epilogue(const KArgs<R>& A, int64_t l, int count_cells, FieldLds& L);

// The collision workgroup bid of nblk: the candidates of both species lists,
// grid-strided, one species at a time; the last workgroup to finish runs the
// epilogue of the step.
template <typename R>
__device__ __forceinline__ void mcc_block(const KArgs<R>& A, int bid, int nblk, int count_cells, unsigned char* smem,
                                          MccShared& sh) {
  const CaseConst& c = A.c;
  const int tid = threadIdx.x;
  Ctrl* C = A.ctrl;
  const int64_t l = C->step;
  const uint32_t buf = C->buf;
  uint64_t* prof = c.prof ? A.g.prof + 8 * (int64_t)bid : nullptr;
  if (prof && tid == 0) prof[5] = wall_clock();
  if (tid < CN_N) sh.cnt[tid] = 0;
  __syncthreads();
  int64_t* Qn = A.g.Q + qbuf_index(l, 1) * 2 * (c.N + 1);
  uint32_t* cc = count_cells ? A.g.cell_count : nullptr;
  for (int s = 0; s < 2; ++s) {
    const uint32_t n = C->n_cand[s];
    const uint32_t* list = A.g.cand + (s ? c.capacity[0] : 0);
    const XU<R>* list_xu = reinterpret_cast<const XU<R>*>(A.g.cand_xu) + (s ? c.capacity[0] : 0);
    const Cold<R> PM_GLOBAL* cs = A.p.cold[s][buf];
    // kMccBatch candidates per lane at a time: every load of the batch is in
    // flight before the first collision is computed.  The list gives the slot,
    // x and v_x; the slot's record gives the rest.
    const uint32_t stride = (uint32_t)nblk * kBlock;
    for (uint32_t i0 = (uint32_t)bid * kBlock + tid; i0 < n; i0 += kMccBatch * stride) {
      int64_t k[kMccBatch];
      bool redraw[kMccBatch];
      XU<R> xu[kMccBatch];
      Cold<R> cr[kMccBatch];
#pragma unroll
      for (int j = 0; j < kMccBatch; ++j) {
        const uint32_t i = i0 + (uint32_t)j * stride;
        k[j] = -1;
        redraw[j] = false;
        if (i < n) {
          const uint32_t e = list[i];
          k[j] = (int64_t)(e & 0x7FFFFFFFu);
          redraw[j] = (e >> 31) != 0u;
          xu[j] = list_xu[i];
        }
      }
#pragma unroll
      for (int j = 0; j < kMccBatch; ++j)
        if (k[j] >= 0) cr[j] = cs[k[j]];
#pragma unroll
      for (int j = 0; j < kMccBatch; ++j)
        if (k[j] >= 0)
          mcc_candidate<R>(A, s, k[j], redraw[j], buf, l, xu[j].x, xu[j].u, cr[j].uy, cr[j].uz, cr[j].id, Qn, cc,
                           sh.cnt);
    }
  }
  __syncthreads();
  if (tid == 0) flush_counters(C, bank_of(A.g, bid), sh.cnt);
  // the epilogue reads the charge (births' deposits) and the slot allocator
  // (births); a workgroup without births has nothing it must wait for
  if (sh.cnt[CN_BIRTH] + sh.cnt[CN_BIRTH + 1]) complete_memory_ops();
  __syncthreads();
  if (prof && tid == 0) prof[6] = wall_clock();
  if (tid == 0)
    sh.last = nblk == 1 ||     // a lone workgroup is the last without the round trip
              __hip_atomic_fetch_add(&C->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (uint32_t)nblk - 1;
  __syncthreads();
  if (!sh.last) {
    if (prof && tid == 0) prof[7] = 0;
    return;
  }
  FieldLds L = carve_field(smem, c.N);
  step_epilogue<R>(A, l, count_cells, L);
  if (prof && tid == 0) prof[7] = wall_clock();
}

// The push kernel comes in four variants: 8 or 16 particles in flight per lane
// (kUnroll), and with the compiler's own register budget (kWaves = 0) or at
// most 80 VGPRs (kWaves = 6), the six waves per SIMD that its LDS tiles allow
// at 1024 cells.
template <typename R, int kUnroll, int kWaves, bool kFlux>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kWaves > 0 ? kWaves : 1)))
void k_step(uintptr_t args, int nwork, int count_cells) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ StepShared<R> sh;
  step_block<R, kUnroll, kFlux>(case_of<R>(args, 0), blockIdx.x, gridDim.x, nwork, count_cells, smem, sh);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_mcc(uintptr_t args, int count_cells) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ MccShared sh;
  mcc_block<R>(case_of<R>(args, 0), blockIdx.x, gridDim.x, count_cells, smem, sh);
}

// Many cases advanced by one launch of each kernel: work[b] = case << 16 |
// workgroup within the case; every case keeps its own workgroup counts, done
// counter and epilogue, so one case's field solve overlaps the other cases'
// collisions.
template <typename R, int kUnroll, int kWaves>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kWaves > 0 ? kWaves : 1)))
void k_step_batch(uintptr_t cases, const uint32_t* __restrict__ work, const uint32_t* __restrict__ nblocks,
                  int count_cells) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ StepShared<R> sh;
  const uint32_t w = work[blockIdx.x];
  if (w == kIdleWork) return;
  const uint32_t nb = nblocks[w >> 16];     // workgroups | working workgroups << 16
  step_block<R, kUnroll, false>(case_of<R>(cases, w >> 16), (int)(w & 0xFFFFu), (int)(nb & 0xFFFFu),
                                (int)(nb >> 16), count_cells, smem, sh);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_mcc_batch(uintptr_t cases, const uint32_t* __restrict__ work,
                                                      const uint32_t* __restrict__ nblocks, int count_cells) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ MccShared sh;
  const uint32_t w = work[blockIdx.x];
  if (w == kIdleWork) return;
  mcc_block<R>(case_of<R>(cases, w >> 16), (int)(w & 0xFFFFu), (int)nblocks[w >> 16], count_cells, smem, sh);
}

// Accumulate the diagnostics of step l, solve the field of step l+1, scan the
// cell counts when a sort follows, and publish step l+1.
template <typename R>
__device__ __forceinline__ void step_epilogue(const KArgs<R>& A, int64_t l, int count_cells, FieldLds& L) {
  const CaseConst& c = A.c;
  Ctrl* C = A.ctrl;
  const int tid = threadIdx.x;
  field_for_step<R>(A, l + 1, true, nullptr, L);
  if (count_cells) scan_cells(c, A.g, C, L.wq);
  if (tid == 0) {
    C->step = l + 1;
    for (int s = 0; s < 2; ++s) {
      // births past the capacity were dropped (and flagged): never scan past the arrays
      const int64_t na = __hip_atomic_load(&C->n_alloc[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      C->n_range[s] = na < c.capacity[s] ? na : c.capacity[s];
      C->n_alloc[s] = C->n_range[s];
      C->n_cand[s] = 0;
    }
    C->done = 0;
  }
}

// ------------------------------------------------------------------ diagnostics
__device__ __forceinline__ double as_double128(const uint64_t* a) {
  return (double)(int64_t)a[1] * 18446744073709551616.0 + (double)a[0];
}

// Averages over the window (bin < 0) or over the steps of one RF phase bin:
// densities from the charge sums, Phi of the averaged charge and drive
// (Poisson's equation is linear, so this equals the average of Phi), and the
// particle flux profiles Gamma_s = w sum(S_m(x) v_x) / (vol_m n_samples) with
// the mean velocities Gamma_s / n_s (0 where a node holds no particles).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_diag_finalize(KArgs<R> A, int bin) {
  __shared__ double q[kMaxCells + 1];
  __shared__ double E[kMaxCells + 1];
  __shared__ double D[kMaxCells + 1];
  __shared__ double wq[8];
  __shared__ double wd[8];
  const CaseConst& c = A.c;
  Ctrl* C = A.ctrl;
  const int N = c.N, nodes = N + 1;
  const uint64_t* SQ = bin < 0 ? A.g.sumQ : A.g.sumQp + (int64_t)bin * 4 * nodes;
  const int64_t ns = bin < 0 ? C->avg_steps : A.g.phase_n[bin];
  const double vs = bin < 0 ? C->v_sum : A.g.phase_v[bin];
  const double n = ns > 0 ? (double)ns : 1.0;
  double* ne = A.g.diag_out;
  double* ni = ne + nodes;
  double* phi = ni + nodes;
  double* gam = phi + nodes;                // [2][nodes]
  double* umean = gam + 2 * nodes;          // [2][nodes]
  const bool self = !(c.flags & 1u);
  const int nf = c.n_phase > 0 ? c.n_phase : 1;
  const int f0 = bin < 0 ? 0 : bin, f1 = bin < 0 ? nf : bin + 1;
  int64_t fn = 0;
  if (c.flux)
    for (int b = f0; b < f1; ++b) fn += A.g.flux_n[b];
  for (int m = threadIdx.x; m < nodes; m += kBlock) {
    double qs[2];
    for (int s = 0; s < 2; ++s) qs[s] = as_double128(&SQ[2 * (s * nodes + m)]);
    const double vol = (m == 0 || m == N) ? 0.5 * c.dx : c.dx;
    const double k = c.w / (4294967296.0 * vol * n);
    ne[m] = qs[0] * k;
    ni[m] = qs[1] * k;
    q[m] = self ? (qs[1] - qs[0]) / n : 0.0;
    for (int s = 0; s < 2; ++s) {
      double f = 0.0;
      if (c.flux)
        for (int b = f0; b < f1; ++b) f += as_double128(&A.g.sumF[((int64_t)b * 2 + s) * 2 * nodes + 2 * m]);
      const double g = fn > 0 ? f * c.v_scale * c.w / (1099511627776.0 * vol * (double)fn) : 0.0;
      const double dens = s ? ni[m] : ne[m];
      gam[s * nodes + m] = g;
      umean[s * nodes + m] = dens > 0.0 ? g / dens : 0.0;
    }
  }
  __syncthreads();
  solve_field<double>(c, [&](int m) { return q[m]; }, vs / n, E, wq, wd, D, phi);
}

__global__ void k_diag_reset(CaseConst c, GridPtrs g, Ctrl* C) {
  const int nodes = c.N + 1;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 4 * nodes) g.sumQ[i] = 0;
  if (i < (int64_t)c.n_phase * 4 * nodes) g.sumQp[i] = 0;
  if (i < c.n_phase) {
    g.phase_v[i] = 0.0;
    g.phase_n[i] = 0;
  }
  const int nf = c.n_phase > 0 ? c.n_phase : 1;
  if (c.flux && i < (int64_t)nf * 4 * nodes) g.sumF[i] = 0;
  if (c.flux && i < nf) g.flux_n[i] = 0;
  if (i < 2 * c.n_ebins) {
    g.iedf[i] = 0;
    g.iedf_taken[i] = 0;
  }
  if (i < 2 * ((c.n_ebins + kIeadEGroup - 1) / kIeadEGroup) * kIeadABins) g.iead[i] = 0;
  if (i < 2 * kAngleBins) g.iadf[i] = 0;
  if (i < kBanks) {
    CtrBank* B = bank_of(g, (int)i);
    const int64_t nl0 = B->n_live[0], nl1 = B->n_live[1];
    *B = CtrBank{};
    B->n_live[0] = nl0;
    B->n_live[1] = nl1;
  }
  if (i == 0) {
    C->avg_steps = 0;
    C->v_sum = 0.0;
    for (int s = 0; s < 2; ++s) {
      C->absorbed[s][0] = C->absorbed[s][1] = 0;
      C->candidates[s] = C->overflow[s] = 0;
      C->ion_e_fx[s] = 0;
    }
    for (int k = 0; k < 5; ++k) C->collisions[k] = 0;
    C->births = 0;
    C->particle_steps = 0;
  }
}

// ------------------------------------------------------------------ launchers
size_t field_lds_bytes(int N) { return (size_t)(2 * (N + 1) + 16) * 8; }

template <typename R>
size_t step_lds_bytes(int N) {
  return (size_t)N * sizeof(Pair<R>) + (size_t)N * sizeof(unsigned long long);
}

template <typename R>
hipError_t launch_load(const KArgs<R>& A, int64_t np_e, int64_t np_i, double sig_e, double sig_i, hipStream_t st) {
  const int64_t n = np_e > np_i ? np_e : np_i;
  dim3 grid((unsigned)((n + kBlock - 1) / kBlock), 2);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_load<R>, grid, dim3(kBlock), 0, st, A, np_e, np_i, sig_e, sig_i);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_deposit_all(const KArgs<R>& A, int64_t nmax, hipStream_t st) {
  unsigned gx = (unsigned)((nmax + kBlock - 1) / kBlock);
  if (gx < 1) gx = 1;
  if (gx > 4096) gx = 4096;
  hipLaunchKernelGGL(k_deposit_all<R>, dim3(gx, 2), dim3(kBlock), 0, st, A);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_sort(const KArgs<R>& A, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_sort_scatter<R>, dim3(grid), dim3(kBlock), (size_t)4 * 2 * A.c.N * 2, st, A);
  return hipGetLastError();
}

hipError_t launch_scan_cells(const CaseConst& c, const GridPtrs& g, Ctrl* C, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_cells, dim3(1), dim3(kBlock), 0, st, c, g, C);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_field(const KArgs<R>& A, int want_phi, hipStream_t st) {
  hipLaunchKernelGGL(k_field<R>, dim3(1), dim3(kBlock), field_lds_bytes(A.c.N), st, A, want_phi);
  return hipGetLastError();
}

template <int V>
using IC = std::integral_constant<int, V>;

// Call f(IC<unroll>, IC<waves>) for the kernel variant of a launch shape.
template <typename F>
hipError_t by_variant(int unroll, int waves, F&& f) {
  if (unroll == 16) return waves == 6 ? f(IC<16>{}, IC<6>{}) : f(IC<16>{}, IC<0>{});
  return waves == 6 ? f(IC<8>{}, IC<6>{}) : f(IC<8>{}, IC<0>{});
}

// Workgroups of the step kernel (plain or batched) that fit on one CU at once.
template <typename R>
int step_blocks_per_cu(int N, int unroll, int waves, bool batch) {
  int nb = 0;
  const hipError_t e = by_variant(unroll, waves, [&](auto u, auto w) {
    return batch ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step_batch<R, u.value, w.value>, kBlock,
                                                                step_lds_bytes<R>(N))
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step<R, u.value, w.value, false>, kBlock,
                                                                step_lds_bytes<R>(N));
  });
  if (e != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

template <typename R>
hipError_t launch_step(const KArgs<R>& A, const KArgs<R>* dev_args, int grid, int nwork, int count_cells,
                       hipStream_t st) {
  const uintptr_t d = (uintptr_t)dev_args;
  return by_variant(A.c.unroll, A.c.waves, [&](auto u, auto w) {
    if (A.c.flux)
      hipLaunchKernelGGL((k_step<R, u.value, w.value, true>), dim3(grid), dim3(kBlock),
                         step_lds_bytes<R>(A.c.N) + (size_t)(A.c.N + 1) * 8, st, d, nwork, count_cells);
    else
      hipLaunchKernelGGL((k_step<R, u.value, w.value, false>), dim3(grid), dim3(kBlock), step_lds_bytes<R>(A.c.N),
                         st, d, nwork, count_cells);
    return hipGetLastError();
  });
}

// Workgroups of the collision kernel (plain or batched) that fit on one CU.
template <typename R>
int mcc_blocks_per_cu(int N, bool batch) {
  int nb = 0;
  const hipError_t e = batch
      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_mcc_batch<R>, kBlock, field_lds_bytes(N))
      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_mcc<R>, kBlock, field_lds_bytes(N));
  if (e != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

template <typename R>
hipError_t launch_mcc(const KArgs<R>& A, const KArgs<R>* dev_args, int grid, int count_cells, hipStream_t st) {
  hipLaunchKernelGGL(k_mcc<R>, dim3(grid), dim3(kBlock), field_lds_bytes(A.c.N), st, (uintptr_t)dev_args,
                     count_cells);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_mcc_batch(const KArgs<R>* cases, const uint32_t* work, const uint32_t* nblocks, int grid,
                            int maxN, int count_cells, hipStream_t st) {
  hipLaunchKernelGGL(k_mcc_batch<R>, dim3(grid), dim3(kBlock), field_lds_bytes(maxN), st, (uintptr_t)cases, work,
                     nblocks, count_cells);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_step_batch(const KArgs<R>* cases, const uint32_t* work, const uint32_t* nblocks, int grid,
                             int maxN, int unroll, int waves, int count_cells, hipStream_t st) {
  const size_t lds = step_lds_bytes<R>(maxN);
  return by_variant(unroll, waves, [&](auto u, auto w) {
    hipLaunchKernelGGL((k_step_batch<R, u.value, w.value>), dim3(grid), dim3(kBlock), lds, st, (uintptr_t)cases,
                       work, nblocks, count_cells);
    return hipGetLastError();
  });
}

template <typename R>
hipError_t launch_sort_batch(const KArgs<R>* cases, const uint32_t* work, const uint32_t* nblocks, int grid,
                             int maxN, hipStream_t st) {
  hipLaunchKernelGGL(k_sort_batch<R>, dim3(grid), dim3(kBlock), (size_t)16 * maxN, st, (uintptr_t)cases, work, nblocks);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_diag_finalize(const KArgs<R>& A, int bin, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_finalize<R>, dim3(1), dim3(kBlock), 0, st, A, bin);
  return hipGetLastError();
}

hipError_t launch_diag_reset(const CaseConst& c, const GridPtrs& g, Ctrl* C, hipStream_t st) {
  int n = 4 * (c.N + 1) * (c.n_phase > 1 ? c.n_phase : 1);
  const int n_iead = 2 * ((c.n_ebins + kIeadEGroup - 1) / kIeadEGroup) * kIeadABins;
  if (n_iead > n) n = n_iead;
  if (2 * c.n_ebins > n) n = 2 * c.n_ebins;
  if (2 * kAngleBins > n) n = 2 * kAngleBins;
  hipLaunchKernelGGL(k_diag_reset, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, c, g, C);
  return hipGetLastError();
}

#define PM_INSTANTIATE(R)                                                                                    \
  template hipError_t launch_load<R>(const KArgs<R>&, int64_t, int64_t, double, double, hipStream_t);      \
  template hipError_t launch_deposit_all<R>(const KArgs<R>&, int64_t, hipStream_t);                         \
  template hipError_t launch_sort<R>(const KArgs<R>&, int, hipStream_t);                                    \
  template hipError_t launch_field<R>(const KArgs<R>&, int, hipStream_t);                                   \
  template hipError_t launch_step<R>(const KArgs<R>&, const KArgs<R>*, int, int, int, hipStream_t);                               \
  template int step_blocks_per_cu<R>(int, int, int, bool);                                                       \
  template int mcc_blocks_per_cu<R>(int, bool);                                                                  \
  template hipError_t launch_mcc<R>(const KArgs<R>&, const KArgs<R>*, int, int, hipStream_t);                   \
  template hipError_t launch_mcc_batch<R>(const KArgs<R>*, const uint32_t*, const uint32_t*, int, int, int,    \
                                          hipStream_t);                                                        \
  template hipError_t launch_diag_finalize<R>(const KArgs<R>&, int, hipStream_t);                          \
  template hipError_t launch_step_batch<R>(const KArgs<R>*, const uint32_t*, const uint32_t*, int, int, int,  \
                                           int, int, hipStream_t);                                            \
  template hipError_t launch_sort_batch<R>(const KArgs<R>*, const uint32_t*, const uint32_t*, int, int,      \
                                           hipStream_t);
PM_INSTANTIATE(float)
PM_INSTANTIATE(double)

}  // namespace pm
