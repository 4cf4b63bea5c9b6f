// Test-particle kernels for gfx950 (Sec. IV.B of arXiv:1607.04069).
//
// k_yield applies the yield rule of 'Wall Interactions' to the recorded Ar+
// impacts on the target: N = ceil(Y) checks R_f <= Y/N per impact.
//
// k_tp_flight flies sputtered Al atoms: Thompson energy and cosine angle at
// emission, straight flights with free-flight times tau = -ln(R_f) / nu_max
// (Eq. (5) with the null-collision majorant of Eq. (6)), a Maxwellian argon
// partner at each candidate, acceptance sigma(g) g / (sigma g)_max with the VHS
// cross section of Eq. (8) (or M1 scattering: deflection pi (1 - b/b_max) about
// the relative velocity, 'Binary Interactions'), isotropic centre-of-mass scattering (Eq. (10) with
// chi = 2 arccos(b/b_max)), and sticking electrodes.  One lane flies one atom
// at a time in registers; a lane whose atom ends takes the next atom of its
// stride at once, so a wavefront keeps all 64 lanes busy while atoms with very
// different event counts finish.  Tallies go to LDS and are flushed once per
// workgroup.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "philox.h"
#include "pm_internal.h"
#include "pm_launch.h"

namespace pm {

// With taken (live injection) only the impacts i >= taken[b] that arrived since
// the previous such call are used, and taken[b] then moves to the record's
// count: impact i of bin b keys its draws by (i, b), so the calls of a window
// add up to exactly what one call over the whole record draws.
__global__ __launch_bounds__(kBlock) void k_yield(const uint64_t* iedf, const double* ybin, int n_ebins,
                                                  uint64_t seed, uint64_t job, uint64_t aux_hi, uint64_t* taken,
                                                  uint64_t* out) {
  __shared__ uint32_t s_cnt;
  const int b = blockIdx.x;
  if (threadIdx.x == 0) s_cnt = 0;
  const uint64_t c = iedf[b];
  const uint64_t t0 = taken ? taken[b] : 0;
  __syncthreads();
  const double Y = ybin[b];
  const int N = (int)ceil(Y);
  uint32_t k = 0;
  if (N > 0) {
    const double p = Y / (double)N;
    for (uint64_t i = t0 + threadIdx.x; i < c; i += kBlock)
      for (int n = 0; n < N; ++n) {
        const Words4 w = philox4x64_10(i, (uint64_t)b, rng_tag(SP_YIELD, PU_YIELD), aux_hi | (uint64_t)n, seed, job);
        if (u_hi<double>(w.w0) <= p) ++k;
      }
  }
  atomicAdd(&s_cnt, k);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_cnt) atomicAdd((unsigned long long*)&out[0], (unsigned long long)s_cnt);
    if (c > t0) atomicAdd((unsigned long long*)&out[1], (unsigned long long)(c - t0));
    if (taken && c > t0) taken[b] = c;
  }
}

hipError_t launch_yield(const uint64_t* iedf, const double* ybin, int n_ebins, uint64_t seed,
                        uint64_t job, int electrode, uint64_t* taken, uint64_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_yield, dim3(n_ebins), dim3(kBlock), 0, st, iedf, ybin, n_ebins, seed, job,
                     (uint64_t)electrode << 32, taken, out);
  return hipGetLastError();
}

struct Atom {
  float x, y, z, vx, vy, vz, t;
  uint32_t e;
};

// A new atom from its emission draw (counter (id, 0, source tag)).
__device__ __forceinline__ void emit(const TpConst& T, const Uniforms8<float>& U, Atom& a) {
  const float smax = (float)T.s_max;
  // the hardware's approximate sqrt and sin/cos (angle in revolutions), as in
  // the event loop
  const float s = __builtin_amdgcn_sqrtf(U[0]) * smax;
  const float E = (float)T.u_s * s / (1.0f - s);       // Thompson flux law by inversion
  const float ct = __builtin_amdgcn_sqrtf(U[1]);         // theta = arccos(sqrt(R_f))
  const float st = __builtin_amdgcn_sqrtf(1.0f - U[1]);
  const float sp = __builtin_amdgcn_sinf(U[2]), cp = __builtin_amdgcn_cosf(U[2]);
  const float v = __builtin_amdgcn_sqrtf(E) * (float)T.v_per_sqrt_ev;
  // from the target into +x, or from the substrate (re-sputtering) into -x
  a.vx = T.electrode ? -(v * ct) : v * ct;
  a.vy = v * st * cp;
  a.vz = v * st * sp;
  a.x = T.electrode ? (float)T.L : 0.0f;
  a.y = (float)T.lat * U[3];
  a.z = (float)T.lat * U[4];
  a.t = 0.0f;
  a.e = 0;
}

__device__ __forceinline__ float wrapf(float v, float L, float inv_L) { return v - L * floorf(v * inv_L); }

// The event loop's variates use the hardware's approximate log2, exp2, sqrt,
// reciprocal and sine/cosine (about 1 ulp; the sine and cosine take the angle
// in revolutions): a random direction or waiting time needs no correctly
// rounded result, and these are most of the loop's arithmetic.
__device__ __forceinline__ float fast_ln(float u) { return __builtin_amdgcn_logf(u) * 0.6931471805599453f; }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// sin and cos of 2 pi r
__device__ __forceinline__ void fast_sincos_rev(float r, float* s, float* c) {
  *s = __builtin_amdgcn_sinf(r);
  *c = __builtin_amdgcn_cosf(r);
}

// Track-length profile units: time in 2^-40 s, displacement in 2^-24 cells.
constexpr float kTimeFx = 1099511627776.0f;
constexpr float kCellFx = 16777216.0f;

// rint(x) as an int64: the hardware's f32 -> i32 conversion when |x| < 2^31
// (almost always), the general (longer) conversion otherwise; the two agree.
__device__ __forceinline__ long long rint_i64(float x) {
  const float r = rintf(x);
  if (__builtin_expect(fabsf(r) < 2147483520.0f, 1)) return (long long)(int)r;
  return (long long)r;
}

// Add a straight flight xa -> xb at x-velocity vx to the LDS profile tallies:
// partial cells directly (time overlap / |vx|, displacement overlap * sign), the
// cells crossed end to end as a difference (+ at the first, - past the last) of
// their common time dx / |vx| and displacement dx * sign, summed up at the end.
__device__ __forceinline__ void track_tally(const TpConst& T, unsigned long long* pt, unsigned long long* dt,
                                            unsigned long long* px, unsigned long long* dd, float xa, float xb,
                                            float vx) {
  if (vx == 0.0f) return;
  const float lo = fminf(xa, xb), hi = fmaxf(xa, xb);
  const float inv_v = __builtin_amdgcn_rcpf(fabsf(vx));
  const float ih = (float)T.inv_xbin, h = (float)T.xbin;
  const int n = T.n_xbins;
  const int ia = min(max((int)(lo * ih), 0), n - 1), ib = min(max((int)(hi * ih), 0), n - 1);
  const long long sgn = vx > 0.0f ? 1 : -1;
  // displacements are at most one cell, 2^24 units: always an int32
  if (ia == ib) {
    atomicAdd(&pt[ia], (unsigned long long)rint_i64((hi - lo) * inv_v * kTimeFx));
    atomicAdd(&px[ia], (unsigned long long)(sgn * (long long)(int)rintf((hi - lo) * ih * kCellFx)));
    return;
  }
  const float fa = (float)(ia + 1) - lo * ih;          // cells of the partial ends
  const float fb = hi * ih - (float)ib;
  atomicAdd(&pt[ia], (unsigned long long)rint_i64(fa * h * inv_v * kTimeFx));
  atomicAdd(&pt[ib], (unsigned long long)rint_i64(fb * h * inv_v * kTimeFx));
  atomicAdd(&px[ia], (unsigned long long)(sgn * (long long)(int)rintf(fa * kCellFx)));
  atomicAdd(&px[ib], (unsigned long long)(sgn * (long long)(int)rintf(fb * kCellFx)));
  if (ib > ia + 1) {
    const long long full = rint_i64(h * inv_v * kTimeFx);
    atomicAdd(&dt[ia + 1], (unsigned long long)full);
    atomicAdd(&dt[ib], (unsigned long long)(-full));
    atomicAdd(&dd[ia + 1], (unsigned long long)(sgn * (long long)kCellFx));
    atomicAdd(&dd[ib], (unsigned long long)(-sgn * (long long)kCellFx));
  }
}

struct TpShared {
  uint32_t n_sub, n_tgt, n_unf, over;
  unsigned long long events, coll;
  long long e_sub, e_tgt;
};

__global__ __launch_bounds__(kBlock) void k_tp_flight(TpConst T, TpTally* tal, uint64_t* e_hist,
                                                      uint64_t* th_hist, uint64_t* tof_hist, TpTrace tr,
                                                      int64_t* prof) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nx1 = T.n_xbins + 1;
  unsigned long long* sP = reinterpret_cast<unsigned long long*>(smem);   // [4][n_xbins + 1]
  uint32_t* sE = reinterpret_cast<uint32_t*>(sP + (T.n_xbins ? 4 * nx1 : 0));
  uint32_t* sTh = sE + T.n_ebins;
  uint32_t* sTof = sTh + kTpThetaBins;
  __shared__ TpShared sh;
  const int tid = threadIdx.x;
  for (int i = tid; i < T.n_ebins + kTpThetaBins + T.n_tbins; i += kBlock) sE[i] = 0;
  if (T.n_xbins)
    for (int i = tid; i < 4 * nx1; i += kBlock) sP[i] = 0ull;
  if (tid == 0) {
    sh.n_sub = sh.n_tgt = sh.n_unf = sh.over = 0;
    sh.events = sh.coll = 0;
    sh.e_sub = sh.e_tgt = 0;
  }
  __syncthreads();

  const float L = (float)T.L, lat = (float)T.lat;
  const float inv_L = (float)(1.0 / T.L), inv_lat = (float)(1.0 / T.lat);
  const float inv_nu = (float)T.inv_nu_max;
  const float sg = (float)T.sig_gas;
  const float mr = (float)T.m_ratio, Mr = (float)T.M_ratio;
  const float sgexp = (float)T.sg_exp, l2cap = (float)T.log2_gcap;
  const bool fixed = T.dt > 0.0;
  const float dt_fixed = (float)T.dt, nu_dt = (float)T.nu_dt;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  int64_t k = (int64_t)blockIdx.x * kBlock + tid;
  uint64_t n_ev = 0, n_coll = 0;
  uint32_t n_over = 0;
  Atom a;
  // Each pass makes one generator call per lane: the emission draw of a lane's
  // next atom or the event draw of its current one, so that a wavefront whose
  // lanes are partly starting new atoms does not issue the generator twice.
  bool fresh = true;
  while (k < T.n_atoms) {
    const uint64_t id = (uint64_t)(T.first_atom + k);
    const Uniforms8<float> U = draw8<float>(id, fresh ? 0ull : (uint64_t)a.e,
                                            fresh ? rng_tag(SP_AL, PU_TP_SRC) : rng_tag(SP_AL, PU_TP_EVT), T.seed,
                                            T.job);
    if (fresh) {
      emit(T, U, a);
      fresh = false;
      continue;
    }
    const float tau = fixed ? dt_fixed : -fast_ln(U[0]) * inv_nu;
    const float xn = a.x + a.vx * tau;
    int wall = -1;
    float tof = 0.0f;
    if (T.mode == 0 && !(xn >= 0.0f && xn < L)) {
      wall = xn >= L ? 1 : 0;
      tof = a.t + (wall ? (L - a.x) : -a.x) / a.vx;
      if (T.n_xbins) track_tally(T, sP, sP + nx1, sP + 2 * nx1, sP + 3 * nx1, a.x, wall ? L : 0.0f, a.vx);
    } else {
      if (T.n_xbins && T.mode == 0) track_tally(T, sP, sP + nx1, sP + 2 * nx1, sP + 3 * nx1, a.x, xn, a.vx);
      a.x = T.mode == 0 ? xn : wrapf(xn, L, inv_L);
      a.y = wrapf(a.y + a.vy * tau, lat, inv_lat);
      a.z = wrapf(a.z + a.vz * tau, lat, inv_lat);
      // a fixed step's clock is its step count (no FP32 accumulation over many steps)
      a.t = fixed ? (float)((double)(a.e + 1) * T.dt) : a.t + tau;
      // candidate: Maxwellian argon partner, accept with (sigma g)/(sigma g)_max = (g/g_cap)^(2 - 2 omega)
      const float r0 = fast_sqrt(-2.0f * fast_ln(U[1]));
      const float r1 = fast_sqrt(-2.0f * fast_ln(U[3]));
      float s0, c0, s1, c1;
      fast_sincos_rev(U[2], &s0, &c0);
      fast_sincos_rev(U[4], &s1, &c1);
      const float bx = sg * r0 * c0, by = sg * r0 * s0, bz = sg * r1 * c1;
      const float gx = a.vx - bx, gy = a.vy - by, gz = a.vz - bz;
      const float gm = fast_sqrt(gx * gx + gy * gy + gz * gz);
      // (sigma g) / (sigma g)_max; with a fixed step the probability n sigma g dt of Eq. (7)
      const float ratio =
          __builtin_amdgcn_exp2f(sgexp * (__builtin_amdgcn_logf(gm) - l2cap)) * (fixed ? nu_dt : 1.0f);
      n_over += ratio > 1.0f;
      if (U[5] < ratio) {
        ++n_coll;
        float sp, cp;
        fast_sincos_rev(U[7], &sp, &cp);
        if (T.scatter == 0) {
          // VHS: isotropic new relative direction
          const float cc = 2.0f * U[6] - 1.0f;
          const float sc = fast_sqrt(fmaxf(0.0f, 1.0f - cc * cc));
          a.vx = mr * a.vx + Mr * bx + Mr * gm * cc;
          a.vy = mr * a.vy + Mr * by + Mr * gm * sc * cp;
          a.vz = mr * a.vz + Mr * bz + Mr * gm * sc * sp;
        } else {
          // M1: g turned by chi = pi (1 - sqrt(U6)) at azimuth psi about itself, in
          // the basis e1 = (x-hat x g)/|.|, e2 = g-hat x e1 (e1 = y-hat along x)
          float sc, cc;
          fast_sincos_rev(0.5f * (1.0f - fast_sqrt(U[6])), &sc, &cc);     // chi = pi (1 - sqrt(U6))
          const float gp = fast_sqrt(gy * gy + gz * gz);
          float hx, hy, hz;
          if (gp > 1e-6f * gm) {
            const float ip = __builtin_amdgcn_rcpf(gp);
            hx = cc * gx + sc * sp * gp;
            hy = cc * gy - sc * (cp * gm * gz + sp * gx * gy) * ip;
            hz = cc * gz + sc * (cp * gm * gy - sp * gx * gz) * ip;
          } else {
            hx = cc * gx;
            hy = gm * sc * cp;
            hz = gm * sc * sp * (gx < 0.0f ? -1.0f : 1.0f);
          }
          a.vx = mr * a.vx + Mr * bx + Mr * hx;
          a.vy = mr * a.vy + Mr * by + Mr * hy;
          a.vz = mr * a.vz + Mr * bz + Mr * hz;
        }
      }
      ++a.e;
      ++n_ev;
      if ((int64_t)a.e >= T.e_max) {
        wall = 2;
        tof = a.t;
      }
    }
    if (wall >= 0) {
      const float v2 = a.vx * a.vx + a.vy * a.vy + a.vz * a.vz;
      const float E = (float)T.e_half_m * v2;
      const float th = acosf(fminf(fabsf(a.vx) / sqrtf(v2), 1.0f)) * 57.29577951308232f;
      const long long efx = rint_i64(E * 1048576.0f);             // E 2^20 is exact in FP32
      if (wall == 1) {
        atomicAdd(&sh.n_sub, 1u);
        atomicAdd(&sE[(int)fminf(fmaxf(E / (float)T.ebin, 0.0f), (float)(T.n_ebins - 1))], 1u);
        atomicAdd(&sTh[(int)fminf(fmaxf(th, 0.0f), (float)(kTpThetaBins - 1))], 1u);
        atomicAdd(&sTof[(int)fminf(fmaxf(tof / (float)T.tbin, 0.0f), (float)(T.n_tbins - 1))], 1u);
        atomicAdd((unsigned long long*)&sh.e_sub, (unsigned long long)efx);
      } else if (wall == 0) {
        atomicAdd(&sh.n_tgt, 1u);
        atomicAdd((unsigned long long*)&sh.e_tgt, (unsigned long long)efx);
      } else {
        atomicAdd(&sh.n_unf, 1u);
      }
      if (tr.wall) tr.wall[k] = wall;
      if (tr.events) tr.events[k] = a.e;
      if (tr.energy_ev) tr.energy_ev[k] = E;
      if (tr.theta_deg) tr.theta_deg[k] = th;
      if (tr.tof_s) tr.tof_s[k] = tof;
      if (tr.vx) tr.vx[k] = a.vx;
      if (tr.vy) tr.vy[k] = a.vy;
      if (tr.vz) tr.vz[k] = a.vz;
      k += stride;
      fresh = true;
    }
  }
  atomicAdd(&sh.events, (unsigned long long)n_ev);
  atomicAdd(&sh.coll, (unsigned long long)n_coll);
  atomicAdd(&sh.over, n_over);
  __syncthreads();
  for (int i = tid; i < T.n_ebins; i += kBlock)
    if (sE[i]) atomicAdd((unsigned long long*)&e_hist[i], (unsigned long long)sE[i]);
  for (int i = tid; i < kTpThetaBins; i += kBlock)
    if (sTh[i]) atomicAdd((unsigned long long*)&th_hist[i], (unsigned long long)sTh[i]);
  for (int i = tid; i < T.n_tbins; i += kBlock)
    if (sTof[i]) atomicAdd((unsigned long long*)&tof_hist[i], (unsigned long long)sTof[i]);
  if (T.n_xbins && prof)
    for (int i = tid; i < 4 * nx1; i += kBlock)
      if (sP[i]) atomicAdd((unsigned long long*)&prof[i], sP[i]);
  if (tid == 0) {
    atomicAdd((unsigned long long*)&tal->n_sub, (unsigned long long)sh.n_sub);
    atomicAdd((unsigned long long*)&tal->n_tgt, (unsigned long long)sh.n_tgt);
    atomicAdd((unsigned long long*)&tal->n_unf, (unsigned long long)sh.n_unf);
    atomicAdd((unsigned long long*)&tal->events, sh.events);
    atomicAdd((unsigned long long*)&tal->collisions, sh.coll);
    atomicAdd((unsigned long long*)&tal->overflow, (unsigned long long)sh.over);
    atomicAdd((unsigned long long*)&tal->e_sub_fx, (unsigned long long)sh.e_sub);
    atomicAdd((unsigned long long*)&tal->e_tgt_fx, (unsigned long long)sh.e_tgt);
  }
}

// Density and mean x-velocity profiles of the test atoms from the track-length
// tallies (Sec. IV.B, last paragraph: time-weighted densities without a grid):
// cell i holds the partial-cell sums plus the running sum of the full-cell
// differences, time in 2^-40 s and displacement in 2^-24 cells.  With S the
// source flux (m^-2 s^-1) carried by n_atoms atoms, an atom spending t in a
// cell of width h adds S / n_atoms * t / h to its density; the mean x-velocity
// is the displacement over the time (0 in a cell no atom entered).  One
// workgroup; out = [4][nx] doubles: time (s), displacement (m), density
// (m^-3), mean v_x (m/s).
__global__ __launch_bounds__(kBlock) void k_tp_profiles(const int64_t* prof, int nx, double h, double per_atom,
                                                        double* out) {
  __shared__ int64_t s_w[2][kBlock / 64];
  const int nx1 = nx + 1, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int per = (nx + kBlock - 1) / kBlock;
  const int b = tid * per, e = min(b + per, nx);
  int64_t lt = 0, lx = 0;
  for (int i = b; i < e; ++i) {
    lt += prof[nx1 + i];
    lx += prof[3 * nx1 + i];
  }
  // exclusive block scans of the two difference arrays (integer: exact in any order)
  int64_t st = lt, sx = lx;
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t a = __shfl_up(st, off, 64), c = __shfl_up(sx, off, 64);
    if (lane >= off) {
      st += a;
      sx += c;
    }
  }
  if (lane == 63) {
    s_w[0][w] = st;
    s_w[1][w] = sx;
  }
  __syncthreads();
  int64_t rt = st - lt, rx = sx - lx;
  for (int k = 0; k < w; ++k) {
    rt += s_w[0][k];
    rx += s_w[1][k];
  }
  for (int i = b; i < e; ++i) {
    rt += prof[nx1 + i];
    rx += prof[3 * nx1 + i];
    const double t = (double)(prof[i] + rt) / 1099511627776.0;
    const double x = (double)(prof[2 * nx1 + i] + rx) / 16777216.0 * h;
    out[i] = t;
    out[nx + i] = x;
    out[2 * nx + i] = per_atom * t / h;
    out[3 * nx + i] = t > 0.0 ? x / t : 0.0;
  }
}

hipError_t launch_tp_profiles(const int64_t* prof, int nx, double h, double per_atom, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_tp_profiles, dim3(1), dim3(kBlock), 0, st, prof, nx, h, per_atom, out);
  return hipGetLastError();
}

// Zero n 64-bit words (a kernel rather than a memset node, so that a captured
// call replays correctly).
__global__ __launch_bounds__(kBlock) void k_zero_u64(uint64_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = 0;
}

hipError_t launch_zero_u64(void* p, size_t bytes, hipStream_t st) {
  const int64_t n = (int64_t)(bytes / 8);
  if (n == 0) return hipSuccess;
  const int64_t want = (n + kBlock - 1) / kBlock;
  const int grid = (int)(want < 1024 ? want : 1024);
  hipLaunchKernelGGL(k_zero_u64, dim3(grid), dim3(kBlock), 0, st, reinterpret_cast<uint64_t*>(p), n);
  return hipGetLastError();
}

// Device scratch of the test-particle runs that cannot allocate (the tallies
// of pm_run_test_particles_static): one copy per GPU, held until the process
// ends.  Host code only ever uses the device address looked up below; the
// array's own name is a host-side stand-in.
static __device__ __align__(256) unsigned char scratch[kTpScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t tp_scratch(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_tp_flight(const TpConst& T, TpTally* tally, uint64_t* e_hist, uint64_t* th_hist,
                            uint64_t* tof_hist, TpTrace trace, int64_t* prof, int grid, hipStream_t st) {
  const size_t lds = (size_t)(T.n_ebins + kTpThetaBins + T.n_tbins) * 4 +
                     (T.n_xbins ? (size_t)4 * (T.n_xbins + 1) * 8 : 0);
  hipLaunchKernelGGL(k_tp_flight, dim3(grid), dim3(kBlock), lds, st, T, tally, e_hist, th_hist, tof_hist, trace,
                     prof);
  return hipGetLastError();
}

}  // namespace pm
