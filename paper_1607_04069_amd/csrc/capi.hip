// C interface of the library (include/picmcc.h): validation, set-up constants,
// arena layout, HIP-graph capture of an RF cycle, read-outs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/picmcc.h"
#include "pm_internal.h"
#include "pm_launch.h"

static_assert(pm::kTpScratchBytes == (size_t)PM_TP_STATIC_BYTES, "static scratch size");

namespace {

// Cells of the test-particle profiles (LDS: 32 B per cell per workgroup).
constexpr int kMaxTpXBins = 1024;

// CODATA 2018
constexpr double kE = 1.602176634e-19;
constexpr double kKB = 1.380649e-23;
constexpr double kME = 9.1093837015e-31;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kAmu = 1.66053906660e-27;
constexpr double kMAr = 39.948 * kAmu;
constexpr double kTwo32 = 4294967296.0;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  }
};

bool valid(const pm_case_params* p) {
  if (!p) return false;
  if (!(p->gap_m > 0) || p->n_cells < 1 || p->n_cells > pm::kMaxCells) return false;
  if (p->steps_per_cycle < 1 || !(p->freq_hz > 0)) return false;
  if (!(p->p_pa >= 0) || !(p->t_gas_k > 0) || !(p->n0_m3 > 0)) return false;
  if (p->np_e < 1 || p->np_i < 0) return false;
  if (p->capacity_e < p->np_e || p->capacity_i < p->np_i) return false;
  if (p->capacity_e > (int64_t)INT32_MAX || p->capacity_i > (int64_t)INT32_MAX) return false;
  if (!(p->te_ev >= 0) || !(p->ti_ev >= 0)) return false;
  if (!(p->ecap_e_ev > 0) || !(p->ecap_i_ev > 0) || p->ecap_i_ev > 1e6) return false;
  if (p->fp64 != 0 && p->fp64 != 1) return false;
  if (p->sort_interval < 0) return false;
  if (!std::isfinite(p->v0_volt) || !std::isfinite(p->phase_rad)) return false;
  if (!std::isfinite(p->v2_volt) || !std::isfinite(p->phase2_rad)) return false;
  if (!(p->cb_f_m2 >= 0) || !std::isfinite(p->cb_f_m2)) return false;
  if (p->n_phase < 0 || p->n_phase > pm::kMaxPhaseBins || p->n_phase > p->steps_per_cycle) return false;
  if (p->flux_profiles != 0 && p->flux_profiles != 1) return false;
  return true;
}

double ln_x_over_x(double eps, double eth, double sigma0) {
  const double x = eps / eth;
  return x > 1.0 ? sigma0 * std::log(x) / x : 0.0;
}

// Eq. (6): the largest n sigma_sum(eps) sqrt(2 eps / m_r) over eps in (0, E_cap],
// on 4096 uniform energies (the cap keeps the constant elastic term bounded).
double nu_max_electron(const pm_case_params* p, double n_gas) {
  const double mr = kME * kMAr / (kME + kMAr);
  double best = 0.0;
  for (int k = 1; k <= 4096; ++k) {
    const double eps = p->ecap_e_ev * (double)k / 4096.0;
    const double sig = p->xs.sigma_el + ln_x_over_x(eps, p->xs.eth_exc, p->xs.sigma0_exc) +
                       ln_x_over_x(eps, p->xs.eth_ion, p->xs.sigma0_ion);
    const double nu = n_gas * sig * std::sqrt(2.0 * eps * kE / mr);
    best = std::max(best, nu);
  }
  return best;
}

// Charge exchange with a constant cross section: the capped ion speed plus ten
// thermal widths of the partner bounds the relative speed.
double nu_max_ion(const pm_case_params* p, double n_gas) {
  const double g = std::sqrt(2.0 * p->ecap_i_ev * kE / kMAr) + 10.0 * std::sqrt(kKB * p->t_gas_k / kMAr);
  return n_gas * p->xs.sigma_cx * g;
}

pm::CaseConst make_const(const pm_case_params* p) {
  pm::CaseConst c;
  std::memset(&c, 0, sizeof(c));
  c.N = p->n_cells;
  c.Nt = p->steps_per_cycle;
  c.n_ebins = (int)std::ceil(p->ecap_i_ev);
  c.sort_interval = p->sort_interval;
  c.flags = p->flags;
  c.fp64 = p->fp64;
  c.dx = p->gap_m / p->n_cells;
  c.dt = 1.0 / (p->freq_hz * p->steps_per_cycle);
  c.w = p->n0_m3 * p->gap_m / (double)p->np_e;
  c.v_scale = c.dx / c.dt;
  c.inv_v_scale = c.dt / c.dx;
  c.c_phi = kE * c.w * c.dx / (kTwo32 * kEps0);
  c.kpush[0] = (-kE / kME) * c.dt * c.dt / c.dx;
  c.kpush[1] = (kE / kMAr) * c.dt * c.dt / c.dx;
  c.ion_over_e = c.kpush[1] / c.kpush[0];
  c.V0 = p->v0_volt;
  c.phase = p->phase_rad;
  c.V2 = p->v2_volt;
  c.phase2 = p->phase2_rad;
  c.cb = p->cb_f_m2;
  c.cgap = kEps0 / p->gap_m;
  c.e_w = kE * c.w;
  c.eps0 = kEps0;
  c.n_gas = p->p_pa / (kKB * p->t_gas_k);
  c.nu_max[0] = nu_max_electron(p, c.n_gas);
  c.nu_max[1] = nu_max_ion(p, c.n_gas);
  c.has_coll = !(p->flags & PM_NO_COLLISIONS) && p->p_pa > 0;
  for (int s = 0; s < 2; ++s) {
    const double P = c.has_coll ? -std::expm1(-c.nu_max[s] * c.dt) : 0.0;
    c.log1m_p[s] = c.has_coll ? std::log1p(-P) : 0.0;
  }
  const double mr_e = kME * kMAr / (kME + kMAr);
  c.half_mr_over_e[0] = 0.5 * mr_e / kE;
  c.half_mr_over_e[1] = 0.5 * (0.5 * kMAr) / kE;
  c.m_ratio_e = kME / (kME + kMAr);
  c.M_ratio_e = kMAr / (kME + kMAr);
  c.two_eexc_over_mr = 2.0 * p->xs.eth_exc * kE / mr_e;
  c.v_e_per_sqrt_ev = std::sqrt(2.0 * kE / kME);
  c.sig_gas = std::sqrt(kKB * p->t_gas_k / kMAr);
  c.sigma_el = p->xs.sigma_el;
  c.eth_exc = p->xs.eth_exc;
  c.sigma0_exc = p->xs.sigma0_exc;
  c.eth_ion = p->xs.eth_ion;
  c.sigma0_ion = p->xs.sigma0_ion;
  c.sigma_cx = p->xs.sigma_cx;
  c.ion_e_factor = 0.5 * kMAr * c.v_scale * c.v_scale / kE;
  c.seed = p->seed;
  c.case_id = p->case_id;
  c.capacity[0] = p->capacity_e;
  c.capacity[1] = p->capacity_i;
  c.n_phase = p->n_phase;
  c.flux = p->flux_profiles;
  // launch shape defaults (pm_set_launch_shape changes them)
  c.dep_mode = 1;
  c.unroll = 8;
  c.waves = 0;
  const char* pf = std::getenv("PM_PROFILE");
  c.prof = pf ? std::atoi(pf) : 0;
  return c;
}

uint32_t warnings_of(const pm_case_params* p, const pm::CaseConst& c) {
  uint32_t w = 0;
  const double lam_d = std::sqrt(kEps0 * p->te_ev / (p->n0_m3 * kE));
  const double omega_p = std::sqrt(p->n0_m3 * kE * kE / (kEps0 * kME));
  if (c.dx > lam_d) w |= PM_WARN_DEBYE;
  if (omega_p * c.dt > 0.2) w |= PM_WARN_PLASMA_FREQ;
  if ((double)p->np_e / p->n_cells < 20.0) w |= PM_WARN_PPC;
  return w;
}

// Workgroups of the step kernel: one per 256 particles (one or more particles
// per lane) up to what fits on the device at once, so every workgroup starts
// with the launch; never fewer than the packed LDS deposit count field allows.
// resident = 0 gives the upper bound used to size the profile buffer.
// Workgroups that share a case's particles: one per 256 initial particles, at
// most one resident wave of the step kernel (resident > 0).
int work_grid_for(const pm_case_params* p, int64_t resident = 0) {
  const int64_t T0 = p->np_e + p->np_i;
  int64_t g = (T0 + pm::kBlock - 1) / pm::kBlock;
  if (resident > 0) g = std::min(g, resident);
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65535));
}

// Workgroups of the step kernel resident on the whole device at once.
int resident_step_blocks(bool fp64, int N, int unroll, int waves, bool batch) {
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
  const int per_cu = fp64 ? pm::step_blocks_per_cu<double>(N, unroll, waves, batch)
                          : pm::step_blocks_per_cu<float>(N, unroll, waves, batch);
  return per_cu * cus;
}

bool valid_shape(const pm_launch_shape* s) {
  return s && (s->unroll == 8 || s->unroll == 16) && (s->waves == 0 || s->waves == 6) && s->work_groups >= 0 &&
         s->deposit_mode >= 0 && s->deposit_mode <= 1 && s->sort_interval >= 0 && s->lanes >= 0 && s->lanes <= 4;
}

// Lower bound of a step launch's grid: capacity / kMaxSlotsPerBlock.  The working
// workgroups cover every slot whatever their number (strided tiles, and a tile
// flush before the per-tile cap), so workgroups beyond them only share the
// rotation of the charge buffers.
int slot_grid_for(const pm_case_params* p) {
  const int64_t cap = p->capacity_e + p->capacity_i;
  return (int)std::max<int64_t>(1, (cap + pm::kMaxSlotsPerBlock - 1) / pm::kMaxSlotsPerBlock);
}

// The largest step grid a case can be launched with (its profile slots).
int max_step_grid_for(const pm_case_params* p) { return std::max(work_grid_for(p), slot_grid_for(p)); }

// Collision candidates a case is expected to list per step at its initial load.
double expected_candidates(const pm_case_params* p, const pm::CaseConst& c) {
  double e = 0.0;
  for (int s = 0; s < 2; ++s) e += (double)(s ? p->np_i : p->np_e) * -std::expm1(c.log1m_p[s]);
  return e;
}

// Expected candidates per collision lane: one while they fit in a resident wave
// of collision workgroups, up to four beyond that (fewer, fuller workgroups
// amortise each workgroup's fixed cost: counter flush, completion wait, done
// count).  resident: collision workgroups resident on the device.
double mcc_per_lane(double candidates, int64_t resident) {
  return std::max(1.0, std::min(4.0, candidates / ((double)resident * pm::kBlock)));
}

// Workgroups of a case's collision launch for a given load per lane (the
// launch grid-strides over any count), at most the case's profile rows.
int mcc_grid_for(const pm_case_params* p, const pm::CaseConst& c, double per_lane) {
  const int64_t g = (int64_t)std::ceil(expected_candidates(p, c) / (per_lane * pm::kBlock));
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, max_step_grid_for(p)));
}

int resident_mcc_blocks(bool fp64, int N, bool batch) {
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
  const int per_cu = fp64 ? pm::mcc_blocks_per_cu<double>(N, batch) : pm::mcc_blocks_per_cu<float>(N, batch);
  return per_cu * cus;
}

struct ArenaMap {
  size_t ctrl, part[2][2][4], Q, sumQ, Epair, E64, phi64, diag_out, iedf, iadf, cell_count, cell_off, ybin,
      yield_out, prof, args, cand, cand_xu, banks, sumQp, phase_v, phase_n, sumF, flux_n, iedf_taken, iead, total;
};

ArenaMap layout(const pm_case_params* p) {
  ArenaMap m;
  Layout L;
  const size_t sr = p->fp64 ? 8 : 4;
  const size_t nodes = (size_t)p->n_cells + 1;
  const size_t N = (size_t)p->n_cells;
  const size_t nb = (size_t)std::ceil(p->ecap_i_ev);
  m.ctrl = L.take(sizeof(pm::Ctrl));
  for (int s = 0; s < 2; ++s) {
    const size_t cap = (size_t)(s ? p->capacity_i : p->capacity_e);
    for (int b = 0; b < 2; ++b) {
      m.part[s][b][0] = L.take(cap * sr);
      m.part[s][b][1] = L.take(cap * sr);
      m.part[s][b][2] = L.take(cap * (p->fp64 ? sizeof(pm::Cold<double>) : sizeof(pm::Cold<float>)));
      m.part[s][b][3] = L.take(cap * 2);
    }
  }
  m.Q = L.take(3 * 2 * nodes * 8);
  m.sumQ = L.take(2 * nodes * 2 * 8);
  m.Epair = L.take(2 * N * 2 * sr);
  m.E64 = L.take(nodes * 8);
  m.phi64 = L.take(nodes * 8);
  m.diag_out = L.take(7 * nodes * 8);
  m.iedf = L.take(2 * nb * 8);
  m.iadf = L.take(2 * pm::kAngleBins * 8);
  m.cell_count = L.take(2 * N * 4);
  m.cell_off = L.take(2 * N * 4);
  m.ybin = L.take(nb * 8);
  m.yield_out = L.take(4 * 8);
  m.prof = L.take((size_t)max_step_grid_for(p) * 8 * 8);
  m.args = L.take(std::max(sizeof(pm::KArgs<float>), sizeof(pm::KArgs<double>)));
  m.cand = L.take((size_t)(p->capacity_e + p->capacity_i) * 4);
  m.cand_xu = L.take((size_t)(p->capacity_e + p->capacity_i) * 2 * sr);
  m.banks = L.take((size_t)pm::kBanks * pm::kBankStride);
  const size_t nph = (size_t)p->n_phase, nf = p->flux_profiles ? std::max<size_t>(nph, 1) : 0;
  m.sumQp = L.take(nph * 2 * nodes * 2 * 8);
  m.phase_v = L.take(nph * 8);
  m.phase_n = L.take(nph * 8);
  m.sumF = L.take(nf * 2 * nodes * 2 * 8);
  m.flux_n = L.take(nf * 8);
  m.iedf_taken = L.take(2 * nb * 8);
  m.iead = L.take(2 * ((nb + pm::kIeadEGroup - 1) / pm::kIeadEGroup) * pm::kIeadABins * 8);
  m.total = L.off;
  return m;
}

template <typename R>
void fill_args(pm::KArgs<R>& A, const pm::CaseConst& c, char* base, const ArenaMap& m) {
  A.c = c;
  A.ctrl = reinterpret_cast<pm::Ctrl*>(base + m.ctrl);
  for (int s = 0; s < 2; ++s)
    for (int b = 0; b < 2; ++b) {
      A.p.xt[s][b] = (std::remove_reference_t<decltype(A.p.xt[s][b])>)(base + m.part[s][b][0]);
      A.p.ux[s][b] = (std::remove_reference_t<decltype(A.p.ux[s][b])>)(base + m.part[s][b][1]);
      A.p.cold[s][b] = (std::remove_reference_t<decltype(A.p.cold[s][b])>)(base + m.part[s][b][2]);
      A.p.next[s][b] = (std::remove_reference_t<decltype(A.p.next[s][b])>)(base + m.part[s][b][3]);
    }
  A.g.Q = reinterpret_cast<int64_t*>(base + m.Q);
  A.g.sumQ = reinterpret_cast<uint64_t*>(base + m.sumQ);
  A.g.Epair = base + m.Epair;
  A.g.E64 = reinterpret_cast<double*>(base + m.E64);
  A.g.phi64 = reinterpret_cast<double*>(base + m.phi64);
  A.g.diag_out = reinterpret_cast<double*>(base + m.diag_out);
  A.g.iedf = reinterpret_cast<uint64_t*>(base + m.iedf);
  A.g.iadf = reinterpret_cast<uint64_t*>(base + m.iadf);
  A.g.cell_count = reinterpret_cast<uint32_t*>(base + m.cell_count);
  A.g.cell_off = reinterpret_cast<uint32_t*>(base + m.cell_off);
  A.g.ybin = reinterpret_cast<double*>(base + m.ybin);
  A.g.yield_out = reinterpret_cast<uint64_t*>(base + m.yield_out);
  A.g.prof = reinterpret_cast<uint64_t*>(base + m.prof);
  A.g.cand = reinterpret_cast<uint32_t*>(base + m.cand);
  A.g.cand_xu = base + m.cand_xu;
  A.g.banks = reinterpret_cast<unsigned char*>(base + m.banks);
  A.g.sumQp = reinterpret_cast<uint64_t*>(base + m.sumQp);
  A.g.phase_v = reinterpret_cast<double*>(base + m.phase_v);
  A.g.phase_n = reinterpret_cast<int64_t*>(base + m.phase_n);
  A.g.sumF = reinterpret_cast<uint64_t*>(base + m.sumF);
  A.g.flux_n = reinterpret_cast<int64_t*>(base + m.flux_n);
  A.g.iedf_taken = reinterpret_cast<uint64_t*>(base + m.iedf_taken);
  A.g.iead = reinterpret_cast<uint64_t*>(base + m.iead);
}

}  // namespace

struct pm_case {
  pm_case_params prm;
  pm::CaseConst c;
  ArenaMap map;
  char* arena;
  size_t bytes;
  uint32_t warnings;
  pm::KArgs<float> af;
  pm::KArgs<double> ad;
  int step_grid;   // workgroups of a step launch
  int work_grid;   // of which share the particles
  int mcc_grid;    // workgroups of the collision launch
  int sort_grid;
  hipStream_t cap_stream;
  hipGraph_t graph;
  hipGraphExec_t exec;
  bool has_graph;
  pm_status failed;
  // live injection (pm_sputter_params.since_last) per electrode: atoms emitted
  // by such calls in the averaging window so far, and the step of the last call
  int64_t live_atoms[2];
  int64_t live_step[2];
  int64_t since_sort;   // steps of plain launches since the last sort
};

namespace {

#define PM_TRY(x)                                   \
  do {                                              \
    if ((x) != hipSuccess) return PM_EDEVICE;       \
  } while (0)

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

template <typename R>
pm::KArgs<R>& args_of(pm_case* c);
template <>
pm::KArgs<float>& args_of<float>(pm_case* c) { return c->af; }
template <>
pm::KArgs<double>& args_of<double>(pm_case* c) { return c->ad; }

// device copy of the case's kernel arguments (written at init)
template <typename R>
const pm::KArgs<R>* dev_args(pm_case* c) {
  return reinterpret_cast<const pm::KArgs<R>*>(c->arena + c->map.args);
}

// Sort cadence.  Plain launches sort after every K-th step counted across
// calls (since: steps since the last sort), so a caller that advances fewer than
// K steps per call still sorts, and births keep being compacted.  A captured RF
// cycle is replayed as a whole, so its sorts fall at fixed places of the cycle:
// every Kc-th step, Kc the largest divisor of N_t not above K (K itself when it
// divides N_t), which keeps the same cadence from one replay to the next.
bool sort_due(int64_t* since, int K) {
  if (K <= 0) return false;
  if (++*since < K) return false;
  *since = 0;
  return true;
}

int cycle_sort_interval(int K, int Nt) {
  if (K <= 0 || Nt < 1) return 0;
  int k = std::min(K, Nt);
  while (Nt % k) --k;
  return k;
}

// Workgroups of a case's sort: one per 2048-slot chunk of the initial particles
// (the scatter grid-strides over however many chunks the slot range holds).
// Sized by the capacity instead, three in four workgroups found no chunk and
// only queued on the case's done counter: the sweep's sorts took 15 % longer.
int sort_grid_for(const pm_case_params* p) {
  const int64_t n0 = p->np_e + p->np_i;
  int64_t g = (n0 + 2047) / 2048;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 2048));
}

// n steps with plain launches; captured (an RF cycle for a graph) sorts at the
// cycle's fixed places instead of by the running count.
template <typename R>
pm_status run_steps(pm_case* c, int64_t n, hipStream_t st, bool captured = false) {
  const pm::KArgs<R>& A = args_of<R>(c);
  const int K = c->prm.sort_interval;
  const int Kc = cycle_sort_interval(K, c->prm.steps_per_cycle);
  for (int64_t i = 0; i < n; ++i) {
    const int sort = captured ? (Kc > 0 && (i + 1) % Kc == 0) : sort_due(&c->since_sort, K);
    PM_TRY(pm::launch_step<R>(A, dev_args<R>(c), c->step_grid, c->work_grid, sort, st));
    PM_TRY(pm::launch_mcc<R>(A, dev_args<R>(c), c->mcc_grid, sort, st));
    if (sort) PM_TRY(pm::launch_sort<R>(A, c->sort_grid, st));
  }
  return PM_OK;
}

template <typename R>
pm_status prepare(pm_case* c, hipStream_t st) {
  // deposit the current particles, sort them by cell and solve the field
  const pm::KArgs<R>& A = args_of<R>(c);
  const int nodes = c->c.N + 1;
  PM_TRY(hipMemsetAsync(A.g.Q, 0, (size_t)3 * 2 * nodes * 8, st));
  PM_TRY(hipMemsetAsync(A.g.cell_count, 0, (size_t)2 * c->c.N * 4, st));
  PM_TRY(pm::launch_deposit_all<R>(A, std::max(c->prm.capacity_e, c->prm.capacity_i), st));
  PM_TRY(pm::launch_scan_cells(A.c, A.g, A.ctrl, st));
  PM_TRY(pm::launch_sort<R>(A, c->sort_grid, st));
  PM_TRY(pm::launch_field<R>(A, 0, st));
  return PM_OK;
}

template <typename R>
pm_status init_impl(pm_case* c, hipStream_t st) {
  const pm::KArgs<R>& A = args_of<R>(c);
  PM_TRY(hipMemsetAsync(c->arena, 0, c->map.total, st));
  pm::Ctrl h;
  std::memset(&h, 0, sizeof(h));
  h.n_range[0] = h.n_alloc[0] = h.n_live[0] = c->prm.np_e;
  h.n_range[1] = h.n_alloc[1] = h.n_live[1] = c->prm.np_i;
  PM_TRY(hipMemcpyAsync(A.ctrl, &h, sizeof(h), hipMemcpyHostToDevice, st));
  const double sig_e = std::sqrt(c->prm.te_ev * kE / kME);
  const double sig_i = std::sqrt(c->prm.ti_ev * kE / kMAr);
  PM_TRY(hipMemcpyAsync(c->arena + c->map.args, &A, sizeof(A), hipMemcpyHostToDevice, st));
  PM_TRY(pm::launch_load<R>(A, c->prm.np_e, c->prm.np_i, sig_e, sig_i, st));
  pm_status s = prepare<R>(c, st);
  if (s != PM_OK) return s;
  PM_TRY(hipStreamSynchronize(st));
  return PM_OK;
}

// The control block with the step counters' banks added in (the host view of
// every counter is the sum).
pm_status read_ctrl(pm_case* c, pm::Ctrl* h, hipStream_t st) {
  // the banks' whole region in one plain copy (64 KiB), picked apart on the host
  std::vector<unsigned char> raw((size_t)pm::kBanks * pm::kBankStride);
  PM_TRY(hipMemcpyAsync(h, c->arena + c->map.ctrl, sizeof(pm::Ctrl), hipMemcpyDeviceToHost, st));
  PM_TRY(hipMemcpyAsync(raw.data(), c->arena + c->map.banks, raw.size(), hipMemcpyDeviceToHost, st));
  PM_TRY(hipStreamSynchronize(st));
  pm::CtrBank b[pm::kBanks];
  for (int i = 0; i < pm::kBanks; ++i) std::memcpy(&b[i], raw.data() + (size_t)i * pm::kBankStride, sizeof(pm::CtrBank));
  for (const pm::CtrBank& k : b) {
    h->particle_steps += k.particle_steps;
    h->births += k.births;
    for (int s = 0; s < 2; ++s) {
      h->candidates[s] += k.candidates[s];
      h->overflow[s] += k.overflow[s];
      h->n_live[s] += k.n_live[s];
      h->absorbed[s][0] += k.absorbed[s][0];
      h->absorbed[s][1] += k.absorbed[s][1];
    }
    for (int j = 0; j < 5; ++j) h->collisions[j] += k.collisions[j];
  }
  return PM_OK;
}

// turn sticky device failure bits into the case's failed status
pm_status check_status(pm_case* c, const pm::Ctrl& h) {
  if (h.status & pm::ST_CAPACITY) c->failed = PM_ECAPACITY;
  else if (h.status & pm::ST_NUMERIC) c->failed = PM_ENUMERIC;
  return c->failed;
}

template <typename R>
pm_status build_graph(pm_case* c) {
  if (c->has_graph) return PM_OK;
  if (!c->cap_stream) PM_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  PM_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  pm_status s = run_steps<R>(c, c->prm.steps_per_cycle, c->cap_stream, true);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
  if (s != PM_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return PM_EDEVICE;
  }
  if (hipGraphInstantiate(&c->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    c->exec = nullptr;                     // never keep what a failed instantiation left there
    (void)hipGraphDestroy(g);
    return PM_EDEVICE;
  }
  c->graph = g;
  c->has_graph = true;
  return PM_OK;
}

template <typename R>
pm_status get_particles_impl(pm_case* c, int s, pm_particles* out, hipStream_t st) {
  pm::Ctrl h;
  pm_status rs = read_ctrl(c, &h, st);
  if (rs != PM_OK) return rs;
  const pm::KArgs<R>& A = args_of<R>(c);
  const int64_t n = h.n_range[s];
  const uint32_t b = h.buf;
  std::vector<R> x(n), ux(n);
  std::vector<pm::Cold<R>> cold(n);
  std::vector<uint16_t> nx(n);
  if (n) {
    PM_TRY(hipMemcpy(x.data(), A.p.xt[s][b], n * sizeof(R), hipMemcpyDeviceToHost));
    PM_TRY(hipMemcpy(ux.data(), A.p.ux[s][b], n * sizeof(R), hipMemcpyDeviceToHost));
    PM_TRY(hipMemcpy(cold.data(), A.p.cold[s][b], n * sizeof(pm::Cold<R>), hipMemcpyDeviceToHost));
    PM_TRY(hipMemcpy(nx.data(), A.p.next[s][b], n * 2, hipMemcpyDeviceToHost));
  }
  const bool coll = c->c.log1m_p[s] != 0.0;
  const uint32_t l15 = (uint32_t)h.step & 0x7FFFu;
  int64_t live = 0;
  for (int64_t k = 0; k < n; ++k) live += x[k] >= (R)0;
  out->n = live;
  if (out->capacity < live) return PM_EINVAL;
  if (live > 0 && (!out->xt || !out->ux || !out->uy || !out->uz || !out->id || !out->next)) return PM_EINVAL;
  int64_t o = 0;
  for (int64_t k = 0; k < n; ++k) {
    if (!(x[k] >= (R)0)) continue;
    out->xt[o] = (double)x[k];
    out->ux[o] = (double)ux[k];
    out->uy[o] = (double)cold[k].uy;
    out->uz[o] = (double)cold[k].uz;
    out->id[o] = cold[k].id;
    // the examination code holds the step modulo 2^15, at most kWaitCap ahead
    out->next[o] = coll ? (uint32_t)(h.step + (int64_t)(((uint32_t)nx[k] - l15) & 0x7FFFu)) |
                              ((nx[k] & pm::kRedraw) ? 0x80000000u : 0u)
                        : 0xFFFFFFFFu;
    ++o;
  }
  return check_status(c, h) == PM_OK ? PM_OK : c->failed;
}

template <typename R>
pm_status set_particles_impl(pm_case* c, int s, const pm_particles* in, hipStream_t st) {
  const int64_t cap = s ? c->prm.capacity_i : c->prm.capacity_e;
  if (in->n < 0 || in->n > cap) return PM_EINVAL;
  if (s == 0 && in->n < 1) return PM_EINVAL;
  const int64_t n = in->n;
  for (int64_t k = 0; k < n; ++k)
    if (!(in->xt[k] >= 0.0 && in->xt[k] < (double)c->c.N)) return PM_EINVAL;
  pm::Ctrl h;
  pm_status rs = read_ctrl(c, &h, st);
  if (rs != PM_OK) return rs;
  const pm::KArgs<R>& A = args_of<R>(c);
  const uint32_t b = h.buf;
  // examination codes: the step (at most kWaitCap ahead of the next step to
  // run) modulo 2^15, with the redraw bit; unused for a species without collisions
  const bool coll = c->c.log1m_p[s] != 0.0;
  std::vector<uint16_t> nx(n, 0);
  for (int64_t k = 0; k < n && coll; ++k) {
    const int64_t at = (int64_t)(in->next[k] & 0x7FFFFFFFu);
    if (at < h.step || at > h.step + pm::kWaitCap) return PM_EINVAL;
    nx[k] = (uint16_t)(((uint32_t)at & 0x7FFFu) | ((in->next[k] >> 31) ? pm::kRedraw : 0u));
  }
  std::vector<R> x(n), ux(n);
  std::vector<pm::Cold<R>> cold(n);
  for (int64_t k = 0; k < n; ++k) {
    x[k] = (R)in->xt[k];
    ux[k] = (R)in->ux[k];
    cold[k].uy = (R)in->uy[k];
    cold[k].uz = (R)in->uz[k];
    cold[k].id = in->id[k];
    if (!(x[k] < (R)c->c.N)) x[k] = std::nextafter((R)c->c.N, (R)0);
  }
  if (n) {
    PM_TRY(hipMemcpy(A.p.xt[s][b], x.data(), n * sizeof(R), hipMemcpyHostToDevice));
    PM_TRY(hipMemcpy(A.p.ux[s][b], ux.data(), n * sizeof(R), hipMemcpyHostToDevice));
    PM_TRY(hipMemcpy(A.p.cold[s][b], cold.data(), n * sizeof(pm::Cold<R>), hipMemcpyHostToDevice));
    PM_TRY(hipMemcpy(A.p.next[s][b], nx.data(), n * 2, hipMemcpyHostToDevice));
  }
  h.n_range[s] = h.n_alloc[s] = h.n_live[s] = n;
  // the control block takes the summed counters; the banks start again from zero
  PM_TRY(hipMemcpy(A.ctrl, &h, sizeof(h), hipMemcpyHostToDevice));
  PM_TRY(hipMemset(c->arena + c->map.banks, 0, (size_t)pm::kBanks * pm::kBankStride));
  pm_status ps = prepare<R>(c, st);
  if (ps != PM_OK) return ps;
  PM_TRY(hipStreamSynchronize(st));
  return PM_OK;
}

template <typename R>
pm_status get_fields_impl(pm_case* c, pm_fields* out, hipStream_t st) {
  const pm::KArgs<R>& A = args_of<R>(c);
  PM_TRY(pm::launch_field<R>(A, 1, st));
  pm::Ctrl h;
  pm_status rs = read_ctrl(c, &h, st);
  if (rs != PM_OK) return rs;
  const int nodes = c->c.N + 1;
  const int64_t* Q = A.g.Q + pm::qbuf_index(h.step, 0) * 2 * nodes;
  if (out->qe) PM_TRY(hipMemcpy(out->qe, Q, nodes * 8, hipMemcpyDeviceToHost));
  if (out->qi) PM_TRY(hipMemcpy(out->qi, Q + nodes, nodes * 8, hipMemcpyDeviceToHost));
  if (out->phi) PM_TRY(hipMemcpy(out->phi, A.g.phi64, nodes * 8, hipMemcpyDeviceToHost));
  if (out->efield) PM_TRY(hipMemcpy(out->efield, A.g.E64, nodes * 8, hipMemcpyDeviceToHost));
  out->sigma_init = c->c.cb > 0.0 ? h.sigma_init : 0.0;
  out->n_absorbed_net = c->c.cb > 0.0 ? h.n_abs_net : 0;
  return PM_OK;
}

template <typename R>
pm_status sample_impl(pm_case* c, pm_diagnostics* out, int reset, hipStream_t st) {
  const pm::KArgs<R>& A = args_of<R>(c);
  PM_TRY(pm::launch_diag_finalize<R>(A, -1, st));
  pm::Ctrl h;
  pm_status rs = read_ctrl(c, &h, st);
  if (rs != PM_OK) return rs;
  const int nodes = c->c.N + 1;
  const int nb = c->c.n_ebins;
  std::vector<double> d(7 * (size_t)nodes);
  PM_TRY(hipMemcpy(d.data(), A.g.diag_out, d.size() * 8, hipMemcpyDeviceToHost));
  if (out->ne) std::memcpy(out->ne, d.data(), nodes * 8);
  if (out->ni) std::memcpy(out->ni, d.data() + nodes, nodes * 8);
  if (out->phi) std::memcpy(out->phi, d.data() + 2 * nodes, nodes * 8);
  if (out->gamma_e) std::memcpy(out->gamma_e, d.data() + 3 * nodes, nodes * 8);
  if (out->gamma_i) std::memcpy(out->gamma_i, d.data() + 4 * nodes, nodes * 8);
  if (out->u_e) std::memcpy(out->u_e, d.data() + 5 * nodes, nodes * 8);
  if (out->u_i) std::memcpy(out->u_i, d.data() + 6 * nodes, nodes * 8);
  if (out->iedf) PM_TRY(hipMemcpy(out->iedf, A.g.iedf, (size_t)2 * nb * 8, hipMemcpyDeviceToHost));
  if (out->iadf) PM_TRY(hipMemcpy(out->iadf, A.g.iadf, (size_t)2 * pm::kAngleBins * 8, hipMemcpyDeviceToHost));
  if (out->iead)
    PM_TRY(hipMemcpy(out->iead, A.g.iead, (size_t)2 * ((nb + pm::kIeadEGroup - 1) / pm::kIeadEGroup) * pm::kIeadABins * 8,
                     hipMemcpyDeviceToHost));
  out->step = h.step;
  out->warnings = c->warnings;
  out->n_e = h.n_live[0];
  out->n_i = h.n_live[1];
  out->avg_steps = h.avg_steps;
  const double tw = (h.avg_steps > 0 ? (double)h.avg_steps : 1.0) * c->c.dt;
  for (int s = 0; s < 2; ++s)
    for (int el = 0; el < 2; ++el) {
      out->absorbed[s][el] = h.absorbed[s][el];
      out->flux[s][el] = (double)h.absorbed[s][el] * c->c.w / tw;
    }
  for (int el = 0; el < 2; ++el)
    out->mean_ion_energy[el] =
        h.absorbed[1][el] ? (double)h.ion_e_fx[el] / 1048576.0 / (double)h.absorbed[1][el] : 0.0;
  for (int k = 0; k < 5; ++k) out->collisions[k] = h.collisions[k];
  for (int s = 0; s < 2; ++s) {
    out->candidates[s] = h.candidates[s];
    out->overflow[s] = h.overflow[s];
  }
  out->births = h.births;
  out->particle_steps = h.particle_steps;
  out->status = (int32_t)check_status(c, h);
  if (reset) {
    PM_TRY(pm::launch_diag_reset(A.c, A.g, A.ctrl, st));
    PM_TRY(hipStreamSynchronize(st));
    for (int e = 0; e < 2; ++e) {
      c->live_atoms[e] = 0;
      c->live_step[e] = h.step;
    }
  }
  return c->failed;
}

template <typename R>
pm_status sample_phase_impl(pm_case* c, int bin, pm_phase_sample* out, hipStream_t st) {
  const pm::KArgs<R>& A = args_of<R>(c);
  PM_TRY(pm::launch_diag_finalize<R>(A, bin, st));
  pm::Ctrl h;
  pm_status rs = read_ctrl(c, &h, st);
  if (rs != PM_OK) return rs;
  const int nodes = c->c.N + 1;
  std::vector<double> d(7 * (size_t)nodes);
  PM_TRY(hipMemcpy(d.data(), A.g.diag_out, d.size() * 8, hipMemcpyDeviceToHost));
  double* dst[7] = {out->ne, out->ni, out->phi, out->gamma_e, out->gamma_i, out->u_e, out->u_i};
  for (int k = 0; k < 7; ++k)
    if (dst[k]) std::memcpy(dst[k], d.data() + (size_t)k * nodes, nodes * 8);
  int64_t v[2] = {0, 0};
  PM_TRY(hipMemcpy(&v[0], A.g.phase_n + bin, 8, hipMemcpyDeviceToHost));
  if (c->c.flux) PM_TRY(hipMemcpy(&v[1], A.g.flux_n + bin, 8, hipMemcpyDeviceToHost));
  out->n_steps = v[0];
  out->n_flux_samples = v[1];
  out->status = (int32_t)check_status(c, h);
  return c->failed;
}

double yield_at(const pm_sputter_params* sp, double e) {
  if (sp->n_table <= 0) return sp->yield_const;
  const double* x = sp->table_e_ev;
  const double* y = sp->table_y;
  const int n = sp->n_table;
  if (e <= x[0]) return y[0];
  if (e >= x[n - 1]) return y[n - 1];
  int k = 0;
  while (k + 1 < n && x[k + 1] < e) ++k;
  const double t = (e - x[k]) / (x[k + 1] - x[k]);
  return y[k] + t * (y[k + 1] - y[k]);
}


// Device layout of a test-particle run (an arena, or the static scratch): the
// counters, the substrate histograms, the track-length tallies ([4][n_xbins + 1]
// int64) and the finished profiles ([4][n_xbins] doubles).
struct TpLayout {
  size_t tally, e_hist, th_hist, tof_hist, prof, prof_out, total;
};

TpLayout tp_layout(const pm_tp_params* tp) {
  Layout L;
  TpLayout m;
  m.tally = L.take(sizeof(pm::TpTally));
  m.e_hist = L.take((size_t)tp->n_ebins * 8);
  m.th_hist = L.take((size_t)pm::kTpThetaBins * 8);
  m.tof_hist = L.take((size_t)tp->n_tbins * 8);
  m.prof = L.take((size_t)4 * (tp->n_xbins + 1) * 8);
  m.prof_out = L.take((size_t)4 * tp->n_xbins * 8);
  m.total = L.off;
  return m;
}

pm_status tp_validate(const pm_tp_params* tp, const pm_tp_source* src) {
  if (!(tp->p_pa >= 0) || !(tp->t_gas_k > 0) || !(tp->d_ref > 0) || !(tp->omega >= 0.5) || !(tp->omega < 1.0))
    return PM_EINVAL;
  if (!(tp->t_ref > 0) || !(tp->m_test_amu > 0) || !(tp->m_gas_amu > 0) || !(tp->gap_m > 0) ||
      !(tp->lateral_m > 0))
    return PM_EINVAL;
  if (tp->mode != PM_TP_NORMAL && tp->mode != PM_TP_BOX) return PM_EINVAL;
  if (tp->scatter != PM_TP_VHS && tp->scatter != PM_TP_M1) return PM_EINVAL;
  if (!(tp->dt_s >= 0) || !std::isfinite(tp->dt_s)) return PM_EINVAL;
  if (tp->e_max < 1 || tp->e_max > (int64_t)UINT32_MAX || tp->n_ebins < 1 || tp->n_tbins < 1) return PM_EINVAL;
  if (!(tp->ebin_ev > 0) || !(tp->tbin_s > 0)) return PM_EINVAL;
  if (tp->n_xbins < 0 || tp->n_xbins > kMaxTpXBins) return PM_EINVAL;
  if (src->n_atoms < 0 || src->first_atom < 0 || !(src->u_s_ev > 0) || !(src->e_cut_ev > 0)) return PM_EINVAL;
  if (src->electrode != 0 && src->electrode != 1) return PM_EINVAL;
  return PM_OK;
}

// The flight of src->n_atoms atoms with its tallies at base (tp_layout bytes,
// 256-byte aligned); fills *out from there.  Allocates nothing: the device
// buffers are the caller's, the read-outs go straight into the caller's host
// arrays and a struct on the stack.  Synchronises the stream.
pm_status tp_run(const pm_tp_params* tp, const pm_tp_source* src, char* base, hipStream_t st, pm_tp_result* out) {
  const double m = tp->m_test_amu * kAmu, M = tp->m_gas_amu * kAmu;
  const double mr = m * M / (m + M);
  const double n_gas = tp->p_pa / (kKB * tp->t_gas_k);
  const double g_cap = std::sqrt(2.0 * src->e_cut_ev * kE / m) + 10.0 * std::sqrt(kKB * tp->t_gas_k / M);
  // Eq. (8): sigma = pi b_max^2 with b_max^2 = d_ref^2 (2 k T_ref / (m_r g^2))^(omega - 1/2) / Gamma(5/2 - omega);
  // M1 reuses the VHS data with d_ref sqrt(4/3)
  const double d2 = tp->d_ref * tp->d_ref * (tp->scatter == PM_TP_M1 ? 4.0 / 3.0 : 1.0);
  const double sig_cap = M_PI * d2 *
                         std::pow(2.0 * kKB * tp->t_ref / (mr * g_cap * g_cap), tp->omega - 0.5) /
                         std::tgamma(2.5 - tp->omega);
  pm::TpConst t;
  std::memset(&t, 0, sizeof(t));
  t.L = tp->gap_m;
  t.lat = tp->lateral_m;
  t.nu_max = n_gas * sig_cap * g_cap;
  t.inv_nu_max = t.nu_max > 0 ? 1.0 / t.nu_max : INFINITY;
  t.sg_exp = 2.0 - 2.0 * tp->omega;
  t.log2_gcap = std::log2(g_cap);
  t.sig_gas = std::sqrt(kKB * tp->t_gas_k / M);
  t.m_ratio = m / (m + M);
  t.M_ratio = M / (m + M);
  t.s_max = src->e_cut_ev / (src->e_cut_ev + src->u_s_ev);
  t.u_s = src->u_s_ev;
  t.v_per_sqrt_ev = std::sqrt(2.0 * kE / m);
  t.e_half_m = 0.5 * m / kE;
  t.ebin = tp->ebin_ev;
  t.tbin = tp->tbin_s;
  t.n_ebins = tp->n_ebins;
  t.n_tbins = tp->n_tbins;
  t.n_xbins = tp->mode == PM_TP_NORMAL ? tp->n_xbins : 0;
  t.xbin = tp->gap_m / std::max(tp->n_xbins, 1);
  t.inv_xbin = 1.0 / t.xbin;
  t.mode = tp->mode;
  t.scatter = tp->scatter;
  t.electrode = src->electrode;
  t.dt = tp->dt_s;
  t.nu_dt = t.nu_max * tp->dt_s;
  t.e_max = tp->e_max;
  t.n_atoms = src->n_atoms;
  t.first_atom = src->first_atom;
  t.seed = src->seed;
  t.job = src->job_id;
  const TpLayout L = tp_layout(tp);
  pm::TpTally* tal = reinterpret_cast<pm::TpTally*>(base + L.tally);
  uint64_t* eh = reinterpret_cast<uint64_t*>(base + L.e_hist);
  uint64_t* th = reinterpret_cast<uint64_t*>(base + L.th_hist);
  uint64_t* tofh = reinterpret_cast<uint64_t*>(base + L.tof_hist);
  int64_t* prof = reinterpret_cast<int64_t*>(base + L.prof);
  double* pout = reinterpret_cast<double*>(base + L.prof_out);
  PM_TRY(pm::launch_zero_u64(base, L.total, st));
  pm::TpTrace tr;
  std::memset(&tr, 0, sizeof(tr));
  if (out->trace) {
    tr.wall = out->trace->wall;
    tr.events = out->trace->events;
    tr.energy_ev = out->trace->energy_ev;
    tr.theta_deg = out->trace->theta_deg;
    tr.tof_s = out->trace->tof_s;
    tr.vx = out->trace->vx;
    tr.vy = out->trace->vy;
    tr.vz = out->trace->vz;
  }
  const int64_t want = (src->n_atoms + pm::kBlock - 1) / pm::kBlock;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, 256 * 8));
  if (src->n_atoms > 0) PM_TRY(pm::launch_tp_flight(t, tal, eh, th, tofh, tr, prof, grid, st));
  const int nx = t.n_xbins;
  if (nx) {
    const double per_atom = src->flux_m2s / (double)std::max<int64_t>(src->n_atoms, 1);
    PM_TRY(pm::launch_tp_profiles(prof, nx, t.xbin, per_atom, pout, st));
  }
  pm::TpTally h;
  PM_TRY(hipMemcpyAsync(&h, tal, sizeof(h), hipMemcpyDeviceToHost, st));
  if (out->e_hist) PM_TRY(hipMemcpyAsync(out->e_hist, eh, (size_t)tp->n_ebins * 8, hipMemcpyDeviceToHost, st));
  if (out->theta_hist)
    PM_TRY(hipMemcpyAsync(out->theta_hist, th, (size_t)pm::kTpThetaBins * 8, hipMemcpyDeviceToHost, st));
  if (out->tof_hist) PM_TRY(hipMemcpyAsync(out->tof_hist, tofh, (size_t)tp->n_tbins * 8, hipMemcpyDeviceToHost, st));
  double* const dst[4] = {out->time_s, out->disp_m, out->density_m3, out->mean_vx};
  for (int q = 0; q < 4; ++q)
    if (dst[q] && tp->n_xbins > 0) {
      if (nx) PM_TRY(hipMemcpyAsync(dst[q], pout + (size_t)q * nx, (size_t)nx * 8, hipMemcpyDeviceToHost, st));
      else std::memset(dst[q], 0, (size_t)tp->n_xbins * 8);    // no profiles in a periodic box
    }
  PM_TRY(hipStreamSynchronize(st));
  out->n_substrate = (int64_t)h.n_sub;
  out->n_target = (int64_t)h.n_tgt;
  out->n_unfinished = (int64_t)h.n_unf;
  out->events = h.events;
  out->collisions = h.collisions;
  out->overflow = h.overflow;
  out->e_sum_substrate = (double)h.e_sub_fx / 1048576.0;
  out->e_sum_target = (double)h.e_tgt_fx / 1048576.0;
  out->eta = src->n_atoms > 0 ? (double)h.n_sub / (double)src->n_atoms : 0.0;
  out->deposition_flux = out->eta * src->flux_m2s;
  out->nu_max = t.nu_max;
  return PM_OK;
}
}  // namespace

extern "C" {

const char* pm_status_string(pm_status s) {
  switch (s) {
    case PM_OK: return "ok";
    case PM_EINVAL: return "invalid argument";
    case PM_ENOSPACE: return "arena smaller than the footprint";
    case PM_EDEVICE: return "HIP call failed";
    case PM_ECAPACITY: return "particle capacity exhausted";
    case PM_ENUMERIC: return "NaN or Inf in the particle state";
    case PM_ESTATE: return "case has failed or the call does not apply";
  }
  return "unknown status";
}

size_t pm_case_footprint(const pm_case_params* p) {
  if (!valid(p)) return 0;
  return layout(p).total;
}

pm_status pm_init_case(const pm_case_params* p, void* arena, size_t bytes, void* stream, pm_case** out) {
  if (!out) return PM_EINVAL;
  *out = nullptr;
  if (!valid(p) || !arena) return PM_EINVAL;
  if ((reinterpret_cast<uintptr_t>(arena) & 255) != 0) return PM_EINVAL;
  const ArenaMap m = layout(p);
  if (bytes < m.total) return PM_ENOSPACE;
  pm_case* c = new (std::nothrow) pm_case();
  if (!c) return PM_EDEVICE;
  c->prm = *p;
  c->c = make_const(p);
  c->map = m;
  c->arena = reinterpret_cast<char*>(arena);
  c->bytes = bytes;
  c->warnings = warnings_of(p, c->c);
  fill_args<float>(c->af, c->c, c->arena, m);
  fill_args<double>(c->ad, c->c, c->arena, m);
  c->work_grid = work_grid_for(p, resident_step_blocks(p->fp64, p->n_cells, c->c.unroll, c->c.waves, false));
  c->step_grid = std::max(c->work_grid, slot_grid_for(p));
  c->mcc_grid = mcc_grid_for(
      p, c->c, mcc_per_lane(expected_candidates(p, c->c), resident_mcc_blocks(p->fp64, p->n_cells, false)));
  c->sort_grid = sort_grid_for(p);
  c->cap_stream = nullptr;
  c->graph = nullptr;
  c->exec = nullptr;
  c->has_graph = false;
  c->failed = PM_OK;
  c->since_sort = 0;
  const pm_status s = p->fp64 ? init_impl<double>(c, as_stream(stream)) : init_impl<float>(c, as_stream(stream));
  if (s != PM_OK) {
    delete c;
    return s;
  }
  *out = c;
  return PM_OK;
}

pm_status pm_step(pm_case* c, int64_t n_steps, void* stream) {
  if (!c || n_steps < 0) return PM_EINVAL;
  if (c->failed != PM_OK) return PM_ESTATE;
  return c->prm.fp64 ? run_steps<double>(c, n_steps, as_stream(stream))
                     : run_steps<float>(c, n_steps, as_stream(stream));
}

pm_status pm_step_rf_cycles(pm_case* c, int32_t n_cycles, void* stream) {
  if (!c || n_cycles < 0) return PM_EINVAL;
  if (c->failed != PM_OK) return PM_ESTATE;
  const pm_status s = c->prm.fp64 ? build_graph<double>(c) : build_graph<float>(c);
  if (s != PM_OK) return s;
  for (int32_t i = 0; i < n_cycles; ++i)
    if (hipGraphLaunch(c->exec, as_stream(stream)) != hipSuccess) return PM_EDEVICE;
  // a captured cycle ends with a sort (its sort interval divides N_t)
  if (n_cycles > 0 && cycle_sort_interval(c->prm.sort_interval, c->prm.steps_per_cycle) > 0) c->since_sort = 0;
  return PM_OK;
}

pm_status pm_sample_diagnostics(pm_case* c, pm_diagnostics* out, int32_t reset, void* stream) {
  if (!c || !out) return PM_EINVAL;
  if (c->failed != PM_OK) return PM_ESTATE;
  return c->prm.fp64 ? sample_impl<double>(c, out, reset, as_stream(stream))
                     : sample_impl<float>(c, out, reset, as_stream(stream));
}

pm_status pm_sample_phase(pm_case* c, int32_t bin, pm_phase_sample* out, void* stream) {
  if (!c || !out || bin < 0 || bin >= c->c.n_phase) return PM_EINVAL;
  if (c->failed != PM_OK) return PM_ESTATE;
  return c->prm.fp64 ? sample_phase_impl<double>(c, bin, out, as_stream(stream))
                     : sample_phase_impl<float>(c, bin, out, as_stream(stream));
}

pm_status pm_diag_sizes(const pm_case* c, int32_t* nodes, int32_t* n_ebins) {
  if (!c) return PM_EINVAL;
  if (nodes) *nodes = c->c.N + 1;
  if (n_ebins) *n_ebins = c->c.n_ebins;
  return PM_OK;
}

pm_status pm_get_particles(pm_case* c, int32_t species, pm_particles* out, void* stream) {
  if (!c || !out || (species != 0 && species != 1)) return PM_EINVAL;
  return c->prm.fp64 ? get_particles_impl<double>(c, species, out, as_stream(stream))
                     : get_particles_impl<float>(c, species, out, as_stream(stream));
}

pm_status pm_set_particles(pm_case* c, int32_t species, const pm_particles* in, void* stream) {
  if (!c || !in || (species != 0 && species != 1)) return PM_EINVAL;
  if (c->failed != PM_OK) return PM_ESTATE;
  if (in->n > 0 && (!in->xt || !in->ux || !in->uy || !in->uz || !in->id || !in->next)) return PM_EINVAL;
  return c->prm.fp64 ? set_particles_impl<double>(c, species, in, as_stream(stream))
                     : set_particles_impl<float>(c, species, in, as_stream(stream));
}

// ---------------------------------------------------------------- checkpoints
namespace {

constexpr uint64_t kCkptMagic = 0x3130545043434d50ull;   // "PMCCPT01"

struct CkptHeader {
  uint64_t magic;
  uint64_t header_bytes, arena_bytes, args_off, args_bytes;
  pm_case_params prm;          // sort_interval as saved; not compared
  int64_t live_atoms[2], live_step[2], since_sort;
  int32_t failed;
  int32_t pad;
};

// The parameters that fix a case's layout and its physics: all of them but the
// sort interval, which only changes the order of the slots.
bool same_case(const pm_case_params& a, const pm_case_params& b) {
  return a.gap_m == b.gap_m && a.n_cells == b.n_cells && a.steps_per_cycle == b.steps_per_cycle &&
         a.freq_hz == b.freq_hz && a.v0_volt == b.v0_volt && a.phase_rad == b.phase_rad && a.p_pa == b.p_pa &&
         a.t_gas_k == b.t_gas_k && a.n0_m3 == b.n0_m3 && a.np_e == b.np_e && a.np_i == b.np_i &&
         a.te_ev == b.te_ev && a.ti_ev == b.ti_ev && a.capacity_e == b.capacity_e &&
         a.capacity_i == b.capacity_i && a.ecap_e_ev == b.ecap_e_ev && a.ecap_i_ev == b.ecap_i_ev &&
         a.xs.sigma_el == b.xs.sigma_el && a.xs.eth_exc == b.xs.eth_exc && a.xs.sigma0_exc == b.xs.sigma0_exc &&
         a.xs.eth_ion == b.xs.eth_ion && a.xs.sigma0_ion == b.xs.sigma0_ion && a.xs.sigma_cx == b.xs.sigma_cx &&
         a.seed == b.seed && a.case_id == b.case_id && a.flags == b.flags && a.fp64 == b.fp64 &&
         a.v2_volt == b.v2_volt && a.phase2_rad == b.phase2_rad && a.cb_f_m2 == b.cb_f_m2 &&
         a.n_phase == b.n_phase && a.flux_profiles == b.flux_profiles;
}

}  // namespace

size_t pm_checkpoint_bytes(const pm_case* c) { return c ? sizeof(CkptHeader) + c->map.total : 0; }

pm_status pm_save_checkpoint(pm_case* c, void* host_buf, size_t bytes, void* stream) {
  if (!c || !host_buf || bytes < pm_checkpoint_bytes(c)) return PM_EINVAL;
  CkptHeader h{};
  h.magic = kCkptMagic;
  h.header_bytes = sizeof(CkptHeader);
  h.arena_bytes = c->map.total;
  h.args_off = c->map.args;
  h.args_bytes = std::max(sizeof(pm::KArgs<float>), sizeof(pm::KArgs<double>));
  h.prm = c->prm;
  for (int e = 0; e < 2; ++e) {
    h.live_atoms[e] = c->live_atoms[e];
    h.live_step[e] = c->live_step[e];
  }
  h.since_sort = c->since_sort;
  h.failed = (int32_t)c->failed;
  const hipStream_t st = as_stream(stream);
  PM_TRY(hipStreamSynchronize(st));
  char* out = static_cast<char*>(host_buf);
  PM_TRY(hipMemcpyAsync(out + sizeof(CkptHeader), c->arena, c->map.total, hipMemcpyDeviceToHost, st));
  PM_TRY(hipStreamSynchronize(st));
  std::memcpy(out, &h, sizeof(h));
  return PM_OK;
}

pm_status pm_load_checkpoint(pm_case* c, const void* host_buf, size_t bytes, void* stream) {
  if (!c || !host_buf || bytes < sizeof(CkptHeader)) return PM_EINVAL;
  CkptHeader h;
  std::memcpy(&h, host_buf, sizeof(h));
  const size_t args_bytes = std::max(sizeof(pm::KArgs<float>), sizeof(pm::KArgs<double>));
  if (h.magic != kCkptMagic || h.header_bytes != sizeof(CkptHeader) || h.arena_bytes != c->map.total ||
      h.args_off != c->map.args || h.args_bytes != args_bytes || bytes < sizeof(CkptHeader) + h.arena_bytes ||
      !same_case(h.prm, c->prm) || h.failed > 0 || h.failed < PM_ESTATE)
    return PM_EINVAL;
  const hipStream_t st = as_stream(stream);
  PM_TRY(hipStreamSynchronize(st));
  // everything but the kernel-argument block, which holds this arena's own addresses
  const char* in = static_cast<const char*>(host_buf) + sizeof(CkptHeader);
  const size_t tail = c->map.args + args_bytes;
  PM_TRY(hipMemcpyAsync(c->arena, in, c->map.args, hipMemcpyHostToDevice, st));
  if (c->map.total > tail)
    PM_TRY(hipMemcpyAsync(c->arena + tail, in + tail, c->map.total - tail, hipMemcpyHostToDevice, st));
  PM_TRY(hipStreamSynchronize(st));
  for (int e = 0; e < 2; ++e) {
    c->live_atoms[e] = h.live_atoms[e];
    c->live_step[e] = h.live_step[e];
  }
  c->since_sort = h.since_sort;
  c->failed = (pm_status)h.failed;
  return PM_OK;
}

pm_status pm_get_fields(pm_case* c, pm_fields* out, void* stream) {
  if (!c || !out) return PM_EINVAL;
  return c->prm.fp64 ? get_fields_impl<double>(c, out, as_stream(stream))
                     : get_fields_impl<float>(c, out, as_stream(stream));
}

pm_status pm_case_info(const pm_case* c, double* dx, double* dt, double* weight, double* nu_max, double* p_tot) {
  if (!c) return PM_EINVAL;
  if (dx) *dx = c->c.dx;
  if (dt) *dt = c->c.dt;
  if (weight) *weight = c->c.w;
  for (int s = 0; s < 2; ++s) {
    if (nu_max) nu_max[s] = c->c.nu_max[s];
    if (p_tot) p_tot[s] = c->c.has_coll ? -std::expm1(-c->c.nu_max[s] * c->c.dt) : 0.0;
  }
  return PM_OK;
}

pm_status pm_get_step_profile(pm_case* c, uint64_t* out, int64_t cap, int32_t* grid, void* stream) {
  if (!c || !grid) return PM_EINVAL;
  const int rows = std::max(c->step_grid, c->mcc_grid);
  *grid = rows;
  if (!out) return PM_OK;
  if (cap < 8 * (int64_t)rows) return PM_EINVAL;
  PM_TRY(hipStreamSynchronize(as_stream(stream)));
  PM_TRY(hipMemcpy(out, c->arena + c->map.prof, (size_t)8 * rows * 8, hipMemcpyDeviceToHost));
  return PM_OK;
}

pm_status pm_get_launch_shape(const pm_case* c, pm_launch_shape* out) {
  if (!c || !out) return PM_EINVAL;
  out->unroll = c->c.unroll;
  out->waves = c->c.waves;
  out->work_groups = c->work_grid;
  out->deposit_mode = c->c.dep_mode;
  out->sort_interval = c->prm.sort_interval;
  out->lanes = 1;
  return PM_OK;
}

pm_status pm_set_launch_shape(pm_case* c, const pm_launch_shape* sh, void* stream) {
  if (!c || !valid_shape(sh)) return PM_EINVAL;
  if (c->failed != PM_OK) return PM_ESTATE;
  const hipStream_t st = as_stream(stream);
  PM_TRY(hipStreamSynchronize(st));      // no step of the old shape may still read the arguments
  c->c.unroll = sh->unroll;
  c->c.waves = sh->waves;
  c->c.dep_mode = sh->deposit_mode;
  c->prm.sort_interval = sh->sort_interval;
  c->c.sort_interval = sh->sort_interval;
  const int most = work_grid_for(&c->prm);
  c->work_grid = sh->work_groups > 0
      ? std::min(sh->work_groups, most)
      : work_grid_for(&c->prm, resident_step_blocks(c->prm.fp64, c->c.N, sh->unroll, sh->waves, false));
  c->step_grid = std::max(c->work_grid, slot_grid_for(&c->prm));
  fill_args<float>(c->af, c->c, c->arena, c->map);
  fill_args<double>(c->ad, c->c, c->arena, c->map);
  if (c->prm.fp64) PM_TRY(hipMemcpyAsync(c->arena + c->map.args, &c->ad, sizeof(c->ad), hipMemcpyHostToDevice, st));
  else PM_TRY(hipMemcpyAsync(c->arena + c->map.args, &c->af, sizeof(c->af), hipMemcpyHostToDevice, st));
  PM_TRY(hipStreamSynchronize(st));
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->exec = nullptr;
  c->graph = nullptr;
  c->has_graph = false;
  return PM_OK;
}

void pm_destroy_case(pm_case* c) {
  if (!c) return;
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

// ---------------------------------------------------------------- sputtering
pm_status pm_inject_sputtered(pm_case* c, const pm_sputter_params* sp, pm_tp_source* out, void* stream) {
  if (!c || !sp || !out) return PM_EINVAL;
  if (c->failed != PM_OK) return PM_ESTATE;
  if (sp->n_table < 0 || (sp->n_table > 0 && (!sp->table_e_ev || !sp->table_y))) return PM_EINVAL;
  if (sp->n_table == 0 && !(sp->yield_const >= 0)) return PM_EINVAL;
  if (!(sp->u_s_ev > 0) || !(sp->e_cut_ev > 0) || sp->n_atoms < 0) return PM_EINVAL;
  if (sp->electrode != 0 && sp->electrode != 1) return PM_EINVAL;
  if (sp->since_last != 0 && sp->since_last != 1) return PM_EINVAL;
  for (int k = 0; k < sp->n_table; ++k) {
    if (!(sp->table_y[k] >= 0)) return PM_EINVAL;
    if (k && !(sp->table_e_ev[k] > sp->table_e_ev[k - 1])) return PM_EINVAL;
  }
  hipStream_t st = as_stream(stream);
  const int nb = c->c.n_ebins;
  std::vector<double> y(nb);
  for (int b = 0; b < nb; ++b) y[b] = yield_at(sp, (double)b + 0.5);
  double* ybin = reinterpret_cast<double*>(c->arena + c->map.ybin);
  uint64_t* yo = reinterpret_cast<uint64_t*>(c->arena + c->map.yield_out);
  const uint64_t* iedf = reinterpret_cast<const uint64_t*>(c->arena + c->map.iedf) + (size_t)sp->electrode * nb;
  PM_TRY(hipMemcpyAsync(ybin, y.data(), nb * 8, hipMemcpyHostToDevice, st));
  PM_TRY(hipMemsetAsync(yo, 0, 4 * 8, st));
  const int e = sp->electrode;
  uint64_t* taken = sp->since_last ? reinterpret_cast<uint64_t*>(c->arena + c->map.iedf_taken) + (size_t)e * nb
                                   : nullptr;
  PM_TRY(pm::launch_yield(iedf, ybin, nb, sp->seed, sp->job_id, e, taken, yo, st));
  uint64_t h[4];
  PM_TRY(hipMemcpyAsync(h, yo, sizeof(h), hipMemcpyDeviceToHost, st));
  pm::Ctrl ctl;
  pm_status rs = read_ctrl(c, &ctl, st);
  if (rs != PM_OK) return rs;
  std::memset(out, 0, sizeof(*out));
  out->n_emitted = (int64_t)h[0];
  out->n_impacts = (int64_t)h[1];
  out->n_atoms = sp->n_atoms > 0 ? sp->n_atoms : out->n_emitted;
  if (sp->since_last) {
    // atom ids continue where the window's previous live call stopped, so the
    // calls' atoms are the atoms of one whole-window source
    const int64_t steps = ctl.step - c->live_step[e];
    out->first_atom = c->live_atoms[e];
    out->flux_m2s = steps > 0 ? (double)h[0] * c->c.w / ((double)steps * c->c.dt) : 0.0;
    c->live_atoms[e] += out->n_emitted;
    c->live_step[e] = ctl.step;
  } else {
    out->first_atom = 0;
    out->flux_m2s = ctl.avg_steps > 0 ? (double)h[0] * c->c.w / ((double)ctl.avg_steps * c->c.dt) : 0.0;
  }
  out->u_s_ev = sp->u_s_ev;
  out->e_cut_ev = sp->e_cut_ev;
  out->seed = sp->seed;
  out->job_id = sp->job_id;
  out->electrode = sp->electrode;
  return PM_OK;
}

size_t pm_tp_footprint(const pm_tp_params* tp) {
  if (!tp || tp->n_ebins < 1 || tp->n_tbins < 1 || tp->n_xbins < 0 || tp->n_xbins > kMaxTpXBins) return 0;
  return tp_layout(tp).total;
}

pm_status pm_run_test_particles(const pm_tp_params* tp, const pm_tp_source* src, void* arena, size_t bytes,
                                void* stream, pm_tp_result* out) {
  if (!tp || !src || !out || !arena) return PM_EINVAL;
  if ((reinterpret_cast<uintptr_t>(arena) & 255) != 0) return PM_EINVAL;
  const pm_status v = tp_validate(tp, src);
  if (v != PM_OK) return v;
  if (bytes < pm_tp_footprint(tp)) return PM_ENOSPACE;
  return tp_run(tp, src, reinterpret_cast<char*>(arena), as_stream(stream), out);
}

pm_status pm_run_test_particles_static(const pm_tp_params* tp, const pm_tp_source* src, void* stream,
                                       pm_tp_result* out) {
  if (!tp || !src || !out) return PM_EINVAL;
  const pm_status v = tp_validate(tp, src);
  if (v != PM_OK) return v;
  if (pm_tp_footprint(tp) > pm::kTpScratchBytes) return PM_ENOSPACE;
  void* base = nullptr;
  PM_TRY(pm::tp_scratch(&base));
  return tp_run(tp, src, reinterpret_cast<char*>(base), as_stream(stream), out);
}

}  // extern "C"

// ------------------------------------------------------------------ batches
// Many independent cases (a parameter sweep) advanced by the same launches, one
// push and one collision launch per time step and lane.  The working workgroups of every case come first in the grid, case by
// case, so the serial part of a case (its field solve) overlaps the particle
// work of the cases after it; the workgroups that hold slots only when a case
// outgrows its share follow.  Device tables in a caller-provided arena:
//   [KArgs of each case][step, collision and sort workgroups per case]
//   [step, collision and sort work lists],  work entry = case << 16 | local
//   workgroup, with room for the largest step grid of every case.
// The cases of a batch may run in up to four lanes, each on its own stream:
// while one lane's collision kernel (latency-bound) runs, another lane's push
// kernel (bandwidth-bound) fills the GPU.  A lane's work lists are a segment of
// the batch's lists.
struct BatchLane {
  int step_off, step_n, mcc_off, mcc_n, sort_off, sort_n, maxN;
  hipStream_t st;          // nullptr for a single lane (the caller's stream)
  hipEvent_t done;
};

struct pm_batch {
  std::vector<pm_case*> cases;
  bool fp64;
  int maxN, steps_per_cycle;
  pm_launch_shape shape;   // work_groups as requested (0: one resident wave)
  int work_total;          // working workgroups in effect
  int step_grid, mcc_grid, sort_grid;
  std::vector<BatchLane> lanes;
  hipEvent_t fork;
  char* arena;
  void* args;
  uint32_t *step_nblk, *mcc_nblk, *sort_nblk, *step_work, *mcc_work, *sort_work;
  hipStream_t cap_stream;
  hipGraph_t graph;
  hipGraphExec_t exec;
  int64_t since_sort;      // steps of plain launches since the last sort
  // A slotted batch (pm_batch_create_slots): cases[i] is null for an empty
  // slot; every lane's work lists have a fixed length (idle entries padding
  // them), so a captured graph stays valid while cases come and go.
  bool slotted;
  int list_cap;            // entries of each work list (the table's room)
  int grid_step, grid_mcc, grid_sort;   // fixed per-lane list lengths (slotted)
};

namespace {

struct BatchLayout {
  size_t args, step_nb, mcc_nb, sort_nb, step_work, mcc_work, sort_work, total;
};

// Upper bound of the workgroups of one launch resident on a device: at most
// eight 256-thread workgroups fit on a compute unit.
int max_resident_blocks() {
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
  return 8 * cus;
}

// Tables of a slotted batch: n_slots case entries and work lists of a fixed
// room (one resident wave of each kernel at most).
void slots_layout(int32_t n, bool fp64, int list_cap, BatchLayout* L) {
  Layout A;
  L->args = A.take((size_t)n * (fp64 ? sizeof(pm::KArgs<double>) : sizeof(pm::KArgs<float>)));
  L->step_nb = A.take((size_t)n * 4);
  L->mcc_nb = A.take((size_t)n * 4);
  L->sort_nb = A.take((size_t)n * 4);
  L->step_work = A.take((size_t)list_cap * 4);
  L->mcc_work = A.take((size_t)list_cap * 4);
  L->sort_work = A.take((size_t)list_cap * 4);
  L->total = A.off;
}

pm_status batch_layout(pm_case* const* cases, int32_t n, BatchLayout* L) {
  if (!cases || n < 1 || n > 65535) return PM_EINVAL;
  std::vector<pm_case*> seen(cases, cases + n);
  std::sort(seen.begin(), seen.end());
  if (!seen.front() || std::adjacent_find(seen.begin(), seen.end()) != seen.end()) return PM_EINVAL;
  const bool fp64 = cases[0]->prm.fp64 != 0;
  int64_t steps = 0, mccs = 0, sorts = 0;
  for (int32_t i = 0; i < n; ++i) {
    const pm_case* c = cases[i];
    if (c->failed != PM_OK) return PM_ESTATE;
    if ((c->prm.fp64 != 0) != fp64) return PM_EINVAL;
    if (c->c.flux) return PM_EINVAL;    // flux samples are taken by the single-case steps only
    steps += max_step_grid_for(&c->prm);
    mccs += max_step_grid_for(&c->prm);
    sorts += c->sort_grid;
  }
  if (steps > INT32_MAX || mccs > INT32_MAX || sorts > INT32_MAX) return PM_EINVAL;
  Layout A;
  L->args = A.take((size_t)n * (fp64 ? sizeof(pm::KArgs<double>) : sizeof(pm::KArgs<float>)));
  L->step_nb = A.take((size_t)n * 4);
  L->mcc_nb = A.take((size_t)n * 4);
  L->sort_nb = A.take((size_t)n * 4);
  L->step_work = A.take((size_t)steps * 4);
  L->mcc_work = A.take((size_t)mccs * 4);
  L->sort_work = A.take((size_t)sorts * 4);
  L->total = A.off;
  return PM_OK;
}

// Share the working workgroups out in proportion to the cases' initial
// particles and write the tables for the batch's shape.  Synchronises.
// Share total workgroups among the cases of one lane in proportion to weight,
// each share rounded up from (total - n), so that they sum to at most total
// and no case gets less than its part; each share at least 1 and at most cap[i].
std::vector<int64_t> shares(const std::vector<double>& weight, int64_t total, const std::vector<int64_t>& cap) {
  const size_t n = weight.size();
  double wsum = 0.0;
  for (double w : weight) wsum += w;
  const double share = (double)std::max<int64_t>(total - (int64_t)n, 1);
  std::vector<int64_t> out(n);
  for (size_t i = 0; i < n; ++i) {
    int64_t w = wsum > 0.0 ? (int64_t)std::ceil(share * weight[i] / wsum) : 1;
    out[i] = std::max<int64_t>(1, std::min<int64_t>(w, cap[i]));
  }
  return out;
}

// Write the batch's tables for its shape and members.  An unslotted batch
// shares one resident wave of push workgroups among all its cases in
// proportion to their initial particles and groups the cases into lanes by
// size; a slotted batch puts slot i in lane i mod lanes, gives each lane a
// fixed part of each kernel's resident wave and pads its lists with idle
// entries.  Synchronises hip_stream.
// Tiles t in [lo, hi) with t = q (mod m): the share of workgroup q of m in a
// strided walk over tiles lo..hi-1.
int64_t strided_count(int64_t lo, int64_t hi, int64_t q, int64_t m) {
  if (hi <= lo || m < 1) return 0;
  const int64_t first = lo + (((q - lo) % m) + m) % m;
  return first < hi ? (hi - 1 - first) / m + 1 : 0;
}

template <typename R>
pm_status write_tables(pm_batch* b, hipStream_t st) {
  const int n = (int)b->cases.size();
  const int nl = std::max(1, std::min({b->shape.lanes, b->slotted ? 4 : n, 4}));
  // lanes and their members (present cases only)
  std::vector<std::vector<int>> members(nl);
  if (b->slotted) {
    for (int i = 0; i < n; ++i)
      if (b->cases[i]) members[i % nl].push_back(i);
  } else {
    // the largest cases first, each to the lane with the fewest particles
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return b->cases[x]->prm.np_e + b->cases[x]->prm.np_i > b->cases[y]->prm.np_e + b->cases[y]->prm.np_i;
    });
    std::vector<int64_t> load(nl, 0);
    for (int i : order) {
      const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      members[g].push_back(i);
      load[g] += b->cases[i]->prm.np_e + b->cases[i]->prm.np_i;
    }
    for (auto& m : members) std::sort(m.begin(), m.end());
  }
  const int64_t step_total = b->shape.work_groups > 0
      ? b->shape.work_groups
      : resident_step_blocks(b->fp64, b->maxN, b->shape.unroll, b->shape.waves, true);
  const int64_t resident_mcc = resident_mcc_blocks(b->fp64, b->maxN, true);
  // a slotted batch's lists have a fixed length per lane
  const int64_t lane_step = std::min<int64_t>(step_total / nl, b->list_cap / nl);
  const int64_t lane_mcc = std::min<int64_t>(resident_mcc / nl, b->list_cap / nl);
  const int64_t lane_sort = std::min<int64_t>(resident_mcc / nl, b->list_cap / nl);
  std::vector<pm::KArgs<R>> args(n);
  std::vector<uint32_t> nb(n, 0), nm(n, 0), ns(n, 0), sw, mw, rw;
  int64_t work_total = 0;
  std::vector<BatchLane> lanes(nl);
  for (int g = 0; g < nl; ++g) {
    const std::vector<int>& mem = members[g];
    const int m = (int)mem.size();
    // push: working workgroups by initial particles
    std::vector<double> wt(m);
    std::vector<int64_t> cap(m), scap(m, 1 << 15);
    int64_t t0_sum = 0;
    for (int k = 0; k < m; ++k) {
      const pm_case* c = b->cases[mem[k]];
      wt[k] = (double)(c->prm.np_e + c->prm.np_i);
      cap[k] = work_grid_for(&c->prm);
      t0_sum += c->prm.np_e + c->prm.np_i;
    }
    int64_t lane_t0 = 0;
    for (const pm_case* c : b->cases)
      if (c) lane_t0 += c->prm.np_e + c->prm.np_i;
    // an unslotted batch shares one wave among all its cases; a slotted lane its part
    const std::vector<int64_t> w = b->slotted
        ? shares(wt, lane_step, cap)
        : shares(wt, std::max<int64_t>(m, (int64_t)std::llround((double)step_total * (double)t0_sum /
                                                                 (double)std::max<int64_t>(lane_t0, 1))), cap);
    // collisions: raise the load per lane until the rounded grids fit the lane's part of a resident wave
    double cand = 0.0;
    for (int i : mem) cand += expected_candidates(&b->cases[i]->prm, b->cases[i]->c);
    const int64_t mcc_budget = b->slotted ? lane_mcc
                                          : std::max<int64_t>(1, (int64_t)std::llround((double)resident_mcc *
                                                                                        (double)t0_sum /
                                                                                        (double)std::max<int64_t>(lane_t0, 1)));
    double per_lane = mcc_per_lane(cand, mcc_budget);
    for (int it = 0; it < 8 && per_lane < 4.0; ++it) {
      int64_t sum = 0;
      for (int i : mem) sum += mcc_grid_for(&b->cases[i]->prm, b->cases[i]->c, per_lane);
      if (sum <= mcc_budget) break;
      per_lane = std::min(4.0, per_lane * (1.0 + (double)(sum - mcc_budget + m) / (double)mcc_budget));
    }
    // sort: slotted lanes share a fixed part by capacity; unslotted cases keep their own grids
    std::vector<double> cw(m);
    for (int k = 0; k < m; ++k) cw[k] = (double)(b->cases[mem[k]]->prm.capacity_e + b->cases[mem[k]]->prm.capacity_i);
    const std::vector<int64_t> sg = b->slotted ? shares(cw, lane_sort, scap) : std::vector<int64_t>();
    BatchLane& L = lanes[g];
    L.maxN = b->slotted ? b->maxN : 0;
    L.step_off = (int)sw.size();
    L.mcc_off = (int)mw.size();
    L.sort_off = (int)rw.size();
    for (int k = 0; k < m; ++k) {
      const int i = mem[k];
      const pm_case* c = b->cases[i];
      L.maxN = std::max(L.maxN, c->c.N);
      const int64_t ww = w[k];
      const int64_t gg = b->slotted ? ww : std::max<int64_t>(ww, slot_grid_for(&c->prm));
      nb[i] = (uint32_t)gg | (uint32_t)ww << 16;
      nm[i] = (uint32_t)mcc_grid_for(&c->prm, c->c, per_lane);
      if (b->slotted) nm[i] = (uint32_t)std::min<int64_t>(nm[i], lane_mcc);
      ns[i] = (uint32_t)(b->slotted ? sg[k] : c->sort_grid);
      work_total += ww;
      args[i] = args_of<R>(const_cast<pm_case*>(c));
      args[i].c.dep_mode = b->shape.deposit_mode;
      args[i].c.unroll = b->shape.unroll;
      args[i].c.waves = b->shape.waves;
    }
    // the lane's working workgroups, those with the most tiles first (the
    // hardware starts workgroups in grid order, so the short ones fill the end
    // of the launch); tiles counted from the initial particles, as each
    // workgroup's strided share of its case's electron and ion tiles
    {
      const int64_t tile = (int64_t)256 * b->shape.unroll;
      std::vector<std::pair<int64_t, uint32_t>> ws;
      for (int i : mem) {
        const pm_case* c = b->cases[i];
        const int64_t te = (c->prm.np_e + tile - 1) / tile, ti = (c->prm.np_i + tile - 1) / tile;
        const int64_t nw = nb[i] >> 16;
        for (int64_t q = 0; q < nw; ++q)
          ws.emplace_back(strided_count(0, te, q, nw) + strided_count(te, te + ti, q, nw),
                          ((uint32_t)i << 16) | (uint32_t)q);
      }
      std::stable_sort(ws.begin(), ws.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
      for (const auto& e : ws) sw.push_back(e.second);
    }
    // workgroups that only rotate the charge buffers when a case outgrows its working share
    for (int i : mem)
      for (uint32_t q = nb[i] >> 16; q < (nb[i] & 0xFFFFu); ++q) sw.push_back(((uint32_t)i << 16) | q);
    for (int i : mem)
      for (uint32_t q = 0; q < nm[i]; ++q) mw.push_back(((uint32_t)i << 16) | q);
    for (int i : mem)
      for (uint32_t q = 0; q < ns[i]; ++q) rw.push_back(((uint32_t)i << 16) | q);
    if (b->slotted) {
      // fixed lengths: idle entries after the lane's own
      if ((int64_t)sw.size() - L.step_off > lane_step || (int64_t)mw.size() - L.mcc_off > lane_mcc ||
          (int64_t)rw.size() - L.sort_off > lane_sort)
        return PM_EINVAL;
      sw.resize((size_t)(L.step_off + lane_step), pm::kIdleWork);
      mw.resize((size_t)(L.mcc_off + lane_mcc), pm::kIdleWork);
      rw.resize((size_t)(L.sort_off + lane_sort), pm::kIdleWork);
    }
    L.step_n = (int)sw.size() - L.step_off;
    L.mcc_n = (int)mw.size() - L.mcc_off;
    L.sort_n = (int)rw.size() - L.sort_off;
  }
  PM_TRY(hipStreamSynchronize(st));      // no launch of the old tables may still read them
  // lane streams and events (the single lane runs on the caller's stream)
  for (size_t g = 0; g < lanes.size(); ++g) {
    if (g < b->lanes.size()) {
      lanes[g].st = b->lanes[g].st;
      lanes[g].done = b->lanes[g].done;
    } else {
      lanes[g].st = nullptr;
      lanes[g].done = nullptr;
    }
    if (nl > 1 && !lanes[g].st) PM_TRY(hipStreamCreateWithFlags(&lanes[g].st, hipStreamNonBlocking));
    if (nl > 1 && !lanes[g].done) PM_TRY(hipEventCreateWithFlags(&lanes[g].done, hipEventDisableTiming));
  }
  for (size_t g = lanes.size(); g < b->lanes.size(); ++g) {
    if (b->lanes[g].st) (void)hipStreamDestroy(b->lanes[g].st);
    if (b->lanes[g].done) (void)hipEventDestroy(b->lanes[g].done);
  }
  // a slotted batch keeps its graph while only its members change (same lanes and lengths)
  bool same_shape = b->slotted && b->exec && b->lanes.size() == lanes.size();
  for (size_t g = 0; same_shape && g < lanes.size(); ++g)
    same_shape = b->lanes[g].step_n == lanes[g].step_n && b->lanes[g].mcc_n == lanes[g].mcc_n &&
                 b->lanes[g].sort_n == lanes[g].sort_n && b->lanes[g].maxN == lanes[g].maxN;
  b->lanes = lanes;
  if (nl > 1 && !b->fork) PM_TRY(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
  for (int i = 0; i < n; ++i)
    if (b->cases[i])
      PM_TRY(hipMemcpyAsync(reinterpret_cast<pm::KArgs<R>*>(b->args) + i, &args[i], sizeof(pm::KArgs<R>),
                            hipMemcpyHostToDevice, st));
  PM_TRY(hipMemcpyAsync(b->step_nblk, nb.data(), nb.size() * 4, hipMemcpyHostToDevice, st));
  PM_TRY(hipMemcpyAsync(b->mcc_nblk, nm.data(), nm.size() * 4, hipMemcpyHostToDevice, st));
  PM_TRY(hipMemcpyAsync(b->sort_nblk, ns.data(), ns.size() * 4, hipMemcpyHostToDevice, st));
  if (!sw.empty()) PM_TRY(hipMemcpyAsync(b->step_work, sw.data(), sw.size() * 4, hipMemcpyHostToDevice, st));
  if (!mw.empty()) PM_TRY(hipMemcpyAsync(b->mcc_work, mw.data(), mw.size() * 4, hipMemcpyHostToDevice, st));
  if (!rw.empty()) PM_TRY(hipMemcpyAsync(b->sort_work, rw.data(), rw.size() * 4, hipMemcpyHostToDevice, st));
  PM_TRY(hipStreamSynchronize(st));
  b->work_total = (int)work_total;
  b->step_grid = (int)sw.size();
  b->mcc_grid = (int)mw.size();
  b->sort_grid = (int)rw.size();
  if (!same_shape) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
  }
  return PM_OK;
}

// Events around every kernel launch of a measured call (pm_*_time_kernels):
// ev[0..1] bracket the push launch, ev[2..3] the collision launch.
struct KernelTimer {
  hipEvent_t ev[4];
  double push_ms = 0.0, mcc_ms = 0.0;
  int64_t launches = 0;
};

pm_status timer_read(KernelTimer* t) {
  PM_TRY(hipEventSynchronize(t->ev[3]));
  float a = 0.f, b = 0.f;
  PM_TRY(hipEventElapsedTime(&a, t->ev[0], t->ev[1]));
  PM_TRY(hipEventElapsedTime(&b, t->ev[2], t->ev[3]));
  t->push_ms += a;
  t->mcc_ms += b;
  t->launches += 1;
  return PM_OK;
}

// n steps of one lane.  sorts[i] says whether step i sorts (the batch's cadence,
// the same for every lane).
template <typename R>
pm_status lane_steps(pm_batch* b, const BatchLane& L, int64_t n, const std::vector<char>& sorts, hipStream_t st,
                     KernelTimer* tm = nullptr) {
  const auto* T = reinterpret_cast<const pm::KArgs<R>*>(b->args);
  for (int64_t i = 0; i < n; ++i) {
    const int sort = sorts[(size_t)i];
    if (tm) PM_TRY(hipEventRecord(tm->ev[0], st));
    PM_TRY(pm::launch_step_batch<R>(T, b->step_work + L.step_off, b->step_nblk, L.step_n, L.maxN,
                                    b->shape.unroll, b->shape.waves, sort, st));
    if (tm) PM_TRY(hipEventRecord(tm->ev[1], st));
    if (tm) PM_TRY(hipEventRecord(tm->ev[2], st));
    PM_TRY(pm::launch_mcc_batch<R>(T, b->mcc_work + L.mcc_off, b->mcc_nblk, L.mcc_n, L.maxN, sort, st));
    if (tm) PM_TRY(hipEventRecord(tm->ev[3], st));
    if (tm) {
      const pm_status ts = timer_read(tm);
      if (ts != PM_OK) return ts;
    }
    if (sort) PM_TRY(pm::launch_sort_batch<R>(T, b->sort_work + L.sort_off, b->sort_nblk, L.sort_n, L.maxN, st));
  }
  return PM_OK;
}

// n steps of every lane: forked from st and joined back into it.  The lanes
// run independently, so one lane's latency-bound collision kernel can overlap
// another lane's bandwidth-bound push.  (Making the lanes' pushes take turns
// through cross-stream events was slower: each wait added latency to the
// chain.)
bool batch_empty(const pm_batch* b) {
  for (const pm_case* c : b->cases)
    if (c) return false;
  return true;
}

// The sorting schedule of n steps: by the batch's running count, or at the
// fixed places of a captured RF cycle.
std::vector<char> batch_sorts(pm_batch* b, int64_t n, bool captured) {
  std::vector<char> v((size_t)n, 0);
  const int K = b->shape.sort_interval;
  const int Kc = cycle_sort_interval(K, b->steps_per_cycle);
  for (int64_t i = 0; i < n; ++i)
    v[(size_t)i] = captured ? (Kc > 0 && (i + 1) % Kc == 0) : sort_due(&b->since_sort, K);
  return v;
}

template <typename R>
pm_status batch_steps(pm_batch* b, int64_t n, hipStream_t st, bool captured = false) {
  const std::vector<char> sorts = batch_sorts(b, n, captured);
  if (!captured && batch_empty(b)) return PM_OK;
  if (b->lanes.size() == 1) return lane_steps<R>(b, b->lanes[0], n, sorts, st);
  PM_TRY(hipEventRecord(b->fork, st));
  for (const BatchLane& L : b->lanes) {
    PM_TRY(hipStreamWaitEvent(L.st, b->fork, 0));
    const pm_status s = lane_steps<R>(b, L, n, sorts, L.st);
    if (s != PM_OK) return s;
    PM_TRY(hipEventRecord(L.done, L.st));
  }
  for (const BatchLane& L : b->lanes) PM_TRY(hipStreamWaitEvent(st, L.done, 0));
  return PM_OK;
}

bool batch_ok(const pm_batch* b) {
  for (const pm_case* c : b->cases)
    if (c && c->failed != PM_OK) return false;
  return true;
}

}  // namespace

extern "C" {

size_t pm_batch_footprint(pm_case* const* cases, int32_t n_cases) {
  BatchLayout L;
  return batch_layout(cases, n_cases, &L) == PM_OK ? L.total : 0;
}

pm_status pm_batch_create(pm_case* const* cases, int32_t n_cases, void* arena, size_t bytes, void* stream,
                          pm_batch** out) {
  if (!out) return PM_EINVAL;
  *out = nullptr;
  BatchLayout L;
  const pm_status ls = batch_layout(cases, n_cases, &L);
  if (ls != PM_OK) return ls;
  if (!arena || (reinterpret_cast<uintptr_t>(arena) & 255) != 0) return PM_EINVAL;
  if (bytes < L.total) return PM_ENOSPACE;
  pm_batch* b = new (std::nothrow) pm_batch();
  if (!b) return PM_EDEVICE;
  b->cases.assign(cases, cases + n_cases);
  b->fp64 = cases[0]->prm.fp64 != 0;
  b->maxN = 0;
  b->steps_per_cycle = cases[0]->prm.steps_per_cycle;
  for (const pm_case* c : b->cases) {
    b->maxN = std::max(b->maxN, c->c.N);
    if (c->prm.steps_per_cycle != b->steps_per_cycle) b->steps_per_cycle = 0;
  }
  b->shape.unroll = 8;
  b->shape.waves = 0;
  b->shape.work_groups = 0;
  b->shape.deposit_mode = 1;
  b->shape.sort_interval = cases[0]->prm.sort_interval;
  b->shape.lanes = 1;
  b->fork = nullptr;
  b->arena = reinterpret_cast<char*>(arena);
  b->args = b->arena + L.args;
  b->step_nblk = reinterpret_cast<uint32_t*>(b->arena + L.step_nb);
  b->mcc_nblk = reinterpret_cast<uint32_t*>(b->arena + L.mcc_nb);
  b->sort_nblk = reinterpret_cast<uint32_t*>(b->arena + L.sort_nb);
  b->step_work = reinterpret_cast<uint32_t*>(b->arena + L.step_work);
  b->mcc_work = reinterpret_cast<uint32_t*>(b->arena + L.mcc_work);
  b->sort_work = reinterpret_cast<uint32_t*>(b->arena + L.sort_work);
  b->cap_stream = nullptr;
  b->graph = nullptr;
  b->exec = nullptr;
  b->since_sort = 0;
  b->slotted = false;
  b->list_cap = INT32_MAX;
  b->grid_step = b->grid_mcc = b->grid_sort = 0;
  const pm_status s = b->fp64 ? write_tables<double>(b, as_stream(stream)) : write_tables<float>(b, as_stream(stream));
  if (s != PM_OK) {
    delete b;
    return s;
  }
  *out = b;
  return PM_OK;
}

size_t pm_batch_slots_footprint(int32_t n_slots, int32_t fp64) {
  if (n_slots < 1 || n_slots > 65535 || (fp64 != 0 && fp64 != 1)) return 0;
  BatchLayout L;
  slots_layout(n_slots, fp64 != 0, max_resident_blocks(), &L);
  return L.total;
}

pm_status pm_batch_create_slots(int32_t n_slots, int32_t fp64, int32_t steps_per_cycle, int32_t max_cells,
                                void* arena, size_t bytes, void* stream, pm_batch** out) {
  if (!out) return PM_EINVAL;
  *out = nullptr;
  if (n_slots < 1 || n_slots > 65535 || (fp64 != 0 && fp64 != 1) || steps_per_cycle < 1 || max_cells < 1 ||
      max_cells > pm::kMaxCells)
    return PM_EINVAL;
  if (!arena || (reinterpret_cast<uintptr_t>(arena) & 255) != 0) return PM_EINVAL;
  BatchLayout L;
  const int cap = max_resident_blocks();
  slots_layout(n_slots, fp64 != 0, cap, &L);
  if (bytes < L.total) return PM_ENOSPACE;
  pm_batch* b = new (std::nothrow) pm_batch();
  if (!b) return PM_EDEVICE;
  b->cases.assign((size_t)n_slots, nullptr);
  b->fp64 = fp64 != 0;
  b->maxN = max_cells;
  b->steps_per_cycle = steps_per_cycle;
  b->shape.unroll = 8;
  b->shape.waves = 0;
  b->shape.work_groups = 0;
  b->shape.deposit_mode = 1;
  b->shape.sort_interval = 50;
  b->shape.lanes = 1;
  b->fork = nullptr;
  b->arena = reinterpret_cast<char*>(arena);
  b->args = b->arena + L.args;
  b->step_nblk = reinterpret_cast<uint32_t*>(b->arena + L.step_nb);
  b->mcc_nblk = reinterpret_cast<uint32_t*>(b->arena + L.mcc_nb);
  b->sort_nblk = reinterpret_cast<uint32_t*>(b->arena + L.sort_nb);
  b->step_work = reinterpret_cast<uint32_t*>(b->arena + L.step_work);
  b->mcc_work = reinterpret_cast<uint32_t*>(b->arena + L.mcc_work);
  b->sort_work = reinterpret_cast<uint32_t*>(b->arena + L.sort_work);
  b->cap_stream = nullptr;
  b->graph = nullptr;
  b->exec = nullptr;
  b->since_sort = 0;
  b->slotted = true;
  b->list_cap = cap;
  const pm_status s = b->fp64 ? write_tables<double>(b, as_stream(stream)) : write_tables<float>(b, as_stream(stream));
  if (s != PM_OK) {
    delete b;
    return s;
  }
  *out = b;
  return PM_OK;
}

pm_status pm_batch_set_slot(pm_batch* b, int32_t slot, pm_case* c, void* stream) {
  if (!b || !b->slotted || slot < 0 || slot >= (int32_t)b->cases.size()) return PM_EINVAL;
  if (c) {
    if (c->failed != PM_OK) return PM_ESTATE;
    if ((c->prm.fp64 != 0) != b->fp64 || c->prm.steps_per_cycle != b->steps_per_cycle || c->c.N > b->maxN ||
        c->c.flux)
      return PM_EINVAL;
    for (size_t i = 0; i < b->cases.size(); ++i)
      if (b->cases[i] == c && (int32_t)i != slot) return PM_EINVAL;
  }
  pm_case* old = b->cases[(size_t)slot];
  b->cases[(size_t)slot] = c;
  const pm_status s = b->fp64 ? write_tables<double>(b, as_stream(stream)) : write_tables<float>(b, as_stream(stream));
  if (s != PM_OK) b->cases[(size_t)slot] = old;
  return s;
}

pm_status pm_batch_get_launch_shape(const pm_batch* b, pm_launch_shape* out) {
  if (!b || !out) return PM_EINVAL;
  *out = b->shape;
  out->work_groups = b->work_total;
  return PM_OK;
}

pm_status pm_batch_set_launch_shape(pm_batch* b, const pm_launch_shape* sh, void* stream) {
  if (!b || !valid_shape(sh)) return PM_EINVAL;
  if (!batch_ok(b)) return PM_ESTATE;
  b->shape = *sh;
  return b->fp64 ? write_tables<double>(b, as_stream(stream)) : write_tables<float>(b, as_stream(stream));
}

pm_status pm_batch_step(pm_batch* b, int64_t n_steps, void* stream) {
  if (!b || n_steps < 0) return PM_EINVAL;
  if (!batch_ok(b)) return PM_ESTATE;
  return b->fp64 ? batch_steps<double>(b, n_steps, as_stream(stream))
                 : batch_steps<float>(b, n_steps, as_stream(stream));
}

pm_status pm_batch_step_rf_cycles(pm_batch* b, int32_t n_cycles, void* stream) {
  if (!b || n_cycles < 0 || b->steps_per_cycle < 1) return PM_EINVAL;
  if (!batch_ok(b)) return PM_ESTATE;
  if (!b->exec) {
    if (!b->cap_stream) PM_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    PM_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    const pm_status s = b->fp64 ? batch_steps<double>(b, b->steps_per_cycle, b->cap_stream, true)
                                : batch_steps<float>(b, b->steps_per_cycle, b->cap_stream, true);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (s != PM_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return PM_EDEVICE;
    }
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
      b->exec = nullptr;
      (void)hipGraphDestroy(g);
      return PM_EDEVICE;
    }
    b->graph = g;
  }
  for (int32_t i = 0; i < n_cycles; ++i)
    if (hipGraphLaunch(b->exec, as_stream(stream)) != hipSuccess) return PM_EDEVICE;
  if (n_cycles > 0 && cycle_sort_interval(b->shape.sort_interval, b->steps_per_cycle) > 0) b->since_sort = 0;
  return PM_OK;
}

pm_status pm_batch_time_kernels(pm_batch* b, int32_t n_steps, void* stream, double* push_ms, double* mcc_ms) {
  if (!b || n_steps < 1 || !push_ms || !mcc_ms) return PM_EINVAL;
  if (!batch_ok(b)) return PM_ESTATE;
  const hipStream_t st = as_stream(stream);
  KernelTimer tm;
  for (int k = 0; k < 4; ++k)
    if (hipEventCreate(&tm.ev[k]) != hipSuccess) return PM_EDEVICE;
  pm_status s = PM_OK;
  const std::vector<char> sorts = batch_sorts(b, n_steps, false);
  for (const BatchLane& L : b->lanes) {
    s = b->fp64 ? lane_steps<double>(b, L, n_steps, sorts, st, &tm)
                : lane_steps<float>(b, L, n_steps, sorts, st, &tm);
    if (s != PM_OK) break;
  }
  for (int k = 0; k < 4; ++k) (void)hipEventDestroy(tm.ev[k]);
  if (s != PM_OK) return s;
  *push_ms = tm.push_ms / (double)tm.launches;
  *mcc_ms = tm.mcc_ms / (double)tm.launches;
  return PM_OK;
}

pm_status pm_time_kernels(pm_case* c, int32_t n_steps, void* stream, double* push_ms, double* mcc_ms) {
  if (!c || n_steps < 1 || !push_ms || !mcc_ms) return PM_EINVAL;
  if (c->failed != PM_OK) return PM_ESTATE;
  const hipStream_t st = as_stream(stream);
  KernelTimer tm;
  for (int k = 0; k < 4; ++k)
    if (hipEventCreate(&tm.ev[k]) != hipSuccess) return PM_EDEVICE;
  pm_status s = PM_OK;
  const int K = c->prm.sort_interval;
  for (int32_t i = 0; i < n_steps && s == PM_OK; ++i) {
    const int sort = sort_due(&c->since_sort, K);
    hipError_t e = hipEventRecord(tm.ev[0], st);
    if (e == hipSuccess)
      e = c->prm.fp64 ? pm::launch_step<double>(c->ad, dev_args<double>(c), c->step_grid, c->work_grid, sort, st)
                      : pm::launch_step<float>(c->af, dev_args<float>(c), c->step_grid, c->work_grid, sort, st);
    if (e == hipSuccess) e = hipEventRecord(tm.ev[1], st);
    if (e == hipSuccess) e = hipEventRecord(tm.ev[2], st);
    if (e == hipSuccess)
      e = c->prm.fp64 ? pm::launch_mcc<double>(c->ad, dev_args<double>(c), c->mcc_grid, sort, st)
                      : pm::launch_mcc<float>(c->af, dev_args<float>(c), c->mcc_grid, sort, st);
    if (e == hipSuccess) e = hipEventRecord(tm.ev[3], st);
    if (e == hipSuccess && sort)
      e = c->prm.fp64 ? pm::launch_sort<double>(c->ad, c->sort_grid, st) : pm::launch_sort<float>(c->af, c->sort_grid, st);
    s = e == hipSuccess ? timer_read(&tm) : PM_EDEVICE;
  }
  for (int k = 0; k < 4; ++k) (void)hipEventDestroy(tm.ev[k]);
  if (s != PM_OK) return s;
  *push_ms = tm.push_ms / (double)tm.launches;
  *mcc_ms = tm.mcc_ms / (double)tm.launches;
  return PM_OK;
}

pm_status pm_batch_info(const pm_batch* b, int32_t* n_cases, int32_t* step_workgroups, int32_t* case_workgroups) {
  if (!b) return PM_EINVAL;
  if (n_cases) *n_cases = (int32_t)b->cases.size();
  if (step_workgroups) *step_workgroups = b->step_grid;
  if (case_workgroups) {
    std::vector<uint32_t> nb(b->cases.size());
    PM_TRY(hipMemcpy(nb.data(), b->step_nblk, nb.size() * 4, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < nb.size(); ++i) case_workgroups[i] = b->cases[i] ? (int32_t)(nb[i] >> 16) : 0;
  }
  return PM_OK;
}

void pm_batch_destroy(pm_batch* b) {
  if (!b) return;
  for (BatchLane& L : b->lanes) {
    if (L.st) {
      (void)hipStreamSynchronize(L.st);
      (void)hipStreamDestroy(L.st);
    }
    if (L.done) (void)hipEventDestroy(L.done);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
}

}  // extern "C"
