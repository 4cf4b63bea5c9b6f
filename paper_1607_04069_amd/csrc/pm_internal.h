// Internal layout shared by the library's kernels and its host code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {

constexpr int kBlock = 256;            // threads per workgroup (4 waves of 64)
constexpr int kMaxCells = 1024;        // LDS-resident grid limit
// A particle's next examination by the null-collision schedule is kept as a
// 16-bit code: the step modulo 2^15, and kRedraw when the geometric wait was cut
// at kWaitCap steps (that examination only draws a fresh wait).  A pending
// examination is never more than kWaitCap steps ahead, so the low 15 bits match
// the step counter first at the examination step itself.
constexpr int kWaitCap = 32767;
constexpr uint32_t kRedraw = 0x8000u;
constexpr int kAngleBins = 360;        // 0.25 degree ion impact-angle bins
constexpr int kTpThetaBins = 90;       // 1 degree test-atom angle bins
// joint ion energy-angle histogram: groups of 4 of the 1 eV and of the 0.25 degree bins
constexpr int kIeadEGroup = 4;
constexpr int kIeadABins = kAngleBins / 4;
constexpr int kMaxPhaseBins = 128;     // phase bins per RF period of the phase-resolved sums
// Most slots a push workgroup deposits into its LDS charge tile before it
// flushes the tile: a cell packs a 16-bit deposit count and a slot deposits once
// (births are deposited by the collision kernel).
constexpr int kMaxSlotsPerBlock = 65532;

// A work-list entry that names no workgroup (a slotted batch pads its lists
// with these): the workgroup ends at once.
constexpr uint32_t kIdleWork = 0xFFFFFFFFu;

// sticky failure bits in Ctrl::status
enum : uint32_t { ST_CAPACITY = 1u, ST_NUMERIC = 2u };

// Device-resident control block of one case.  Written by the last collision
// workgroup of each step (the step epilogue) and read by every workgroup of the
// next step.
struct Ctrl {
  int64_t step;              // index l of the next step to run
  int64_t n_range[2];        // slots [0, n_range) are scanned this step
  int64_t n_alloc[2];        // slot allocator; births append here
  int64_t n_live[2];         // live particles
  uint32_t done;             // workgroups finished in the running step
  uint32_t buf;              // particle buffer in use (ping-pong with the sort)
  uint32_t status;           // ST_* bits
  uint32_t sort_due;         // 1 when this step's deposit also counts cells
  int64_t avg_steps;         // steps in the averaging window
  double v_sum;              // sum of V(t_l) over the window
  uint64_t absorbed[2][2];   // [species][electrode]
  uint64_t collisions[5];    // e el, e exc, e ion, unused, Ar+ cx
  uint64_t candidates[2];
  uint64_t overflow[2];
  uint64_t births;
  uint64_t particle_steps;
  int64_t ion_e_fx[2];       // sum of impact energies, units of 2^-20 eV
  uint32_t n_cand[2];        // collision candidates listed in the running step
  int64_t n_abs_net;         // Ar+ minus electrons absorbed at electrode 0 since the load
  double sigma_init;         // surface charge of electrode 0 at the first field solve
  double phi0;               // potential of electrode 0 in the field of step `step`
  uint32_t circ_ready;       // sigma_init recorded
  uint32_t pad32;
  uint64_t pad[3];
};

// Step counters that every push and collision workgroup adds to, spread over
// kBanks copies kBankStride bytes apart (workgroup b adds to copy b mod kBanks):
// on one copy the device-scope atomics of a large case's thousands of
// workgroups per step serialise on one cache line.  The host adds the copies to
// the control block's fields when it reads them; the live counts are made whole
// on the device by the cell scan before each sort.
constexpr int kBanks = 16;
constexpr int kBankStride = 4096;
struct CtrBank {
  uint64_t particle_steps;
  uint64_t candidates[2];
  uint64_t collisions[5];
  uint64_t overflow[2];
  uint64_t births;
  uint64_t absorbed[2][2];
  int64_t n_live[2];
  uint64_t pad[1];
};
static_assert(sizeof(CtrBank) <= kBankStride, "bank stride");

// Derived constants of a case (computed once on the host).
struct CaseConst {
  int N, Nt;
  int n_ebins;
  int sort_interval;
  uint32_t flags;
  int fp64;
  double dx, dt, w;
  double v_scale;            // dx / dt: cells per step -> m/s
  double inv_v_scale;        // dt / dx
  double c_phi;              // e w dx / (2^32 eps0): volts per unit of q
  double kpush[2];           // (q/m) dt^2 / dx: V/m -> cells per step^2
  double ion_over_e;         // kpush[1] / kpush[0] = -m_e / M
  double V0, phase;
  double V2, phase2;         // second harmonic
  double cb;                 // blocking capacitance per area, F/m^2 (0: ideal source)
  double cgap;               // eps0 / L, F/m^2
  double e_w;                // e w: charge per area of one super-particle, C/m^2
  double eps0;
  double n_gas;
  double nu_max[2];
  double log1m_p[2];         // log1p(-P_tot); 0 when there are no collisions
  int has_coll;
  int dep_mode;               // LDS deposit: 0 per lane, 1 DPP sum of one-cell wavefronts
  int prof;                   // 1: record per-workgroup timestamps of each step
  int unroll;                 // particles per lane loaded together in the step (8 or 16)
  int waves;                  // register budget of the push kernel: 0 free, 6 waves per SIMD
  double half_mr_over_e[2];  // 0.5 m_r / e: eV per (m/s)^2
  double m_ratio_e;          // m_e / (m_e + M)
  double M_ratio_e;          // M / (m_e + M)
  double two_eexc_over_mr;   // 2 E_exc e / m_r(e)
  double v_e_per_sqrt_ev;    // sqrt(2 e / m_e): speed of 1 eV electron per sqrt(eV)
  double sig_gas;            // sqrt(k_B T_gas / M)
  double sigma_el, eth_exc, sigma0_exc, eth_ion, sigma0_ion, sigma_cx;
  double ion_e_factor;       // 0.5 M (dx/dt)^2 / e: eV per (cells/step)^2
  uint64_t seed;
  uint64_t case_id;
  int64_t capacity[2];
  int n_phase;               // phase bins per RF period (0: no phase-resolved sums)
  int flux;                  // 1: the particle flux profiles are averaged too
};

// Phase bin of step l: the RF phase (l mod N_t) / N_t cut into n_phase equal bins.
__host__ __device__ inline int phase_bin(const CaseConst& c, int64_t l) {
  return (int)(((l % c.Nt) * (int64_t)c.n_phase) / c.Nt);
}

// Device code sees the particle arrays as global-memory pointers: in the
// batched kernels they are read from a device table rather than from kernel
// arguments, and without the address space every access would be a flat one.
// The layout (64-bit pointers) is the same for host and device compilation.
#if defined(__HIP_DEVICE_COMPILE__)
#define PM_GLOBAL __attribute__((address_space(1)))
#else
#define PM_GLOBAL
#endif

// What the push leaves alone: the transverse velocity and the identity that
// keys the particle's random numbers, one record per slot, so that the gather
// of a collision candidate fetches one record rather than three scattered
// words (16 bytes in FP32, one vector load).
template <typename R>
struct alignas(sizeof(R) == 4 ? 16 : 8) Cold {
  R uy, uz;
  uint64_t id;
};

// A collision candidate's position x^(l+1) and velocity v_x^(l+1/2) (cells,
// cells per step) as the push left them, listed beside its slot.
template <typename R>
struct alignas(2 * sizeof(R)) XU {
  R x, u;
};

// Pointers into the case arena.
template <typename R>
struct Particles {
  R PM_GLOBAL* xt[2][2];     // [species][buffer]
  R PM_GLOBAL* ux[2][2];
  Cold<R> PM_GLOBAL* cold[2][2];
  uint16_t PM_GLOBAL* next[2][2];  // examination codes
};

struct GridPtrs {
  int64_t* Q;                // [3][2][nodes]: charge of x^(l) cycles through 3 buffers
  uint64_t* sumQ;            // [2][nodes][2]: 128-bit (lo, hi) accumulators
  void* Epair;               // [2][N] (E'_j, E'_{j+1} - E'_j) in particle precision
  double* E64;               // [nodes] field of the next step
  double* phi64;             // [nodes] potential (filled on request)
  double* diag_out;          // [3][nodes] staging for sampled ne, ni, phi
  uint64_t* iedf;            // [2][n_ebins]
  uint64_t* iadf;            // [2][kAngleBins]
  uint32_t* cell_count;      // [2][N] per-cell live counts / sort cursors
  uint32_t* cell_off;        // [2][N] sorted cell offsets
  double* ybin;              // [n_ebins] sputter yield per energy bin
  uint64_t* yield_out;       // [2] emitted atoms, impacts
  uint64_t* prof;            // [grid][8] timestamps of the last step (when enabled)
  uint32_t* cand;            // [capacity_e + capacity_i] candidate slots of the running step
  void* cand_xu;             // [capacity_e + capacity_i] XU<R> of those candidates
  unsigned char* banks;      // [kBanks] CtrBank, kBankStride apart
  uint64_t* sumQp;           // [n_phase][2][nodes][2]: charge sums of each phase bin
  double* phase_v;           // [n_phase] driven-electrode potential summed per bin
  int64_t* phase_n;          // [n_phase] steps per bin
  uint64_t* sumF;            // [max(n_phase, 1)][2][nodes][2]: flux sums, 2^-40 cells per step
  int64_t* flux_n;           // [max(n_phase, 1)] flux samples per bin
  uint64_t* iedf_taken;      // [2][n_ebins] impacts already turned into atoms by live injection
  uint64_t* iead;            // [2][ceil(n_ebins / 4)][kIeadABins] joint energy-angle histogram
};

__host__ __device__ inline CtrBank* bank_of(const GridPtrs& g, int b) {
  return reinterpret_cast<CtrBank*>(g.banks + (size_t)(b % kBanks) * kBankStride);
}

template <typename R>
struct KArgs {
  CaseConst c;
  Ctrl* ctrl;
  Particles<R> p;
  GridPtrs g;
};

__host__ __device__ inline int64_t qbuf_index(int64_t step, int which) {  // which: 0 read, 1 deposit, 2 clear
  return (step + which) % 3;
}

}  // namespace pm
