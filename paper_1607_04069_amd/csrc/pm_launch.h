// Host launchers of the library's kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pm_internal.h"

namespace pm {

size_t field_lds_bytes(int N);
template <typename R> hipError_t launch_load(const KArgs<R>&, int64_t np_e, int64_t np_i, double sig_e,
                                             double sig_i, hipStream_t);
template <typename R> hipError_t launch_deposit_all(const KArgs<R>&, int64_t nmax, hipStream_t);
template <typename R> hipError_t launch_sort(const KArgs<R>&, int grid, hipStream_t);
template <typename R> hipError_t launch_field(const KArgs<R>&, int want_phi, hipStream_t);
// the step reads the case's arguments from their device copy (dev_args); A is
// the host copy, for the launch shape
template <typename R> hipError_t launch_step(const KArgs<R>& A, const KArgs<R>* dev_args, int grid, int nwork,
                                             int count_cells, hipStream_t);
template <typename R> int step_blocks_per_cu(int N, int unroll, int waves, bool batch);
template <typename R> int mcc_blocks_per_cu(int N, bool batch);
template <typename R> hipError_t launch_mcc(const KArgs<R>& A, const KArgs<R>* dev_args, int grid, int count_cells,
                                            hipStream_t);
template <typename R> hipError_t launch_mcc_batch(const KArgs<R>* cases, const uint32_t* work,
                                                  const uint32_t* nblocks, int grid, int maxN, int count_cells,
                                                  hipStream_t);
template <typename R> hipError_t launch_diag_finalize(const KArgs<R>&, int bin, hipStream_t);  // bin < 0: window
template <typename R> hipError_t launch_step_batch(const KArgs<R>* cases, const uint32_t* work,
                                                   const uint32_t* nblocks, int grid, int maxN, int unroll,
                                                   int waves, int count_cells, hipStream_t);
template <typename R> hipError_t launch_sort_batch(const KArgs<R>* cases, const uint32_t* work,
                                                   const uint32_t* nblocks, int grid, int maxN, hipStream_t);
hipError_t launch_scan_cells(const CaseConst&, const GridPtrs&, Ctrl*, hipStream_t);
hipError_t launch_diag_reset(const CaseConst&, const GridPtrs&, Ctrl*, hipStream_t);

// sputter yield and test-particle flight
struct TpConst {
  double L, lat;
  double nu_max;             // n_gas (sigma g)_max
  double inv_nu_max;
  double sg_exp;             // 2 - 2 omega: (sigma g) ~ g^sg_exp for VHS
  double log2_gcap;          // log2 of the majorant's relative speed
  double sig_gas;            // sqrt(k_B T / m_gas)
  double m_ratio, M_ratio;   // m/(m+M), M/(m+M)
  double s_max, u_s;         // Thompson inversion
  double v_per_sqrt_ev;      // sqrt(2 e / m_test)
  double e_half_m;           // 0.5 m / e: eV per (m/s)^2
  double ebin, tbin;
  int n_ebins, n_tbins;
  int n_xbins;               // cells of the track-length profiles (0: none)
  double xbin, inv_xbin;     // cell width and its inverse, m
  int mode;
  int scatter;               // 0 VHS isotropic, 1 M1
  int electrode;             // emission from the target (0) or the substrate (1)
  double dt;                 // fixed flight time (0: gridless, from the majorant)
  double nu_dt;              // nu_max dt: the fixed-step probability at the majorant
  int64_t e_max;
  int64_t n_atoms, first_atom;
  uint64_t seed, job;
};

struct TpTally {              // device tallies (zeroed before a run)
  uint64_t n_sub, n_tgt, n_unf;
  uint64_t events, collisions, overflow;
  int64_t e_sub_fx, e_tgt_fx;  // energy sums, units of 2^-20 eV
  uint64_t pad[8];
};

struct TpTrace {
  int32_t* wall;
  uint32_t* events;
  float* energy_ev;
  float* theta_deg;
  float* tof_s;
  float* vx;
  float* vy;
  float* vz;
};

// prof: [4][n_xbins + 1] int64 track-length tallies (partial-cell times, full-cell
// time differences, partial-cell displacements, full-cell displacement
// differences), or null
hipError_t launch_tp_flight(const TpConst&, TpTally* tally, uint64_t* e_hist, uint64_t* th_hist,
                            uint64_t* tof_hist, TpTrace trace, int64_t* prof, int grid, hipStream_t);
// track-length tallies -> [4][nx] doubles: time (s), displacement (m), density (m^-3), mean v_x (m/s)
hipError_t launch_tp_profiles(const int64_t* prof, int nx, double h, double per_atom, double* out, hipStream_t st);
hipError_t launch_zero_u64(void* p, size_t bytes, hipStream_t st);
// Bytes of the per-GPU scratch of pm_run_test_particles_static, and its device
// address on the current device (looked up once per device).
constexpr size_t kTpScratchBytes = (size_t)1 << 20;
hipError_t tp_scratch(void** ptr);
hipError_t launch_yield(const uint64_t* iedf, const double* ybin, int n_ebins, uint64_t seed,
                        uint64_t job, int electrode, uint64_t* taken, uint64_t* out, hipStream_t st);

}  // namespace pm
