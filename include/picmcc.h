/*
 * picmcc.h -- C interface of the MI355X PIC/MCC + test-particle library.
 *
 * Method: Trieschmann, Schmidt, Mussenbrock, "Particle-in-Cell/Test-Particle
 * Simulations of Technological Plasmas: Sputtering Transport in Capacitive
 * Radio Frequency Discharges" (arXiv:1607.04069).  The charged-particle module
 * is the PIC/MCC cycle of Sec. IV.A (Fig. 4); the neutral module is the test
 * particle method of Sec. IV.B; they are joined one way by the ion flux onto the
 * target (Sec. III, Fig. 3).
 *
 * Conventions
 *  - Every call returns pm_status; no exception crosses the interface.
 *  - Device memory is owned by the caller: the library places a case (or a
 *    test-particle job) inside an arena the caller allocated on the GPU and
 *    passes in with its size in bytes.  The library allocates only small host
 *    handles, pinned host staging for read-outs, and its HIP graphs.
 *  - Streams are hipStream_t values passed as void*; NULL is the default stream.
 *  - Host buffers named in structs below are owned by the caller and must hold
 *    the sizes stated; the library never keeps pointers to them after a call.
 *  - Positions are in cell units xt = x / dx (node m at xt = m); internal
 *    velocities u are in cells per time step (v * dt / dx).
 *  - A case that hits a run-time failure (particle capacity, NaN/Inf) becomes
 *    sticky-failed: the failing call returns the error and every later call on
 *    the case returns PM_ESTATE.  Other cases are unaffected.
 *  - One case is not thread-safe; different cases may be driven from different
 *    host threads and streams.
 */
#ifndef PICMCC_H
#define PICMCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PM_OK = 0,
  PM_EINVAL = -1,     /* invalid argument; no side effects */
  PM_ENOSPACE = -2,   /* arena smaller than the footprint */
  PM_EDEVICE = -3,    /* a HIP call failed */
  PM_ECAPACITY = -4,  /* particle slots exhausted by births; case failed */
  PM_ENUMERIC = -5,   /* NaN or Inf found in the particle state; case failed */
  PM_ESTATE = -6      /* call on a failed case or an unsupported state */
} pm_status;

/* pm_case_params.flags: test modes of the cycle */
enum { PM_NO_SELF_FIELD = 1u,   /* charges feel only the applied field */
       PM_NO_COLLISIONS = 2u }; /* skip the Monte Carlo collision step */

/* pm_diagnostics.warnings: the limits of Sec. IV.A 'Limitations and
 * Constraints', checked at init from n0 and T_e (warnings, not errors) */
enum { PM_WARN_DEBYE = 1u,        /* dx > Debye length                */
       PM_WARN_PLASMA_FREQ = 2u,  /* omega_p dt > 0.2                 */
       PM_WARN_PPC = 4u };        /* fewer than 20 super-particles per cell */

enum { PM_ELECTRON = 0, PM_ION = 1 };
enum { PM_N_ANGLE_BINS = 360 };   /* ion impact angle histogram, 0.25 deg bins */
enum { PM_TP_THETA_BINS = 90 };   /* test-atom impact angle histogram, 1 deg bins */
enum { PM_IEAD_E_GROUP = 4,       /* joint ion energy-angle histogram: 4 eV ...  */
       PM_IEAD_A_BINS = 90 };     /* ... by 1 deg bins                           */

/* Analytic cross sections (Sec. IV.A 'Particle Collisions'; the paper's LXcat
 * tables are replaced by these forms).  Energies in eV, areas in m^2. */
typedef struct {
  double sigma_el;               /* e-Ar elastic, constant                     */
  double eth_exc, sigma0_exc;    /* e-Ar excitation sigma0 ln(x)/x, x=eps/eth  */
  double eth_ion, sigma0_ion;    /* e-Ar ionisation sigma0 ln(x)/x             */
  double sigma_cx;               /* Ar+-Ar resonant charge exchange, constant  */
} pm_xsec;

/* One discharge (Sec. III scenario; Sec. IV.A cycle). */
typedef struct {
  double gap_m;                  /* electrode gap L                                    */
  int32_t n_cells;               /* N cells, N+1 nodes; 1 <= N <= 1024                 */
  int32_t steps_per_cycle;       /* N_t; dt = 1 / (freq_hz * N_t)                      */
  double freq_hz;                /* RF frequency                                       */
  double v0_volt, phase_rad;     /* source V(t) = V0 cos(wt + phase) + V2 cos(2wt + phase2),
                                    wt = 2 pi (l mod N_t)/N_t (Sec. III: two harmonics) */
  double p_pa, t_gas_k;          /* argon background, n = p / (k_B T)                  */
  double n0_m3;                  /* initial plasma density; weight w = n0 L / np_e     */
  int64_t np_e, np_i;            /* initial super-particles per species                */
  double te_ev, ti_ev;           /* Maxwellian loading temperatures                    */
  int64_t capacity_e, capacity_i;/* particle slots per species (>= np)                 */
  double ecap_e_ev, ecap_i_ev;   /* energy caps of the null-collision majorant (Eq. 6) */
  pm_xsec xs;
  uint64_t seed;                 /* Philox key word 0                                  */
  uint32_t case_id;              /* Philox key word 1                                  */
  uint32_t flags;                /* PM_NO_SELF_FIELD | PM_NO_COLLISIONS                */
  int32_t fp64;                  /* 1: FP64 particles and push; 0: FP32                */
  int32_t sort_interval;         /* steps between cell sorts, 0 = never.  Plain launches
                                    (pm_step) count steps across calls; a captured RF
                                    cycle sorts every Kc-th step, Kc the largest
                                    divisor of N_t not above sort_interval          */
  double v2_volt, phase2_rad;    /* second-harmonic amplitude and phase (0: one sinusoid) */
  double cb_f_m2;                /* blocking capacitor between the source and the driven
                                    electrode, per electrode area, F/m^2 (Sec. III, Sec.
                                    IV.A 'External Lumped Circuits'); 0: the source
                                    drives the electrode directly.  The capacitor is
                                    uncharged at the load; the electrode's surface
                                    charge (Gauss over the half cell) then equals its
                                    value at the load plus what the circuit delivered,
                                    cb (V(t) - Phi_0), plus the net charge absorbed from
                                    particles.  The time-averaged phi[0] of
                                    pm_diagnostics is the DC self-bias. */
  int32_t n_phase;               /* phase-resolved averages (Sec. IV: the solution is
                                    averaged over time and also resolved in the RF
                                    phase): step l belongs to bin
                                    floor((l mod N_t) n_phase / N_t); 0 = none,
                                    at most 128 and at most N_t; read by
                                    pm_sample_phase */
  int32_t flux_profiles;         /* 1: average the particle flux profiles Gamma_s(x) too
                                    (Fig. 8: fluxes and mean velocities of e and Ar+),
                                    sampled before every step of pm_step and
                                    pm_step_rf_cycles (an extra read of x and v_x,
                                    8 B per particle in FP32); such a case cannot
                                    join a pm_batch */
} pm_case_params;

typedef struct pm_case pm_case;  /* opaque host handle owned by the library */

/* Time-averaged diagnostics (Sec. IV: averages over a period once steady).
 * Caller-owned host arrays; nodes = n_cells + 1, n_ebins = ceil(ecap_i_ev).
 * Electrode 0 is the driven target at x = 0, electrode 1 the substrate at x = L. */
typedef struct {
  double* ne;                    /* [nodes] electron density, m^-3              */
  double* ni;                    /* [nodes] Ar+ density, m^-3                   */
  double* phi;                   /* [nodes] potential, V                        */
  uint64_t* iedf;                /* [2][n_ebins] Ar+ impact energy, 1 eV bins   */
  uint64_t* iadf;                /* [2][PM_N_ANGLE_BINS] Ar+ impact angle       */
  /* filled by the call: */
  int64_t step;                  /* steps taken since init                      */
  int32_t status;                /* pm_status of the case                       */
  uint32_t warnings;             /* PM_WARN_* bits                              */
  int64_t n_e, n_i;              /* live super-particles now                    */
  int64_t avg_steps;             /* steps in the averaging window               */
  uint64_t absorbed[2][2];       /* [species][electrode] absorbed super-particles */
  double flux[2][2];             /* [species][electrode] wall flux, m^-2 s^-1   */
  double mean_ion_energy[2];     /* [electrode] eV                              */
  uint64_t collisions[5];        /* e elastic, e excitation, e ionisation, unused, Ar+ CX */
  uint64_t candidates[2];        /* null-collision candidates per species       */
  uint64_t overflow[2];          /* candidates above the majorant              */
  uint64_t births;               /* super-particles created by ionisation      */
  uint64_t particle_steps;       /* particles advanced by one dt, summed        */
  double* gamma_e;               /* [nodes] electron flux profile, m^-2 s^-1 (+x toward
                                    the substrate); may be NULL; zeros unless the case
                                    has flux_profiles.  Each sample is the state a step
                                    starts from (x^(l), v_x^(l-1/2)) weighted onto the
                                    nodes like the charge. */
  double* gamma_i;               /* [nodes] Ar+ flux profile, same form           */
  double* u_e;                   /* [nodes] electron mean velocity gamma_e / ne, m/s
                                    (0 where ne = 0); may be NULL                 */
  double* u_i;                   /* [nodes] Ar+ mean velocity gamma_i / ni, m/s    */
  uint64_t* iead;                /* [2][ceil(n_ebins / 4)][PM_IEAD_A_BINS] Ar+ impacts by
                                    energy (4 eV) and angle (1 deg) together (Fig. 7: the
                                    energy-angle distribution at the target); its sums
                                    over one axis are iedf and iadf grouped by 4; may be
                                    NULL */
} pm_diagnostics;

/* Averages over the steps of one RF phase bin of the window (caller-owned host
 * arrays of nodes doubles, each may be NULL). */
typedef struct {
  double* ne;                    /* [nodes] m^-3                                 */
  double* ni;                    /* [nodes] m^-3                                 */
  double* phi;                   /* [nodes] V: Phi of the bin's averaged charge and drive */
  double* gamma_e;               /* [nodes] m^-2 s^-1 (zeros without flux_profiles) */
  double* gamma_i;               /* [nodes] m^-2 s^-1                            */
  double* u_e;                   /* [nodes] m/s, gamma_e / ne (0 where ne = 0)    */
  double* u_i;                   /* [nodes] m/s, gamma_i / ni                     */
  /* filled by the call: */
  int64_t n_steps;               /* steps of the window in this bin              */
  int64_t n_flux_samples;        /* flux samples of the window in this bin       */
  int32_t status;                /* pm_status of the case                        */
} pm_phase_sample;

/* Host copy of one species in internal units (live particles only). */
typedef struct {
  int64_t n;                     /* get: live count written; set: count given   */
  int64_t capacity;              /* get: length of the arrays below             */
  double* xt;                    /* cells                                        */
  double* ux; double* uy; double* uz;   /* cells per step                       */
  uint64_t* id;
  uint32_t* next;                /* step of the next null-collision examination,
                                    bits 0-30; bit 31 set when that examination
                                    only draws a fresh wait (the geometric wait
                                    was cut at 32767 steps); all bits set for a
                                    species without collisions.  set: the step
                                    must lie within 32767 steps at or after the
                                    next step to run, else PM_EINVAL           */
} pm_particles;

/* Host copy of the grid state for the next step to run. */
typedef struct {
  int64_t* qe; int64_t* qi;      /* [nodes] charge in units of 2^-32 super-particle */
  double* phi;                   /* [nodes] potential of this charge and V(t_l)     */
  double* efield;                /* [nodes] E, V/m                                  */
  /* filled by the call (blocking-capacitor state, zero without a capacitor): */
  double sigma_init;             /* driven electrode's surface charge at the load, C/m^2 */
  int64_t n_absorbed_net;        /* Ar+ minus electrons absorbed there since the load   */
} pm_fields;

/* Sputter source (Sec. IV.B 'Wall Interactions'). */
typedef struct {
  double yield_const;            /* Y when n_table == 0                          */
  int32_t n_table;               /* >0: Y(E) by linear interpolation in the table */
  const double* table_e_ev;      /* [n_table] host, ascending                    */
  const double* table_y;         /* [n_table] host                               */
  double u_s_ev, e_cut_ev;       /* Thompson binding energy and cut-off          */
  int64_t n_atoms;               /* > 0: launch this many atoms, 0: yield-derived */
  uint64_t seed;
  uint32_t job_id;
  int32_t electrode;             /* 0: the target's ion impacts (x = 0); 1: the
                                    substrate's (x = L), re-sputtering its Al coat */
  int32_t since_last;            /* 0: every impact of the averaging window; 1: live
                                    coupling -- only the impacts recorded since the
                                    previous since_last call on this electrode in the
                                    window (call it every step or RF cycle and fly
                                    what it returns).  Impact i of energy bin b keys
                                    its draws by (i, b) and the returned first_atom
                                    continues the window's atom ids, so a window's
                                    live calls emit and fly exactly the atoms of one
                                    whole-window call; flux_m2s is then the flux
                                    since the previous call. */
} pm_sputter_params;

typedef struct {
  int64_t n_atoms;               /* atoms to fly                                  */
  int64_t first_atom;            /* id of the first atom (a shard's offset)       */
  int64_t n_impacts;             /* target ion impacts the count came from        */
  int64_t n_emitted;             /* atoms emitted by the yield rule               */
  double flux_m2s;               /* emitted flux, m^-2 s^-1 (0 if not known)      */
  double u_s_ev, e_cut_ev;
  uint64_t seed;
  uint32_t job_id;
  int32_t electrode;             /* emission from the target (0: x = 0, into +x) or
                                    the substrate (1: x = L, into -x)             */
} pm_tp_source;

enum { PM_TP_NORMAL = 0, PM_TP_BOX = 1 };
enum { PM_TP_VHS = 0, PM_TP_M1 = 1 };     /* pm_tp_params.scatter */

/* Test-particle flight (Sec. IV.B): VHS collisions (Eq. 8) with a Maxwellian
 * argon background, sticking electrodes, periodic lateral directions. */
typedef struct {
  double p_pa, t_gas_k;
  double d_ref, omega, t_ref;    /* VHS reference diameter, viscosity index, T_ref */
  double m_test_amu, m_gas_amu;
  double gap_m, lateral_m;
  int32_t mode;                  /* PM_TP_NORMAL or PM_TP_BOX (periodic in x too) */
  int64_t e_max;                 /* candidate events before an atom is unfinished */
  int32_t n_ebins; double ebin_ev;   /* substrate energy histogram               */
  int32_t n_tbins; double tbin_s;    /* substrate time-of-flight histogram       */
  int32_t n_xbins;               /* cells of the gap (0..1024) for the density and */
                                 /* mean velocity profiles (PM_TP_NORMAL; 0 none)  */
  int32_t scatter;               /* PM_TP_VHS: isotropic in the centre-of-mass frame;
                                    PM_TP_M1: deflection chi = pi (1 - b/b_max) about
                                    the relative velocity, with the VHS cross section
                                    at d_ref sqrt(4/3) ('Binary Interactions') */
  double dt_s;                   /* 0: gridless flight, free-flight times from the
                                    majorant (Eq. 5); > 0: fixed step ('Collisional
                                    Transport'): flights of dt, then a collision with
                                    the linearised probability n sigma(g) g dt of
                                    Eq. (7) for a fresh partner (> 1 counted as an
                                    overflow); e_max then counts steps */
} pm_tp_params;

/* Optional per-atom records, DEVICE arrays of length n_atoms (any may be NULL). */
typedef struct {
  int32_t* wall;                 /* 0 target, 1 substrate, 2 unfinished          */
  uint32_t* events;              /* candidate events flown                       */
  float* energy_ev; float* theta_deg; float* tof_s;
  float* vx; float* vy; float* vz;   /* velocity at the end, m/s                 */
} pm_tp_trace;

typedef struct {
  uint64_t* e_hist;              /* [n_ebins] host, substrate energies           */
  uint64_t* theta_hist;          /* [PM_TP_THETA_BINS] host                      */
  uint64_t* tof_hist;            /* [n_tbins] host                               */
  const pm_tp_trace* trace;      /* optional device records                      */
  double* time_s;                /* [n_xbins] host or NULL: residence time of all */
                                 /* atoms in each cell, s (the density of a cell */
                                 /* is flux / n_atoms * time_s / dx)             */
  double* disp_m;                /* [n_xbins] host or NULL: signed x-displacement */
                                 /* in each cell, m (mean v_x = disp_m / time_s) */
  /* filled by the call: */
  int64_t n_substrate, n_target, n_unfinished;
  uint64_t events, collisions, overflow;
  double e_sum_substrate, e_sum_target;   /* eV */
  double eta;                    /* n_substrate / n_atoms                        */
  double deposition_flux;        /* eta * source flux, m^-2 s^-1                 */
  double nu_max;                 /* null-collision majorant, s^-1                */
  double* density_m3;            /* [n_xbins] host or NULL: test-atom density of each
                                    cell, m^-3, from the time-weighted track lengths
                                    (Sec. IV.B, last paragraph): the source flux
                                    src->flux_m2s shared by the n_atoms atoms, times
                                    the cell's residence time, over the cell width
                                    (0 everywhere when the flux is 0)            */
  double* mean_vx;               /* [n_xbins] host or NULL: mean x-velocity of the
                                    atoms in each cell, m/s (displacement over
                                    residence time; 0 in a cell no atom entered) */
} pm_tp_result;

/* --- the five calls --------------------------------------------------------- */

/* Device bytes a case needs (0 if the parameters are invalid). */
size_t pm_case_footprint(const pm_case_params* params);

/* Validate, lay out the case in dev_arena, load particles (uniform positions,
 * Maxwellian velocities by Box-Muller; Sec. IV), sort them by cell, deposit the
 * initial charge and solve the initial field.  Enqueued on hip_stream; the
 * call synchronises that stream before returning.  *out receives the handle. */
pm_status pm_init_case(const pm_case_params* params, void* dev_arena, size_t arena_bytes,
                       void* hip_stream, pm_case** out);

/* Advance n_cycles RF cycles (n_cycles * N_t steps of the Fig. 4 cycle).  One
 * cycle is captured once as a HIP graph and replayed.  Asynchronous. */
pm_status pm_step_rf_cycles(pm_case* c, int32_t n_cycles, void* hip_stream);

/* Copy and convert the time averages since the last reset (synchronises).
 * reset != 0 starts a new averaging window after the read. */
pm_status pm_sample_diagnostics(pm_case* c, pm_diagnostics* out, int32_t reset, void* hip_stream);

/* Phase-resolved averages (Sec. IV) of bin 0 <= bin < n_phase over the window
 * that pm_sample_diagnostics(reset) started, synchronises.  PM_EINVAL for a bin
 * out of range (every bin when the case has n_phase = 0).  The bins' averages
 * weighted by their n_steps give the window's time averages. */
pm_status pm_sample_phase(pm_case* c, int32_t bin, pm_phase_sample* out, void* hip_stream);

/* Count the atoms the recorded target impacts sputter (yield rule of Sec. IV.B:
 * N = ceil(Y) checks R <= Y/N per impact, at the impact energy's bin centre),
 * on the GPU, and describe the source.  Synchronises. */
pm_status pm_inject_sputtered(pm_case* c, const pm_sputter_params* sp, pm_tp_source* out,
                              void* hip_stream);

/* Fly source->n_atoms test atoms to the walls (Sec. IV.B) with tallies in an
 * arena of pm_tp_footprint bytes.  Synchronises; fills *out. */
pm_status pm_run_test_particles(const pm_tp_params* tp, const pm_tp_source* src,
                                void* dev_arena, size_t arena_bytes, void* hip_stream,
                                pm_tp_result* out);

/* --- the rest of the interface ------------------------------------------------ */

size_t pm_tp_footprint(const pm_tp_params* tp);

/* Bytes of the per-GPU scratch that pm_run_test_particles_static uses. */
enum { PM_TP_STATIC_BYTES = 1 << 20 };

/* pm_run_test_particles without an arena, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the tallies live in a static device array of
 * PM_TP_STATIC_BYTES per GPU, which the library holds until the process ends.
 * Computes exactly what pm_run_test_particles computes for the same arguments.
 * PM_ENOSPACE, with no side effects, when pm_tp_footprint(tp) exceeds
 * PM_TP_STATIC_BYTES; PM_EINVAL as pm_run_test_particles.  The call allocates
 * nothing on the device or the host; it clears the array with a kernel, copies
 * the results into the caller's host arrays of *out and synchronises
 * hip_stream.  Every call on one GPU shares that GPU's array (the last call's
 * contents stay in it): calls that overlap on one GPU, from several host
 * threads or on streams that run concurrently, race and must be serialised by
 * the caller. */
pm_status pm_run_test_particles_static(const pm_tp_params* tp, const pm_tp_source* src, void* hip_stream,
                                       pm_tp_result* out);

/* Advance n_steps single steps with plain launches (no graph). Asynchronous. */
pm_status pm_step(pm_case* c, int64_t n_steps, void* hip_stream);

/* Sizes of the diagnostic arrays of a case. */
pm_status pm_diag_sizes(const pm_case* c, int32_t* nodes, int32_t* n_ebins);

/* Live particles of one species (compacted, slot order) to host; synchronises.
 * out->capacity must be >= the live count, else PM_EINVAL with out->n set (a
 * capacity of 0 with null arrays asks for the count); PM_EINVAL too for a null
 * array when there are particles to copy. */
pm_status pm_get_particles(pm_case* c, int32_t species, pm_particles* out, void* hip_stream);

/* Replace one species' particles with in->n particles (checkpoint restore,
 * constructed test states); re-sorts, re-deposits and re-solves the field.
 * Synchronises. */
pm_status pm_set_particles(pm_case* c, int32_t species, const pm_particles* in, void* hip_stream);

/* Checkpoint and resume.  A case's whole state is its device arena (particles,
 * charge buffers, running sums and histograms, counters, the circuit's state)
 * plus a few host counters; every random number is keyed by (seed, case, id,
 * step), so a case restored from a checkpoint continues exactly, bit for bit,
 * as the saved case would have.  pm_checkpoint_bytes: size of a checkpoint of
 * c (a header and the arena).  pm_save_checkpoint synchronises hip_stream and
 * copies the state into host_buf (caller-owned, at least that many bytes;
 * PM_EINVAL if smaller).  pm_load_checkpoint puts a saved state into c, which
 * must have been created from the same case parameters (grid, capacities,
 * precision, seed and case id, phase bins, flux profiles, cross sections):
 * PM_EINVAL, with c unchanged, for a buffer that is too small, not a
 * checkpoint, or written for other parameters; a case may be restored into
 * another arena, another process or another device.  The saved launch shape
 * is not part of the state (c keeps its own).  A restored failed case is
 * failed again.  A member of a batch may be restored between batch calls; it
 * continues from the restored step beside its neighbours.  Both synchronise
 * hip_stream; c must not be stepping on any other stream meanwhile. */
size_t pm_checkpoint_bytes(const pm_case* c);
pm_status pm_save_checkpoint(pm_case* c, void* host_buf, size_t bytes, void* hip_stream);
pm_status pm_load_checkpoint(pm_case* c, const void* host_buf, size_t bytes, void* hip_stream);

/* Charge, potential and field of the next step to run; synchronises. */
pm_status pm_get_fields(pm_case* c, pm_fields* out, void* hip_stream);

/* Derived set-up values: dx, dt, weight, nu_max[2], p_tot[2] (any may be NULL). */
pm_status pm_case_info(const pm_case* c, double* dx, double* dt, double* weight,
                       double* nu_max, double* p_tot);

/* Per-workgroup timestamps of the last step when the environment variable
 * PM_PROFILE=1 was set at pm_init_case, in the 100 MHz device wall clock.  A
 * step is two launches.  Push workgroup g writes out[8*g + k]: its start (k=0),
 * after staging the field (k=1), after its particle loop (k=2), after listing
 * its collision candidates (k=3) and at its end, after the charge flush (k=4).
 * Collision workgroup g writes its start (k=5), the end of its collisions
 * (k=6) and, for the one that ran the field solve, the end of that epilogue
 * (k=7, else 0).  *grid receives the number of rows, the larger of the two
 * workgroup counts (a row beyond a launch's count holds stale values); out may
 * be NULL to query it; cap is the length of out.  Synchronises. */
pm_status pm_get_step_profile(pm_case* c, uint64_t* out, int64_t cap, int32_t* grid, void* hip_stream);

/* --- launch shape ---------------------------------------------------------------
 * How the step kernels (push, collisions, sort) are launched.  The shape changes
 * speed only: every shape computes the same particles (by id), charges and
 * diagnostics, because the random numbers depend on (seed, case_id, particle
 * id, step) and the charge sums are integers. */
typedef struct {
  int32_t unroll;         /* particles per lane in flight: 8 or 16                      */
  int32_t waves;          /* register budget of the push kernel: 0 the compiler's own,  */
                          /* 6 at most 80 VGPRs so that six waves fit per SIMD         */
  int32_t work_groups;    /* workgroups that share the particles (a case: at most one   */
                          /* per 256 initial particles; a batch: over all its cases);   */
                          /* 0 = one resident wave of the device                        */
  int32_t deposit_mode;   /* charge into the LDS tile: 0 an atomic per particle, 1 a    */
                          /* wavefront in one cell summed by DPP, per-particle atomics */
                          /* otherwise                                                 */
  int32_t sort_interval;  /* steps between cell sorts, 0 = never                        */
  int32_t lanes;          /* a batch: its cases split into this many groups (1-4; 0 as */
                          /* 1) stepped concurrently on the library's own streams; a   */
                          /* case: ignored (reported as 1)                             */
} pm_launch_shape;

/* The case's shape; work_groups is the count in effect. */
pm_status pm_get_launch_shape(const pm_case* c, pm_launch_shape* out);

/* Change the case's shape (PM_EINVAL for values outside the ranges above; a
 * work_groups above one per 256 initial particles is lowered to that).
 * Synchronises hip_stream first; the next pm_step_rf_cycles captures a new graph. */
pm_status pm_set_launch_shape(pm_case* c, const pm_launch_shape* shape, void* hip_stream);

/* Frees the host handle and graphs; the arena stays the caller's. */
void pm_destroy_case(pm_case* c);

/* --- batches: many independent cases in the same launches ---------------------
 * A parameter sweep (the discharge of Sec. III and IV.A at several pressures,
 * voltages and grid sizes, across the collisional regimes of Sec. II) is a set
 * of cases that never interact.  A batch advances all of them together:
 * each time step of every case in the batch is one launch of the push and one
 * of the collision kernel (per lane, below), the workgroups of case 0 first,
 * then those of case 1, and so on, each case receiving a share of one resident
 * wave of workgroups in proportion to its particles.  Every case computes exactly what pm_step computes for it
 * alone: its random numbers depend only on (seed, case_id, particle id, step),
 * and its charge sums are integers, so the state of each case, compared
 * particle by particle by id, is bit-identical alone and in a batch.
 *
 * The batch keeps device tables (a copy of each case's device arguments and
 * the work lists, entry = case << 16 | workgroup within the case) in a
 * caller-provided arena of pm_batch_footprint bytes, 256-byte aligned.  The
 * cases stay owned by the caller and stay usable alone (pm_step, diagnostics,
 * particle I/O); a case must not be in two batches that run at the same time,
 * and a case must outlive every batch that holds it. */
typedef struct pm_batch pm_batch;  /* opaque host handle owned by the library */

/* Device bytes of the batch tables for these cases, 0 if they cannot form a
 * batch: n_cases outside 1..65535, a NULL or repeated case, cases that differ
 * in precision (fp64), or a case whose run has failed. */
size_t pm_batch_footprint(pm_case* const* cases, int32_t n_cases);

/* Form a batch of n_cases cases (same conditions as pm_batch_footprint:
 * PM_EINVAL, or PM_ESTATE for a failed case; PM_ENOSPACE if arena_bytes is too
 * small).  The batch has its own launch shape, initially unroll 8, waves 0,
 * one resident wave of workgroups shared out in proportion to the cases'
 * initial particles, deposit mode 1 and the first case's sort interval.
 * Writes the tables with copies enqueued on hip_stream and synchronises that
 * stream.  *out receives the handle. */
pm_status pm_batch_create(pm_case* const* cases, int32_t n_cases, void* dev_arena, size_t arena_bytes,
                          void* hip_stream, pm_batch** out);

/* The batch's launch shape (work_groups: the working workgroups in effect) and
 * a new one (rewrites the tables; synchronises hip_stream; PM_EINVAL as for
 * pm_set_launch_shape). */
pm_status pm_batch_get_launch_shape(const pm_batch* b, pm_launch_shape* out);
pm_status pm_batch_set_launch_shape(pm_batch* b, const pm_launch_shape* shape, void* hip_stream);

/* Advance every case of the batch n_steps steps, sorting after every
 * sort_interval-th step counted across calls (a captured RF cycle: every Kc-th
 * step, as for a case).  Asynchronous.  PM_ESTATE if a case of
 * the batch is known to have failed; a failure during these steps is sticky in
 * that case only and is reported by the case's next pm_sample_diagnostics. */
pm_status pm_batch_step(pm_batch* b, int64_t n_steps, void* hip_stream);

/* Advance n_cycles RF cycles; every case must have the same steps_per_cycle
 * (else PM_EINVAL).  One cycle of the whole batch is captured once as a HIP
 * graph and replayed.  Asynchronous. */
pm_status pm_batch_step_rf_cycles(pm_batch* b, int32_t n_cycles, void* hip_stream);

/* Number of cases, the workgroups of one step launch, and (if case_workgroups
 * is not NULL, an array of n_cases) the working workgroups of each case. */
pm_status pm_batch_info(const pm_batch* b, int32_t* n_cases, int32_t* step_workgroups,
                        int32_t* case_workgroups);

/* Frees the host handle and graph; the arena and the cases stay the caller's. */
void pm_batch_destroy(pm_batch* b);

/* --- slotted batches: cases that come and go -------------------------------------
 * For a served stream of sweep cases (continuous batching): a batch of n_slots
 * slots, initially empty, whose RF cycle is captured as a HIP graph once.  A
 * case joins a slot or a slot is emptied by pm_batch_set_slot, which rewrites
 * the batch's device tables: its work lists have a fixed length (one resident
 * wave of each kernel per lane, padded with entries whose workgroups end at
 * once), so the captured graph stays valid while the members change; a new
 * launch shape captures a new graph.  Slot i runs in lane i mod lanes.  Every
 * member computes exactly what it computes alone (its random numbers and
 * charge sums depend on it alone).  The other pm_batch_* calls apply; n_cases
 * reports the slots and an empty slot has no workgroups.  Lengths of the work
 * lists are fixed for the current device: pm_batch_slots_footprint must be
 * called with it current. */
size_t pm_batch_slots_footprint(int32_t n_slots, int32_t fp64);

/* An empty slotted batch for cases of precision fp64, steps_per_cycle steps per
 * RF cycle and at most max_cells cells (PM_EINVAL otherwise, PM_ENOSPACE for a
 * short arena).  Synchronises hip_stream. */
pm_status pm_batch_create_slots(int32_t n_slots, int32_t fp64, int32_t steps_per_cycle, int32_t max_cells,
                                void* dev_arena, size_t arena_bytes, void* hip_stream, pm_batch** out);

/* Put case c in slot (NULL: empty the slot).  PM_EINVAL for a slot out of range,
 * a case of another precision, steps per cycle or more cells than the batch's,
 * a case with flux profiles, or one already in another slot; PM_ESTATE for a
 * failed case.  The slot's previous case stays the caller's.  Synchronises
 * hip_stream (no step of the old membership may still run). */
pm_status pm_batch_set_slot(pm_batch* b, int32_t slot, pm_case* c, void* hip_stream);

/* --- measurement --------------------------------------------------------------
 * Advance n_steps steps with plain launches (the sorting schedule of pm_step),
 * bracketing every push and collision launch with HIP events on the stream it
 * runs on, and return the average duration of each kind of launch in ms.  A
 * batch runs its lanes one after another here, so each launch has the device
 * to itself.  Synchronises. */
pm_status pm_time_kernels(pm_case* c, int32_t n_steps, void* hip_stream, double* push_ms, double* mcc_ms);
pm_status pm_batch_time_kernels(pm_batch* b, int32_t n_steps, void* hip_stream, double* push_ms,
                                double* mcc_ms);

/* The library's generator (Philox4x64-10; Salmon et al., SC'11), from which
 * every random sample of the method is drawn (loading, the waits of Eq. (5),
 * the selection after Eq. (6), scattering angles, the sputter source): for
 * 0 <= i < n, out_dev[4 i .. 4 i + 3] receive the four output words for the
 * counter (id0 + i, index, tag, aux) under the key (seed, stream_key).
 * out_dev: device array of 4 n words (caller-owned).  PM_EINVAL for n < 0 or
 * a null array with n > 0.  Asynchronous on hip_stream.  For checking the
 * generator against an independent implementation. */
pm_status pm_philox_words(uint64_t id0, uint64_t index, uint64_t tag, uint64_t aux, uint64_t seed,
                          uint64_t stream_key, int64_t n, uint64_t* out_dev, void* hip_stream);

const char* pm_status_string(pm_status s);

#ifdef __cplusplus
}
#endif
#endif /* PICMCC_H */
