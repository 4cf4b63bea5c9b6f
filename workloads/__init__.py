"""Seeded synthetic workloads: parameter sets only, no arithmetic of the method.

Both the oracle (tests, CPU baseline) and the GPU path (tests, bench) take their
inputs from here.  The paper states the physics of its example discharge
(Sec. III) but no particle counts, grid or time step and no data set; these
workloads stand in for it with analytic cross sections:

  discharge_small   25 mm gap, 64 cells, 5k + 5k particles, 100 V, Ar 1 Pa 300 K,
                    dt = T_rf / 400, 50 RF cycles, FP64 particles.
  discharge_working 40 mm gap, 1024 cells, 1M + 1M particles, 300 V, Ar 0.5 Pa
                    300 K, dt = T_rf / 2000, 500 RF cycles, FP32 particles.
  discharge_paper   the Sec. III example: 75 mm gap, Ar 0.5 Pa 650 K, two harmonics
                    (V0 = 300 V, dphi = 0) through a blocking capacitor; 512 cells,
                    dt = T_rf / 2000, 2e5 + 2e5 particles, FP32 particles.
  sputter_transport 1e7 Al atoms, Thompson U_s = 3.4 eV cut at 200 eV, cosine
                    law, 40 mm gap, 100 mm periodic lateral, VHS Ar at 300 K,
                    0.5-5 Pa, omega = 0.8, d_ref = 3.6e-10 m, T_ref = 273 K.
  sweep_cases       64 discharges: p log-uniform 0.5-10 Pa, V0 uniform 50-500 V,
                    cells in {128, 256, 512, 1024}, 2e4-5e5 particles per species,
                    dt = T_rf / 1000.
  served stream     Poisson arrivals (4 per s); half discharges drawn as in the
                    sweep, half test-particle jobs of 1e5-1e6 atoms at 0.5-5 Pa.

All workloads share the e-Ar and Ar+-Ar cross sections: elastic 1e-19 m^2,
excitation threshold 11.5 eV and ionisation threshold 15.8 eV with
2.5e-20 ln(x)/x m^2, charge exchange 5e-19 m^2.
"""
import math

import numpy as np

BASE_SEED = 1607

XSEC = dict(sigma_el=1e-19, eth_exc=11.5, sigma0_exc=2.5e-20,
            eth_ion=15.8, sigma0_ion=2.5e-20, sigma_cx=5e-19)

AL_AMU = 26.9815385
AR_AMU = 39.948


def discharge(gap_m, n_cells, v0, steps_per_cycle, p_pa, np_each, n0, t_gas_k=300.0,
              seed=BASE_SEED, case_id=0, fp64=False, flags=0, capacity_factor=4,
              sort_interval=25):
    """A discharge case: 13.56 MHz sinusoid V0 sin(omega t) on the left electrode."""
    p = dict(gap_m=gap_m, n_cells=n_cells, freq_hz=13.56e6, v0_volt=float(v0),
             phase_rad=-math.pi / 2, steps_per_cycle=steps_per_cycle, p_pa=float(p_pa),
             t_gas_k=t_gas_k, n0_m3=n0, np_e=int(np_each), np_i=int(np_each),
             te_ev=2.0, ti_ev=0.026,
             capacity_e=int(capacity_factor * np_each), capacity_i=int(capacity_factor * np_each),
             ecap_e_ev=2.0 * v0 + 100.0, ecap_i_ev=2.0 * v0 + 100.0,
             seed=seed, case_id=case_id, flags=flags, fp64=int(fp64),
             sort_interval=sort_interval)
    p.update(XSEC)
    return p


def discharge_small(seed=1, **kw):
    """Plain 1D3V PIC/MCC argon CCP, 25 mm, 64 cells, 5k + 5k, FP64 (50 RF cycles)."""
    kw.setdefault("fp64", True)
    return discharge(0.025, 64, 100.0, 400, 1.0, 5000, 1e15, seed=seed, case_id=1, **kw)


def discharge_working(seed=BASE_SEED, np_each=1_000_000, **kw):
    """Single discharge at working size, 40 mm, 1024 cells, 1M + 1M (500 RF cycles)."""
    return discharge(0.04, 1024, 300.0, 2000, 0.5, np_each, 4e15, seed=seed, case_id=2, **kw)


def discharge_paper(seed=BASE_SEED, np_each=200_000, delta_phi=0.0, **kw):
    """The example discharge of Sec. III: 75 mm gap, Ar 0.5 Pa at 650 K, the
    electrical-asymmetry drive V0 [cos(wt + dphi) + cos(2wt)] with V0 = 300 V at
    13.56 MHz through a blocking capacitor, with the grid, step and particle count
    chosen here: 512 cells, dt = T_rf / 2000, 2e5 + 2e5 particles at
    n0 = 4e15 m^-3, FP32 particles.  The paper's 1 uF is for an electrode area it
    does not give; per m^2, 2e-8 F (about ten times a 5 mm sheath's eps0 / s) keeps
    the capacitor's share of the RF voltage under a tenth and lets the DC
    self-bias build within a few hundred RF cycles (a larger capacitor gives the
    same bias, more slowly)."""
    p = discharge(0.075, 512, 300.0, 2000, 0.5, np_each, 4e15, t_gas_k=650.0, seed=seed, case_id=5, **kw)
    p.update(v2_volt=300.0, phase_rad=float(delta_phi), phase2_rad=0.0, cb_f_m2=2e-8,
             ecap_e_ev=1300.0, ecap_i_ev=1300.0)
    return p


RF_CYCLES = {"discharge_small": 50, "discharge_working": 500, "sweep": 200}


def sputter_transport(p_pa=0.5, n_atoms=10_000_000, seed=BASE_SEED, job_id=3, mode=0):
    """(source, flight parameters) of the sputtered-atom transport workload."""
    src = dict(n_atoms=int(n_atoms), u_s_ev=3.4, e_cut_ev=200.0, seed=seed, job_id=job_id)
    tp = dict(p_pa=float(p_pa), t_gas_k=300.0, d_ref=3.6e-10, omega=0.8, t_ref=273.0,
              m_test_amu=AL_AMU, m_gas_amu=AR_AMU, gap_m=0.04, lateral_m=0.1, mode=mode,
              e_max=1_000_000, n_ebins=200, ebin_ev=1.0, n_tbins=200, tbin_s=5e-6, n_xbins=100)
    return src, tp


def sweep_case(rng, case_id, seed=BASE_SEED):
    """One discharge of the sweep's distribution, drawn from rng."""
    p_pa = math.exp(rng.uniform(math.log(0.5), math.log(10.0)))
    v0 = rng.uniform(50.0, 500.0)
    n_cells = int(rng.choice([128, 256, 512, 1024]))
    np_each = int(math.exp(rng.uniform(math.log(2e4), math.log(5e5))))
    return discharge(0.04, n_cells, v0, 1000, p_pa, np_each, 4e15, seed=seed, case_id=case_id)


def sweep_cases(n=64, seed=BASE_SEED):
    """The batched parameter sweep: n cases drawn from a seeded numpy generator."""
    rng = np.random.default_rng(seed)
    return [sweep_case(rng, 100 + k, seed) for k in range(n)]


def served_discharge(i, rng):
    """A served discharge request: drawn as in the sweep, case_id 10000 + i."""
    return sweep_case(rng, 10000 + i)


def served_tpm(i, rng):
    """A served test-particle job: 1e5-1e6 atoms and 0.5-5 Pa, both log-uniform."""
    n_atoms = int(math.exp(rng.uniform(math.log(1e5), math.log(1e6))))
    p_pa = math.exp(rng.uniform(math.log(0.5), math.log(5.0)))
    src, tp = sputter_transport(p_pa=p_pa, n_atoms=n_atoms, job_id=10000 + i)
    return {"src": src, "tp": tp}
