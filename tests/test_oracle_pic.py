"""The PIC/MCC oracle against closed forms, library routines and the paper's
printed gas density (CPU only)."""
import os

import numpy as np

from oracle import constants as C
from oracle import pic as P
import workloads as W
from tests import oracle_pins as pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_gas_density_printed_value():
    # Sec. III prints n_Ar ~ 5.57e13 cm^-3 for 0.5 Pa and 650 K
    rows = np.loadtxt(os.path.join(GOLDEN, "gas_density.txt"), ndmin=2)
    for p_pa, t_k, n_cm3, digits in rows:
        n = C.gas_density(p_pa, t_k) * 1e-6
        assert abs(n - n_cm3) <= 0.5 * 10 ** (np.floor(np.log10(n_cm3)) - digits + 1)


def test_deposit_exact():
    pins.check_deposit_exact()


def test_poisson_uniform_rho_is_exact_parabola():
    pins.check_poisson_uniform_rho_exact()
    pins.check_poisson_uniform_rho_exact(N=1024, L=0.04, V=-300.0, q=-7 * 2 ** 33)


def test_poisson_random_matches_dense_solve():
    pins.check_poisson_random_vs_dense()


def test_gather_linear_field_exact():
    pins.check_gather_linear_exact()


def test_uniform_field_trajectory():
    pins.check_uniform_field_trajectory()


def test_time_centred_energy_conserved():
    pins.check_time_centred_energy_conserved()


def test_ionisation_cross_section_peak():
    pins.check_ionisation_peak()


def test_null_collision_selection_frequencies():
    pins.check_null_collision_selection()


def test_first_collision_hazard_over_many_steps():
    pins.check_first_collision_law()


def test_skip_schedule_is_geometric():
    pins.check_skip_law()
    pins.check_skip_law(p_tot=0.3, n=200000)


def test_two_harmonic_waveform():
    pins.check_two_harmonic_waveform()


def test_blocking_capacitor_vacuum_divider():
    pins.check_circuit_vacuum_divider()


def test_blocking_capacitor_limit_is_the_ideal_source():
    pins.check_circuit_large_capacitor_is_the_ideal_source()


def test_skip_cut_and_redraw_keep_the_geometric_law():
    pins.check_skip_cap_memoryless()


def test_cut_wait_examination_only_redraws():
    pins.check_redraw_examination_only_redraws()


def test_collision_kinematics():
    pins.check_elastic_excitation_ionisation_kinematics()


def test_charge_exchange_thermalises():
    pins.check_charge_exchange_thermalises()


def test_loading_moments():
    pins.check_loading_moments()


def test_density_normalisation():
    pins.check_density_normalisation()


def test_nu_max_is_the_cap_value_for_monotone_sum():
    p = W.discharge_working()
    d = P.derived(p)
    at_cap = float(P.nu_sum_electron(np.array([p["ecap_e_ev"]]), p, d["n_gas"])[0])
    assert d["nu_max"][0] == at_cap


def test_small_run_is_deterministic_and_conserves_counts():
    p = W.discharge_small()
    a = P.Discharge(p)
    b = P.Discharge(p)
    a.run(40)
    b.run(40)
    for s in (0, 1):
        assert np.array_equal(a.sp[s].xt, b.sp[s].xt)
        assert np.array_equal(a.sp[s].id, b.sp[s].id)
    acc = a.acc
    n_e = len(a.sp[0])
    n_i = len(a.sp[1])
    assert n_e == p["np_e"] - acc["absorbed"][0].sum() + acc["births"] // 2
    assert n_i == p["np_i"] - acc["absorbed"][1].sum() + acc["births"] // 2


def test_flux_over_density_is_the_beam_velocity():
    pins.check_flux_over_density_is_the_beam_velocity()


def test_phase_bins_resolve_the_drive():
    pins.check_phase_bins_resolve_the_drive()


def test_iead_of_a_known_beam():
    pins.check_iead_of_a_known_beam()


def test_charge_exchange_rate_is_n_sigma_g_over_the_majorant():
    pins.check_charge_exchange_rate()


def test_ion_majorant_bounds_the_capped_energy():
    pins.check_ion_majorant_bounds_the_capped_energy()


def test_wall_flux_and_impact_energy_of_a_uniform_beam():
    pins.check_wall_flux_and_impact_energy()


def test_failures_are_flagged_per_case():
    """The oracle's failure flags, as the library's: a NaN velocity makes the
    case ENUMERIC at the next step; births beyond the slots make it ECAPACITY;
    a neighbour stepped beside it is untouched (each case is its own object)."""
    p = W.discharge_small(seed=9)
    ok, nan = P.Discharge(p), P.Discharge(p)
    nan.sp[0].v[17, 0] = np.nan
    ok.step()
    nan.step()
    assert nan.status == P.ENUMERIC and ok.status == P.OK
    q = W.discharge(0.025, 64, 500.0, 1000, 10.0, 2000, 1e15, seed=3, case_id=1)
    q.update(capacity_e=2001, capacity_i=2001)
    full = P.Discharge(q)
    for _ in range(200):
        full.step()
        if full.status != P.OK:
            break
    assert full.status == P.ECAPACITY
    assert len(full.sp[0]) > 2001 or len(full.sp[1]) > 2001
