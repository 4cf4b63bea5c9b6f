"""Plant plausible mistakes in the oracle (on the CPU) and check that a pin fails.

Each case monkeypatches one oracle function with a wrong variant: a dropped
term, a wrong sign or index, a transposed operand.  A pin that still passed
would be too weak to trust.
"""
import math

import numpy as np
import pytest

from oracle import pic as P
from oracle import tpm as T
from tests import oracle_pins as pins
from tests import test_oracle_tpm as tpm_tests


def _charge_density_full_boundary_cells(Qe, Qi, w, dx, N):
    from oracle import constants as C
    return C.E_CHARGE * w * (Qi - Qe).astype(np.float64) / (2 ** 32 * dx)


def _field_wrong_sign(Phi, rho, dx):
    E = P.__dict__["_orig_electric_field"](Phi, rho, dx)
    E[1:-1] = -E[1:-1]
    return E


def _field_no_boundary_charge(Phi, rho, dx):
    N = Phi.size - 1
    E = np.empty(N + 1)
    E[1:N] = -(Phi[2:] - Phi[:-2]) / (2.0 * dx)
    E[0] = (Phi[0] - Phi[1]) / dx
    E[N] = (Phi[N - 1] - Phi[N]) / dx
    return E


def _deposit_floor(xt, N):
    xt = np.asarray(xt, dtype=np.float64)
    j = np.floor(xt).astype(np.int64)
    W = np.floor((xt - j) * 2 ** 32).astype(np.int64)
    Q = np.zeros(N + 1, dtype=np.int64)
    np.add.at(Q, j, 2 ** 32 - W)
    np.add.at(Q, j + 1, W)
    return Q


def _gather_swapped(E, xt):
    j = np.floor(xt).astype(np.int64)
    f = xt - j
    return f * E[j] + (1.0 - f) * E[j + 1]


def _iso_half_angle(Ua, Ub):
    chi = np.arccos(np.sqrt(Ua))
    psi = 2.0 * np.pi * Ub
    return np.stack([np.cos(chi), np.sin(chi) * np.cos(psi), np.sin(chi) * np.sin(psi)], axis=-1)


def _thompson_linear(U, u_s, e_cut):
    s_max = e_cut / (e_cut + u_s)
    s = U * s_max
    return u_s * s / (1.0 - s)


def _skip_off_by_one(U, step, p_tot, wait_cap=None):
    nxt, redraw, tie = P.__dict__["_orig_skip"](U, step, p_tot, wait_cap)
    return nxt + 1, redraw, tie


def _skip_cut_without_redraw(U, step, p_tot, wait_cap=None):
    nxt, redraw, tie = P.__dict__["_orig_skip"](U, step, p_tot, wait_cap)
    return nxt, np.zeros_like(redraw), tie         # the cut wait taken as a real test


def _circuit_capacitor_sign(rho, dx, cb, sigma_rhs):
    return P.__dict__["_orig_solve_potential_circuit"](rho, dx, -cb, sigma_rhs)


def _flux_weights_swapped(xt, vx, N):
    # node floor(x) given f and the next node 1 - f
    xt = np.asarray(xt, dtype=np.float64)
    j = np.floor(xt).astype(np.int64)
    f = xt - j
    F = np.zeros(N + 1)
    np.add.at(F, j, f * vx)
    np.add.at(F, j + 1, (1.0 - f) * vx)
    return F


def _flux_weights_after_push(xt, vx, N):
    # sampled a quarter cell along the drift, as if taken after the push
    xt = np.clip(np.asarray(xt, dtype=np.float64) + 0.25 * np.sign(vx), 0.0, N - 1e-9)
    return P.__dict__["_orig_flux_weights"](xt, vx, N)


def _phase_bin_rounded(l, steps_per_cycle, n_phase):
    return int(round((l % steps_per_cycle) * n_phase / steps_per_cycle)) % n_phase


def _phase_bin_next_step(l, steps_per_cycle, n_phase):
    return P.__dict__["_orig_phase_bin"](l + 1, steps_per_cycle, n_phase)


MUTATIONS = [
    ("charge_density", _charge_density_full_boundary_cells, pins.check_poisson_uniform_rho_exact),
    ("electric_field", _field_wrong_sign, pins.check_poisson_uniform_rho_exact),
    ("electric_field", _field_no_boundary_charge, pins.check_poisson_uniform_rho_exact),
    ("deposit", _deposit_floor, pins.check_deposit_exact),
    ("gather", _gather_swapped, pins.check_gather_linear_exact),
    ("isotropic_direction", _iso_half_angle, pins.check_elastic_excitation_ionisation_kinematics),
    ("skip", _skip_off_by_one, pins.check_skip_law),
    ("skip", _skip_off_by_one, pins.check_first_collision_law),
    ("skip", _skip_cut_without_redraw, pins.check_skip_cap_memoryless),
    ("solve_potential_circuit", _circuit_capacitor_sign, pins.check_circuit_vacuum_divider),
    ("flux_weights", _flux_weights_swapped, pins.check_flux_over_density_is_the_beam_velocity),
    ("flux_weights", _flux_weights_after_push, pins.check_flux_over_density_is_the_beam_velocity),
    ("phase_bin", _phase_bin_rounded, pins.check_phase_bins_resolve_the_drive),
    ("phase_bin", _phase_bin_next_step, pins.check_phase_bins_resolve_the_drive),
]


@pytest.mark.parametrize("name,bad,check", MUTATIONS, ids=[f"{m[0]}-{m[1].__name__}" for m in MUTATIONS])
def test_pin_catches_planted_mistake(monkeypatch, name, bad, check):
    monkeypatch.setitem(P.__dict__, "_orig_" + name, getattr(P, name))
    monkeypatch.setattr(P, name, bad)
    with pytest.raises(AssertionError):
        check()


def test_pin_catches_wrong_leapfrog_order(monkeypatch):
    # position advanced with the old velocity v^(l-1/2) instead of v^(l+1/2)
    orig = P.Discharge.step

    def bad_step(self, record=False):
        olds = [sp.v[:, 0].copy() for sp in self.sp]
        rec = orig(self, record)
        for sp, v_old in zip(self.sp, olds):
            if sp.xt.size == v_old.size:
                sp.xt = sp.xt - (sp.v[:, 0] - v_old) * self.d["dt"] / self.d["dx"]
        return rec

    monkeypatch.setattr(P.Discharge, "step", bad_step)
    with pytest.raises(AssertionError):
        pins.check_uniform_field_trajectory()


def test_pin_catches_wrong_thompson_inversion(monkeypatch):
    monkeypatch.setattr(T, "thompson_energy", _thompson_linear)
    with pytest.raises(AssertionError):
        tpm_tests.test_thompson_source_law()


def test_pin_catches_wrong_process_order(monkeypatch):
    from oracle import xsec

    def swapped(eps_ev, xs):
        s_el, s_exc, s_ion = xsec.electron_sigmas(eps_ev, xs)
        return s_el, s_ion, s_exc

    monkeypatch.setattr(P, "electron_sigmas", swapped)
    with pytest.raises(AssertionError):
        pins.check_null_collision_selection()


def _overlaps_full_cells_only(xa, xb, n_bins, L):
    """Wrong: only cells crossed end to end are counted (partial cells dropped)."""
    dx = L / n_bins
    lo, hi = np.minimum(xa, xb)[:, None], np.maximum(xa, xb)[:, None]
    edges = np.arange(n_bins + 1) * dx
    return np.where((lo <= edges[None, :-1]) & (hi >= edges[None, 1:]), dx, 0.0)


def _overlaps_shifted(xa, xb, n_bins, L):
    """Wrong: every flight tallied one cell too far towards the substrate."""
    ov = T.__dict__["_orig_cell_overlaps"](xa, xb, n_bins, L)
    return np.roll(ov, 1, axis=1)


@pytest.mark.parametrize("bad", [_overlaps_full_cells_only, _overlaps_shifted])
def test_pin_catches_wrong_track_tally(monkeypatch, bad):
    monkeypatch.setitem(T.__dict__, "_orig_cell_overlaps", T.cell_overlaps)
    monkeypatch.setattr(T, "cell_overlaps", bad)
    failed = 0
    for pin in (tpm_tests.test_cell_overlaps_match_brute_force,
                lambda: tpm_tests.test_profiles_add_up_to_the_flight_times_and_displacements(0.5)):
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed >= 1


def test_pin_catches_reversed_m1_deflection(monkeypatch):
    # chi and pi - chi swapped: forward and backward scattering exchanged
    orig = T.rotate_relative
    monkeypatch.setattr(T, "rotate_relative", lambda g, chi, psi: orig(g, np.pi - chi, psi))
    from tests import test_oracle_tpm as tt
    with pytest.raises(AssertionError):
        tt.check_m1_deflection_law()


def test_pin_catches_exponential_step_probability(monkeypatch):
    # 1 - exp(-n sigma g dt) in place of the linearised Eq. (7)
    monkeypatch.setattr(T, "collision_probability", lambda n, sg, dt: -np.expm1(-n * sg * dt))
    with pytest.raises(AssertionError):
        tpm_tests.test_fixed_step_collides_with_the_linear_probability()


def test_pin_catches_yield_pieces_restarting_the_impact_index(monkeypatch):
    # each piece keys its impacts from 0 again: the pieces re-use the first
    # impacts' draws instead of the new ones'
    orig = T.sputtered_count

    def restarted(iedf, yld, seed, job_id, ebin_ev=1.0, electrode=0, taken=None):
        new = np.asarray(iedf) - (0 if taken is None else np.asarray(taken))
        return orig(new, yld, seed, job_id, ebin_ev=ebin_ev, electrode=electrode)

    monkeypatch.setattr(T, "sputtered_count", restarted)
    with pytest.raises(AssertionError):
        tpm_tests.check_yield_count_in_pieces()


def test_pin_catches_charge_exchange_partner_at_rest(monkeypatch):
    # the ion's collision partner taken at rest (relative speed = ion speed)
    from oracle import philox as R
    monkeypatch.setattr(R, "maxwell_velocity", lambda U, sig: np.zeros((U.shape[0], 3)))
    with pytest.raises(AssertionError):
        pins.check_charge_exchange_rate(n=100000)


def test_pin_catches_ion_majorant_without_thermal_margin(monkeypatch):
    # nu_max of the ions from the capped ion speed alone (the partner's motion dropped)
    from oracle import constants as C

    def bad(p, d):
        return d["n_gas"] * p["sigma_cx"] * math.sqrt(2.0 * p["ecap_i_ev"] * C.E_CHARGE / C.M_AR)

    monkeypatch.setattr(P, "nu_max_ion", bad)
    with pytest.raises(AssertionError):
        pins.check_ion_majorant_bounds_the_capped_energy()


@pytest.mark.parametrize("mistake", ["steps_plus_one", "energy_over_all_absorbed", "electrodes_swapped"])
def test_pin_catches_wrong_wall_normalisation(monkeypatch, mistake):
    orig = P.Discharge.sample_diagnostics

    def bad(self):
        out = orig(self)
        a = self.acc
        if mistake == "steps_plus_one":          # the window counted one step too long
            out["flux"] = a["absorbed"] * self.d["w"] / ((a["n_steps"] + 1) * self.d["dt"])
        elif mistake == "energy_over_all_absorbed":                                    # energy divided by the impacts of both species
            out["mean_ion_energy"] = a["ion_energy_sum"] / np.maximum(a["absorbed"].sum(axis=0), 1)
        if mistake == "electrodes_swapped":      # fluxes booked at the other electrode
            out["flux"] = out["flux"][:, ::-1]
        return out

    monkeypatch.setattr(P.Discharge, "sample_diagnostics", bad)
    with pytest.raises(AssertionError):
        pins.check_wall_flux_and_impact_energy()


def _tally_rounded(wall, E, theta, tof, tp):
    # energies binned to the nearest bin edge instead of the bin they fall in
    r = T.__dict__["_orig_tally"](wall, E, theta, tof, tp)
    sub = wall == T.WALL_SUBSTRATE
    nb = int(tp["n_ebins"])
    r["e_hist"] = np.bincount(np.minimum(np.rint(E[sub] / tp["ebin_ev"]).astype(np.int64), nb - 1), minlength=nb)
    return r


def _tally_target_in_histograms(wall, E, theta, tof, tp):
    # the target's atoms added to the substrate's histograms
    w2 = np.where(wall == T.WALL_TARGET, T.WALL_SUBSTRATE, wall)
    r = T.__dict__["_orig_tally"](w2, E, theta, tof, tp)
    r.update({k: v for k, v in T.__dict__["_orig_tally"](wall, E, theta, tof, tp).items() if not k.endswith("hist")})
    return r


@pytest.mark.parametrize("bad", [_tally_rounded, _tally_target_in_histograms])
def test_pin_catches_wrong_tally_bins(monkeypatch, bad):
    monkeypatch.setitem(T.__dict__, "_orig_tally", T.tally)
    monkeypatch.setattr(T, "tally", bad)
    with pytest.raises(AssertionError):
        tpm_tests.check_tally_bins_of_known_atoms()


def test_pin_catches_wait_and_acceptance_sharing_one_uniform(monkeypatch):
    # the acceptance test reads the uniform the candidate wait was drawn from
    import types
    from oracle import philox as R

    def draw(*a, **k):
        U = R.draw(*a, **k).copy()
        U[:, 5] = U[:, 0]
        return U

    shim = types.SimpleNamespace(**{k: getattr(R, k) for k in dir(R) if not k.startswith("__")})
    shim.draw = draw
    monkeypatch.setattr(T, "R", shim)
    with pytest.raises(AssertionError):
        tpm_tests.check_uncollided_transmission(0.5)


def test_pin_catches_candidate_rate_below_the_majorant(monkeypatch):
    # candidate events at half the rate that the acceptance test assumes
    orig = T.majorant
    monkeypatch.setattr(T, "majorant", lambda src, tp: (orig(src, tp)[0], 0.5 * orig(src, tp)[1]))
    with pytest.raises(AssertionError):
        tpm_tests.check_uncollided_transmission(0.5)


def test_pin_catches_m1_flight_with_the_vhs_diameter(monkeypatch):
    # M1 atoms flown with the VHS reference diameter (the sqrt(4/3) factor dropped)
    monkeypatch.setattr(T, "d_ref_of", lambda tp: tp["d_ref"])
    with pytest.raises(AssertionError):
        tpm_tests.check_uncollided_transmission(0.5, scatter=T.SCATTER_M1)
