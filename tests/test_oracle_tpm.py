"""The test-particle oracle against closed forms and numerical integrals (CPU only)."""
import math

import numpy as np
import pytest
from scipy import integrate, optimize, stats

from oracle import constants as C
from oracle import tpm as T
from oracle.xsec import vhs_sigma
import workloads as W


def _thompson_density(E, U):
    return E / (E + U) ** 3


def _thompson_cdf_quad(U, cut):
    Z = integrate.quad(_thompson_density, 0, cut, args=(U,))[0]
    return lambda E: np.array([integrate.quad(_thompson_density, 0, e, args=(U,))[0] / Z
                               for e in np.atleast_1d(E)])


def test_thompson_source_law():
    src, tp = W.sputter_transport(n_atoms=200000)
    _, _, v, E = T.source(200000, src, tp)
    U, cut = src["u_s_ev"], src["e_cut_ev"]
    Z = integrate.quad(_thompson_density, 0, cut, args=(U,))[0]
    mean = integrate.quad(lambda e: e * _thompson_density(e, U), 0, cut)[0] / Z
    assert abs(mean - 18.460) < 5e-3                         # closed-form value
    cdf = _thompson_cdf_quad(U, cut)
    median = optimize.brentq(lambda e: cdf(e)[0] - 0.5, 0.1, cut)
    assert abs(median - 7.758) < 5e-3
    assert E.max() <= cut and E.min() > 0
    assert abs(E.mean() / mean - 1) < 0.01
    assert abs(np.median(E) / median - 1) < 0.01
    sub = np.sort(E[:4000])
    assert stats.kstest(sub, lambda e: cdf(e)).pvalue > 1e-4
    # the speed follows from the energy
    m = W.AL_AMU * C.AMU
    assert np.allclose(0.5 * m * np.sum(v ** 2, axis=1) / C.E_CHARGE, E, rtol=1e-12)


def test_cosine_emission_law():
    src, tp = W.sputter_transport()
    _, pos, v, _ = T.source(200000, src, tp)
    c = v[:, 0] / np.linalg.norm(v, axis=1)
    assert np.all(c > 0)
    assert abs(c.mean() - 2 / 3) < 3e-3
    assert abs((c ** 2).mean() - 1 / 2) < 3e-3
    # P(theta <= theta0) = sin^2 theta0, i.e. 1 - cos^2 theta is uniform
    assert stats.kstest(1 - c ** 2, "uniform").pvalue > 1e-4
    assert np.all(pos[:, 0] == 0) and np.all((pos[:, 1:] >= 0) & (pos[:, 1:] < tp["lateral_m"]))


def test_vhs_hard_sphere_limit_and_scaling():
    d = 3.6e-10
    g = np.array([10.0, 300.0, 3e4])
    assert np.allclose(vhs_sigma(g, 1e-26, d, 0.5, 273.0), math.pi * d * d, rtol=1e-14)
    mr = 16.1 * C.AMU
    # at 2 k T_ref / (m_r g^2) = 1 the power-law factor is 1
    g1 = math.sqrt(2 * C.K_B * 273.0 / mr)
    assert abs(vhs_sigma(g1, mr, d, 0.8, 273.0) / (math.pi * d * d / math.gamma(1.7)) - 1) < 1e-12
    s = vhs_sigma(np.array([100.0, 200.0]), mr, d, 0.8, 273.0)
    assert abs(s[1] / s[0] - 2.0 ** (1 - 2 * 0.8)) < 1e-12


def test_ballistic_flight_is_exact():
    src, tp = W.sputter_transport(p_pa=0.0, n_atoms=20000)
    res = T.run(src, tp, trace=True)
    assert res["n_substrate"] == 20000 and res["n_target"] == 0 and res["n_unfinished"] == 0
    tr = res["trace"]
    _, _, v, E = T.source(20000, src, tp)
    assert np.allclose(tr["E"], E, rtol=1e-12)
    assert np.allclose(tr["tof"], tp["gap_m"] / v[:, 0], rtol=1e-12)
    c = np.cos(np.radians(tr["theta"]))
    assert abs(c.mean() - 2 / 3) < 0.01


def test_deposition_fraction_falls_with_pressure():
    eta = []
    for p in (0.5, 2.0):
        src, tp = W.sputter_transport(p_pa=p, n_atoms=3000)
        r = T.run(src, tp)
        assert r["n_substrate"] + r["n_target"] + r["n_unfinished"] == 3000
        eta.append(r["n_substrate"] / 3000)
    assert eta[0] > eta[1] + 0.1


def _box(p_pa, e_max, n):
    src, tp = W.sputter_transport(p_pa=p_pa, n_atoms=n, mode=T.MODE_BOX)
    tp["e_max"] = e_max
    return T.run(src, tp, trace=True), tp


def test_box_thermalises_and_collides_at_the_vhs_equilibrium_rate():
    n = 4000
    r1, tp = _box(0.5, 600, n)
    r2, _ = _box(0.5, 1200, n)
    m, M = T.masses(tp)
    kT = C.K_B * tp["t_gas_k"]
    # thermalisation: <0.5 m v^2> = 1.5 k T and a Maxwell speed law
    v = r2["trace"]["v"]
    ke = 0.5 * m * np.sum(v ** 2, axis=1)
    assert abs(ke.mean() / (1.5 * kT) - 1) < 0.04
    speed = np.linalg.norm(v, axis=1)
    assert stats.kstest(speed, "maxwell", args=(0, math.sqrt(kT / m))).pvalue > 1e-4
    # equilibrium real-collision rate n <sigma g> of VHS (derived closed form)
    mr = m * M / (m + M)
    n_gas = C.gas_density(tp["p_pa"], tp["t_gas_k"])
    nu_eq = n_gas * 2 * math.sqrt(math.pi) * tp["d_ref"] ** 2 * math.sqrt(2 * kT / mr) \
        * (tp["t_ref"] / tp["t_gas_k"]) ** (tp["omega"] - 0.5)
    assert abs(nu_eq / 3.00e4 - 1) < 0.01
    rate = (r2["collisions"] - r1["collisions"]) / (r2["trace"]["tof"].sum() - r1["trace"]["tof"].sum())
    assert abs(rate / nu_eq - 1) < 0.03, (rate, nu_eq)


@pytest.mark.parametrize("Y", [1.0, 0.3, 2.5])
def test_yield_rule_expectation(Y):
    hist = np.zeros(700, dtype=np.int64)
    hist[250] = 40000
    hist[300] = 20000
    k = T.sputtered_count(hist, Y, seed=1, job_id=2)
    n = hist.sum()
    if Y == 1.0:
        assert k == n                                 # R_f <= 1 always succeeds
    else:
        N = math.ceil(Y)
        sd = math.sqrt(n * N * (Y / N) * (1 - Y / N))
        assert abs(k - n * Y) < 5 * sd


def check_yield_count_in_pieces(Y=0.3):
    """Impacts arriving in three stages: counting each stage's new impacts
    (taken = the record at the previous count) adds up to the count of the final
    record, and each stage alone has the binomial expectation Y per new impact."""
    rng = np.random.default_rng(8)
    stages = [rng.integers(0, 4000, 60) for _ in range(3)]
    rec = np.zeros(60, dtype=np.int64)
    parts = []
    for add in stages:
        taken = rec.copy()
        rec = rec + add
        k = T.sputtered_count(rec, Y, seed=5, job_id=6, taken=taken)
        n = int(add.sum())
        N = math.ceil(Y)
        sd = math.sqrt(n * N * (Y / N) * (1 - Y / N))
        assert abs(k - n * Y) < 5 * sd
        parts.append(k)
    assert sum(parts) == T.sputtered_count(rec, Y, seed=5, job_id=6)


def test_yield_count_in_pieces():
    check_yield_count_in_pieces()


def test_yield_table_interpolation():
    hist = np.zeros(10, dtype=np.int64)
    hist[4] = 50000                                  # bin centre 4.5 eV
    table = ([0.0, 9.0], [0.0, 1.8])                 # Y(4.5) = 0.9
    k = T.sputtered_count(hist, table, seed=3, job_id=4)
    assert abs(k / 50000 - 0.9) < 0.01


def test_ballistic_profiles_cross_every_cell_once():
    """Without gas every atom crosses every cell once: the residence time of a
    cell is the sum over atoms of dx / v_x, its displacement n_atoms * dx."""
    n = 5000
    src, tp = W.sputter_transport(p_pa=0.0, n_atoms=n)
    res = T.run(src, tp, trace=True)
    _, _, v, _ = T.source(n, src, tp)
    dx = tp["gap_m"] / tp["n_xbins"]
    want = np.sum(dx / v[:, 0])
    assert np.allclose(res["time_s"], want, rtol=1e-12)
    assert np.allclose(res["disp_m"], n * dx, rtol=1e-12)
    # density is uniform and equals the flux times the mean of 1 / v_x
    dens, ux = T.profiles(res, dict(src, flux_m2s=1e18), n, tp["gap_m"])
    assert np.allclose(dens, 1e18 * np.mean(1.0 / v[:, 0]), rtol=1e-12)
    assert np.allclose(ux, n / np.sum(1.0 / v[:, 0]), rtol=1e-12)       # harmonic mean of v_x


@pytest.mark.parametrize("p_pa", [0.5, 2.0])
def test_profiles_add_up_to_the_flight_times_and_displacements(p_pa):
    """With collisions the cell times add up to the total time in flight of all
    atoms, and the displacements to L per substrate atom (0 per target atom,
    the final x of an unfinished one)."""
    n = 2000
    src, tp = W.sputter_transport(p_pa=p_pa, n_atoms=n)
    tp["e_max"] = 300                       # leaves some atoms unfinished at 2 Pa
    res = T.run(src, tp, trace=True)
    tr = res["trace"]
    assert np.isclose(res["time_s"].sum(), tr["tof"].sum(), rtol=1e-10)
    unf = tr["wall"] == T.UNFINISHED
    want = tp["gap_m"] * res["n_substrate"] + tr["x"][unf].sum()
    assert np.isclose(res["disp_m"].sum(), want, rtol=1e-10, atol=1e-12)
    assert np.all(res["time_s"] > 0)


def test_cell_overlaps_match_brute_force():
    rng = np.random.default_rng(3)
    L, nb = 0.04, 17
    xa = rng.uniform(0, L, 50)
    xb = rng.uniform(0, L, 50)
    ov = T.cell_overlaps(xa, xb, nb, L)
    assert np.allclose(ov.sum(axis=1), np.abs(xb - xa), rtol=1e-12)
    # fine sampling of each flight
    for i in range(0, 50, 7):
        s = np.linspace(min(xa[i], xb[i]), max(xa[i], xb[i]), 200001)
        mid = 0.5 * (s[1:] + s[:-1])
        cnt = np.bincount(np.minimum((mid / (L / nb)).astype(int), nb - 1), minlength=nb) * (s[1] - s[0])
        assert np.allclose(ov[i], cnt, atol=2 * (s[1] - s[0]))


def test_rotation_keeps_speed_and_turns_by_chi():
    """rotate_relative: |g'| = |g|, the angle between g and g' is chi, and over a
    uniform azimuth the turned direction averages to cos(chi) g-hat."""
    rng = np.random.default_rng(4)
    n = 20000
    g = rng.normal(size=(n, 3)) * 300.0
    g[:3] = [[500.0, 0, 0], [-20.0, 0, 0], [0, 0, 7.0]]          # along the axes
    chi = rng.uniform(0, np.pi, n)
    psi = rng.uniform(0, 2 * np.pi, n)
    gp = T.rotate_relative(g, chi, psi)
    gm = np.linalg.norm(g, axis=1)
    assert np.allclose(np.linalg.norm(gp, axis=1), gm, rtol=1e-13)
    cosang = np.sum(g * gp, axis=1) / gm ** 2
    assert np.allclose(cosang, np.cos(chi), atol=1e-12)
    # one g, a fixed chi, many azimuths: the mean turned direction is cos(chi) g-hat
    g1 = np.tile(np.array([[1.0, -2.0, 0.5]]), (n, 1))
    d = T.rotate_relative(g1, np.full(n, 1.1), rng.uniform(0, 2 * np.pi, n)) / np.linalg.norm(g1[0])
    assert np.allclose(d.mean(axis=0), math.cos(1.1) * g1[0] / np.linalg.norm(g1[0]), atol=0.02)


def _m1_collisions(n=60000):
    src, tp = W.sputter_transport(p_pa=5.0, n_atoms=n, mode=T.MODE_BOX)
    tp.update(scatter=T.SCATTER_M1, e_max=1)
    return src, tp


def test_m1_deflection_law_and_viscosity_equivalence():
    """M1: chi = pi (1 - b / b_max) with b = b_max sqrt(R) gives P(chi <= x) =
    1 - (1 - x / pi)^2 and <sin^2 chi> = 1/2; with d_ref,M1 = sqrt(4/3) d_ref the
    viscosity cross section sigma_T <sin^2 chi> equals the isotropic VHS one,
    sigma_T * 2/3 ('Binary Interactions')."""
    check_m1_deflection_law()
    src, tp = _m1_collisions()
    ratio = (T.d_ref_of(tp) / tp["d_ref"]) ** 2
    assert abs(ratio * 0.5 - 2.0 / 3.0) < 1e-12


def check_m1_deflection_law(n=200000):
    """The deflection between the relative velocities before and after the oracle's
    M1 collision (recovered from the atom's velocities) has P(chi <= x) = 1 - (1 -
    x / pi)^2 and <sin^2 chi> = 1/2; the turned direction has a uniform azimuth."""
    rng = np.random.default_rng(9)
    m, M = 27.0, 40.0
    v = rng.normal(size=(n, 3)) * 2e3
    vbg = rng.normal(size=(n, 3)) * 300.0
    vp = T.scatter(v, vbg, rng.uniform(size=n), rng.uniform(size=n), m, M, T.SCATTER_M1)
    Vcm = (m * v + M * vbg) / (m + M)
    g = v - vbg
    gp = (vp - Vcm) * (m + M) / M
    assert np.allclose(np.linalg.norm(gp, axis=1), np.linalg.norm(g, axis=1), rtol=1e-10)
    ang = np.arccos(np.clip(np.sum(g * gp, axis=1) / np.sum(g * g, axis=1), -1, 1))
    assert stats.kstest(ang, lambda x: 1 - (1 - x / np.pi) ** 2).pvalue > 1e-4
    s2 = np.sin(ang) ** 2
    assert abs(s2.mean() - 0.5) < 4 * s2.std() / math.sqrt(n)
    # azimuth about g: uniform (the component along a fixed normal averages to 0)
    ghat = g / np.linalg.norm(g, axis=1)[:, None]
    perp = gp - np.sum(gp * ghat, axis=1)[:, None] * ghat
    e1 = np.cross(ghat, np.array([0.3, 0.5, 0.81]))
    e1 /= np.linalg.norm(e1, axis=1)[:, None]
    c = np.sum(perp * e1, axis=1) / np.maximum(np.linalg.norm(perp, axis=1), 1e-300)
    assert abs(c.mean()) < 4 / math.sqrt(2 * n) and abs(np.mean(c * c) - 0.5) < 0.01


def test_m1_box_thermalises_at_four_thirds_the_vhs_rate():
    """M1 conserves momentum and energy per collision, so the box still relaxes to
    the gas temperature; its cross section is 4/3 of VHS, so the equilibrium
    real-collision rate is 4/3 of the VHS closed form."""
    n = 4000
    res = []
    for e_max in (600, 1200):
        src, tp = W.sputter_transport(p_pa=0.5, n_atoms=n, mode=T.MODE_BOX)
        tp.update(e_max=e_max, scatter=T.SCATTER_M1)
        res.append(T.run(src, tp, trace=True))
    r1, r2 = res
    m, M = T.masses(tp)
    kT = C.K_B * tp["t_gas_k"]
    v = r2["trace"]["v"]
    ke = 0.5 * m * np.sum(v ** 2, axis=1)
    assert abs(ke.mean() / (1.5 * kT) - 1) < 0.04
    mr = m * M / (m + M)
    n_gas = C.gas_density(tp["p_pa"], tp["t_gas_k"])
    nu_vhs = n_gas * 2 * math.sqrt(math.pi) * tp["d_ref"] ** 2 * math.sqrt(2 * kT / mr) \
        * (tp["t_ref"] / tp["t_gas_k"]) ** (tp["omega"] - 0.5)
    rate = (r2["collisions"] - r1["collisions"]) / (r2["trace"]["tof"].sum() - r1["trace"]["tof"].sum())
    assert abs(rate / (4.0 / 3.0 * nu_vhs) - 1) < 0.03, (rate, nu_vhs)


def test_fixed_step_ballistic_flight_is_exact():
    """Fixed dt without gas: straight flights, the wall reached at the exact
    crossing time (the last step is cut at the wall)."""
    src, tp = W.sputter_transport(p_pa=0.0, n_atoms=5000)
    tp.update(dt_s=1e-7, e_max=10 ** 6)
    res = T.run(src, tp, trace=True)
    assert res["n_substrate"] == 5000
    _, _, v, E = T.source(5000, src, tp)
    tr = res["trace"]
    assert np.allclose(tr["tof"], tp["gap_m"] / v[:, 0], rtol=1e-12)
    assert np.array_equal(tr["events"], np.floor(tp["gap_m"] / v[:, 0] / 1e-7).astype(np.int64))


def test_fixed_step_collides_with_the_linear_probability():
    """Eq. (7): per step a thermalised atom collides with probability n <sigma g> dt
    -- linear in dt (0.30 here, where an exponential law would give 0.26) -- and the
    box still relaxes to the gas temperature."""
    n = 20000
    res = []
    for e_max in (400, 800):
        src, tp = W.sputter_transport(p_pa=0.5, n_atoms=n, mode=T.MODE_BOX)
        tp.update(e_max=e_max, dt_s=1.0e-5)
        res.append(T.run(src, tp, trace=True))
    m, M = T.masses(tp)
    kT = C.K_B * tp["t_gas_k"]
    v = res[1]["trace"]["v"]
    assert abs(0.5 * m * np.sum(v ** 2, axis=1).mean() / (1.5 * kT) - 1) < 0.03
    mr = m * M / (m + M)
    n_gas = C.gas_density(tp["p_pa"], tp["t_gas_k"])
    nu_eq = n_gas * 2 * math.sqrt(math.pi) * tp["d_ref"] ** 2 * math.sqrt(2 * kT / mr) \
        * (tp["t_ref"] / tp["t_gas_k"]) ** (tp["omega"] - 0.5)
    p_step = (res[1]["collisions"] - res[0]["collisions"]) / (n * 400)
    want = nu_eq * tp["dt_s"]
    assert abs(want - 0.30) < 0.01
    assert abs(p_step / want - 1) < 0.02, (p_step, want)


def test_substrate_emission_is_the_mirror_image():
    """Re-sputtered atoms leave the substrate (x = L) into -x: without gas each one
    reaches the target after L / |v_x|, with the same energies and angles as the
    target's emission of the same atom ids."""
    src, tp = W.sputter_transport(p_pa=0.0, n_atoms=5000)
    res_t = T.run(src, tp, trace=True)
    res_s = T.run(dict(src, electrode=1), tp, trace=True)
    assert res_s["n_target"] == 5000 and res_s["n_substrate"] == 0
    _, pos, v, E = T.source(5000, dict(src, electrode=1), tp)
    assert np.all(pos[:, 0] == tp["gap_m"]) and np.all(v[:, 0] < 0)
    tr = res_s["trace"]
    assert np.allclose(tr["tof"], res_t["trace"]["tof"], rtol=1e-12)
    assert np.allclose(tr["E"], res_t["trace"]["E"], rtol=1e-12)
    assert np.allclose(tr["theta"], res_t["trace"]["theta"], atol=1e-9)


def check_tally_bins_of_known_atoms():
    """Atoms of known wall, energy, angle and time of flight land in the bins
    their values name: bin k of width b holds [k b, (k + 1) b), the last bin also
    everything beyond it, angles in 1 degree bins; only substrate atoms enter the
    histograms, and the energy sums add the atoms of each wall."""
    tp = dict(W.sputter_transport()[1], n_ebins=50, ebin_ev=2.0, n_tbins=40, tbin_s=1e-6)
    E = np.array([0.1, 1.99, 2.0, 13.7, 99.9, 100.0, 512.0, 7.3, 40.0])
    th = np.array([0.0, 0.99, 1.0, 45.5, 89.99, 12.2, 3.0, 60.0, 1.5])
    tof = np.array([1e-8, 9.9e-7, 1.0e-6, 2.55e-5, 3.999e-5, 4.0e-5, 1e-3, 5e-6, 2e-6])
    wall = np.array([T.WALL_SUBSTRATE] * 7 + [T.WALL_TARGET, T.UNFINISHED])
    r = T.tally(wall, E, th, tof, tp)
    want_e = np.zeros(50, dtype=np.int64)
    want_t = np.zeros(90, dtype=np.int64)
    want_f = np.zeros(40, dtype=np.int64)
    # bins of the seven substrate atoms, written out
    for eb, ab, tb in ((0, 0, 0), (0, 0, 0), (1, 1, 1), (6, 45, 25), (49, 89, 39), (49, 12, 39), (49, 3, 39)):
        want_e[eb] += 1
        want_t[ab] += 1
        want_f[tb] += 1
    assert np.array_equal(r["e_hist"], want_e)
    assert np.array_equal(r["theta_hist"], want_t)
    assert np.array_equal(r["tof_hist"], want_f)
    assert (r["n_substrate"], r["n_target"], r["n_unfinished"]) == (7, 1, 1)
    assert abs(r["e_sum_substrate"] - E[:7].sum()) < 1e-12 and r["e_sum_target"] == 7.3


def test_tally_bins_of_known_atoms():
    check_tally_bins_of_known_atoms()


def test_ballistic_histograms_follow_the_source_laws():
    """With no gas every atom reaches the substrate as emitted: its energy
    histogram follows the Thompson law (bin probabilities by quadrature) and its
    angle histogram the cosine law, P(theta in [k, k + 1) deg) =
    sin^2(k + 1) - sin^2(k)."""
    n = 100000
    src, tp = W.sputter_transport(p_pa=0.0, n_atoms=n)
    tp.update(n_ebins=40, ebin_ev=5.0)
    r = T.run(src, tp)
    U, cut = src["u_s_ev"], src["e_cut_ev"]
    Z = integrate.quad(_thompson_density, 0, cut, args=(U,))[0]
    edges = np.arange(41) * 5.0
    pe = np.array([integrate.quad(_thompson_density, a, b, args=(U,))[0] / Z for a, b in zip(edges[:-1], edges[1:])])
    assert r["e_hist"].sum() == n
    assert stats.chisquare(r["e_hist"], n * pe / pe.sum()).pvalue > 1e-5
    k = np.arange(91)
    pt = np.diff(np.sin(np.radians(k)) ** 2)
    assert stats.chisquare(r["theta_hist"], n * pt / pt.sum()).pvalue > 1e-5


def _vhs_rate_coefficient(u, tp):
    """<sigma(g) g> of a test atom at speed u against the Maxwellian gas, with the
    VHS cross section written out from its definition (sigma g = A g^(2 - 2 omega))
    and the relative-speed law of a fixed velocity against an isotropic Gaussian
    (a noncentral chi law of 3 degrees of freedom), integrated by quadrature."""
    m, M = T.masses(tp)
    mr = m * M / (m + M)
    om = tp["omega"]
    A = math.pi * tp["d_ref"] ** 2 * (2 * C.K_B * tp["t_ref"] / mr) ** (om - 0.5) / math.gamma(2.5 - om)
    s = math.sqrt(C.K_B * tp["t_gas_k"] / M)

    def dens(g):
        return g / (u * s * math.sqrt(2 * math.pi)) * (math.exp(-(g - u) ** 2 / (2 * s * s))
                                                       - math.exp(-(g + u) ** 2 / (2 * s * s)))
    lo, hi = max(0.0, u - 14 * s), u + 14 * s
    norm = integrate.quad(dens, lo, hi, epsabs=0, epsrel=1e-11)[0]
    mom = integrate.quad(lambda g: A * g ** (2 - 2 * om) * dens(g), lo, hi, epsabs=0, epsrel=1e-11)[0]
    return mom / norm


def check_uncollided_transmission(p_pa, n=20000, scatter=T.SCATTER_VHS):
    """Beer-Lambert: an atom crosses the gap without a real collision with
    probability exp(-n_gas <sigma g>(|v|) L / v_x), whatever the majorant and the
    null events in between (Eq. (6) thinning).  Uncollided atoms are those reaching
    the substrate with their emitted velocity unchanged; their count must match the
    sum of the per-atom probabilities within the binomial spread."""
    src, tp = W.sputter_transport(p_pa=p_pa, n_atoms=n)
    tp["scatter"] = scatter
    res = T.run(src, tp, trace=True)
    assert res["overflow"] == 0
    _, _, v0, _ = T.source(n, src, tp)
    tr = res["trace"]
    free = (tr["wall"] == T.WALL_SUBSTRATE) & np.all(tr["v"] == v0, axis=1)
    u = np.linalg.norm(v0, axis=1)
    grid = np.geomspace(u.min() * 0.999, u.max() * 1.001, 160)
    # M1 reuses the VHS law with the reference diameter sqrt(4/3) d_ref: 4/3 the cross section
    k = np.array([_vhs_rate_coefficient(g, tp) for g in grid]) * (4.0 / 3.0 if scatter == T.SCATTER_M1 else 1.0)
    k_u = np.exp(np.interp(np.log(u), np.log(grid), np.log(k)))
    n_gas = C.gas_density(p_pa, tp["t_gas_k"])
    p = np.exp(-n_gas * k_u * tp["gap_m"] / v0[:, 0])
    mean, sd = p.sum(), math.sqrt(np.sum(p * (1 - p)))
    assert abs(free.sum() - mean) < 4.5 * sd, (p_pa, int(free.sum()), mean, sd)
    # the uncollided atoms keep their time of flight L / v_x exactly
    assert np.allclose(tr["tof"][free], tp["gap_m"] / v0[free, 0], rtol=1e-12)
    return free.sum(), mean, sd


@pytest.mark.parametrize("p_pa,scatter", [(0.5, T.SCATTER_VHS), (2.0, T.SCATTER_VHS), (0.5, T.SCATTER_M1)])
def test_uncollided_transmission_follows_beer_lambert(p_pa, scatter):
    check_uncollided_transmission(p_pa, scatter=scatter)


def check_fixed_step_uncollided_transmission(n=20000, dt=2e-7):
    """Eq. (7), step by step: with a fresh partner at every step an atom collides
    with probability n_gas sigma(g) g dt, so on average p = n_gas <sigma g>(|v|) dt
    per step; the atoms that reach the substrate untouched after the
    floor(L / (v_x dt)) whole steps before the wall (the last, partial step ends
    at the wall without a test) number sum (1 - p)^k within the binomial spread."""
    src, tp = W.sputter_transport(p_pa=0.5, n_atoms=n)
    tp.update(dt_s=dt, e_max=10 ** 6)
    res = T.run(src, tp, trace=True)
    _, _, v0, _ = T.source(n, src, tp)
    tr = res["trace"]
    free = (tr["wall"] == T.WALL_SUBSTRATE) & np.all(tr["v"] == v0, axis=1)
    u = np.linalg.norm(v0, axis=1)
    grid = np.geomspace(u.min() * 0.999, u.max() * 1.001, 160)
    k_g = np.array([_vhs_rate_coefficient(g, tp) for g in grid])
    k_u = np.exp(np.interp(np.log(u), np.log(grid), np.log(k_g)))
    p = C.gas_density(tp["p_pa"], tp["t_gas_k"]) * k_u * dt
    assert p.max() < 0.05
    steps = np.floor(tp["gap_m"] / (v0[:, 0] * dt))
    q = (1.0 - p) ** steps
    mean, sd = q.sum(), math.sqrt(np.sum(q * (1 - q)))
    assert abs(free.sum() - mean) < 4.5 * sd, (int(free.sum()), mean, sd)
    return free.sum(), mean, sd


def test_fixed_step_uncollided_transmission():
    check_fixed_step_uncollided_transmission()
