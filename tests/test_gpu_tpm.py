"""GPU test-particle path against the oracle (runs on an MI355X).

Each atom's random numbers depend only on (job, atom id, event index), so the GPU
and the oracle fly the same trajectories until an FP32/FP64 rounding difference
flips a decision (an acceptance test or a wall crossing within ~1e-6 of its
threshold).  Per atom, the absorbing wall and the event count must agree for
all but a small fraction; final energy, angle and time of flight of agreeing
atoms within 1e-4 relative; tallies statistically.
"""
import math

import numpy as np
import pytest

from oracle import constants as C
from oracle import tpm as T
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_04069_amd as mod
    return mod


def _compare_atoms(g, o, max_mismatch, tof_rtol=1e-4):
    gt, ot = g["trace"], o["trace"]
    same = (gt["wall"] == ot["wall"]) & (gt["events"].astype(np.int64) == ot["events"])
    frac = 1 - same.mean()
    assert frac <= max_mismatch, frac
    s = same & (ot["wall"] == T.WALL_SUBSTRATE)
    assert np.all(np.abs(gt["energy_ev"][s] - ot["E"][s]) <= 1e-4 * np.maximum(ot["E"][s], 1e-3))
    assert np.all(np.abs(gt["tof_s"][s] - ot["tof"][s]) <= tof_rtol * ot["tof"][s])
    assert np.all(np.abs(gt["theta_deg"][s] - ot["theta"][s]) <= 2e-2)
    return same


@pytest.mark.parametrize("p_pa", [0.5, 2.0])
def test_flight_matches_oracle_atom_by_atom(pm, p_pa):
    n = 20000 if p_pa < 1 else 5000
    src, tp = W.sputter_transport(p_pa=p_pa, n_atoms=n)
    g = pm.run_test_particles(src, tp, trace=True)
    o = T.run(src, tp, trace=True)
    _compare_atoms(g, o, max_mismatch=0.01)
    assert g["n_substrate"] + g["n_target"] + g["n_unfinished"] == n
    assert abs(g["nu_max"] / o["nu_max"] - 1) < 1e-12
    # deposition fraction within 3 % (statistics of the same atoms)
    assert abs(g["eta"] - o["n_substrate"] / n) <= 0.03 * (o["n_substrate"] / n)
    assert abs(g["events"] / o["events"] - 1) < 0.01
    # track-length profiles: the same atoms, so cell by cell within the share of
    # atoms whose path differs; the GPU's cells add up to its own flight times
    assert np.allclose(g["time_s"], o["time_s"], rtol=0.03)
    assert np.allclose(g["disp_m"], o["disp_m"], rtol=0.03)
    if g["n_unfinished"] == 0:
        assert abs(g["time_s"].sum() / g["trace"]["tof_s"].astype(np.float64).sum() - 1) < 1e-4
        assert abs(g["disp_m"].sum() / (tp["gap_m"] * g["n_substrate"]) - 1) < 1e-5


@pytest.mark.parametrize("p_pa", [0.5, 2.0])
def test_m1_flight_matches_oracle_atom_by_atom(pm, p_pa):
    """M1 scattering (deflection pi (1 - b/b_max) about the relative velocity, d_ref
    sqrt(4/3)): the same atoms reach the same wall after the same events."""
    n = 20000 if p_pa < 1 else 5000
    src, tp = W.sputter_transport(p_pa=p_pa, n_atoms=n)
    tp["scatter"] = T.SCATTER_M1
    g = pm.run_test_particles(src, tp, trace=True)
    o = T.run(src, tp, trace=True)
    _compare_atoms(g, o, max_mismatch=0.01)
    assert abs(g["nu_max"] / o["nu_max"] - 1) < 1e-12
    assert abs(g["eta"] - o["n_substrate"] / n) <= 0.03 * (o["n_substrate"] / n)
    # forward-peaked M1 scattering lets more atoms through than isotropic VHS at
    # the same viscosity cross section
    tp_v = dict(tp, scatter=T.SCATTER_VHS)
    gv = pm.run_test_particles(src, tp_v)
    assert g["eta"] > gv["eta"]


def test_m1_box_thermalises_at_four_thirds_the_vhs_rate(pm):
    n = 20000
    outs = []
    for e_max in (600, 1200):
        src, tp = W.sputter_transport(p_pa=0.5, n_atoms=n, mode=T.MODE_BOX)
        tp.update(e_max=e_max, scatter=T.SCATTER_M1)
        outs.append(pm.run_test_particles(src, tp, trace=True))
    m, M = W.AL_AMU * C.AMU, W.AR_AMU * C.AMU
    kT = C.K_B * 300.0
    v = np.stack([outs[1]["trace"][k] for k in ("vx", "vy", "vz")], axis=1).astype(np.float64)
    ke = 0.5 * m * np.sum(v * v, axis=1)
    assert abs(ke.mean() / (1.5 * kT) - 1) < 0.03
    mr = m * M / (m + M)
    n_gas = C.gas_density(0.5, 300.0)
    nu_eq = n_gas * 2 * math.sqrt(math.pi) * (3.6e-10) ** 2 * math.sqrt(2 * kT / mr) * (273.0 / 300.0) ** 0.3
    dt = outs[1]["trace"]["tof_s"].astype(np.float64).sum() - outs[0]["trace"]["tof_s"].astype(np.float64).sum()
    rate = (outs[1]["collisions"] - outs[0]["collisions"]) / dt
    assert abs(rate / (4.0 / 3.0 * nu_eq) - 1) < 0.02


def test_fixed_step_flight_matches_oracle_atom_by_atom(pm):
    """Fixed dt (Eq. (7), 'Collisional Transport'): flights of dt, then a collision
    with probability n sigma g dt -- the same atoms, walls and step counts."""
    n = 8000
    src, tp = W.sputter_transport(p_pa=0.5, n_atoms=n)
    tp.update(dt_s=1e-7, e_max=10 ** 6)
    g = pm.run_test_particles(src, tp, trace=True)
    o = T.run(src, tp, trace=True)
    # FP32 positions take one rounding per step: over the ~1e3 steps of a slow
    # atom the crossing time drifts by up to ~1e-4 (measured max 1.2e-4)
    _compare_atoms(g, o, max_mismatch=0.01, tof_rtol=5e-4)
    assert abs(g["eta"] - o["n_substrate"] / n) <= 0.03 * (o["n_substrate"] / n)
    assert g["n_unfinished"] == 0


def test_fixed_step_collides_with_the_linear_probability(pm):
    n = 20000
    outs = []
    for e_max in (400, 800):
        src, tp = W.sputter_transport(p_pa=0.5, n_atoms=n, mode=T.MODE_BOX)
        tp.update(e_max=e_max, dt_s=1.0e-5)
        outs.append(pm.run_test_particles(src, tp, trace=True))
    m, M = W.AL_AMU * C.AMU, W.AR_AMU * C.AMU
    kT = C.K_B * 300.0
    v = np.stack([outs[1]["trace"][k] for k in ("vx", "vy", "vz")], axis=1).astype(np.float64)
    assert abs(0.5 * m * np.sum(v * v, axis=1).mean() / (1.5 * kT) - 1) < 0.03
    mr = m * M / (m + M)
    n_gas = C.gas_density(0.5, 300.0)
    nu_eq = n_gas * 2 * math.sqrt(math.pi) * (3.6e-10) ** 2 * math.sqrt(2 * kT / mr) * (273.0 / 300.0) ** 0.3
    p_step = (outs[1]["collisions"] - outs[0]["collisions"]) / (n * 400)
    assert abs(p_step / (nu_eq * 1.0e-5) - 1) < 0.02


def test_ballistic_flight_is_exact(pm):
    src, tp = W.sputter_transport(p_pa=0.0, n_atoms=50000)
    g = pm.run_test_particles(src, tp, trace=True)
    o = T.run(src, tp, trace=True)
    assert g["n_substrate"] == 50000 and g["eta"] == 1.0
    gt, ot = g["trace"], o["trace"]
    assert np.all(gt["wall"] == 1) and np.all(gt["events"] == 0)
    # FP32 bar: near the 200 eV cut the inversion divides by 1 - s ~ 0.017, which
    # amplifies one rounding of s to ~4e-6 relative
    assert np.allclose(gt["energy_ev"], ot["E"], rtol=1e-5, atol=0)
    assert np.allclose(gt["tof_s"], ot["tof"], rtol=1e-5, atol=0)
    # the substrate histograms of the GPU are the oracle's (its tally is pinned by
    # atoms of known bins and by the source laws)
    for k in ("e_hist", "theta_hist", "tof_hist"):
        assert np.abs(g[k].astype(np.int64) - o[k]).sum() <= 20, k      # bin-edge rounding only
    # every atom crosses every cell once: uniform profiles equal to the oracle's
    assert np.allclose(g["time_s"], o["time_s"], rtol=1e-5)
    assert np.allclose(g["disp_m"], o["disp_m"], rtol=1e-6)
    src2 = dict(src, flux_m2s=1e18)
    dens_o, ux_o = T.profiles(o, src2, 50000, tp["gap_m"])
    g2 = pm.run_test_particles(src2, tp)
    assert np.allclose(g2["density_m3"], dens_o, rtol=1e-5)
    assert np.allclose(g2["mean_vx"], ux_o, rtol=1e-5)


def test_box_thermalises_at_the_vhs_rate(pm):
    n = 20000
    rates = []
    outs = []
    for e_max in (600, 1200):
        src, tp = W.sputter_transport(p_pa=0.5, n_atoms=n, mode=T.MODE_BOX)
        tp["e_max"] = e_max
        outs.append(pm.run_test_particles(src, tp, trace=True))
    m, M = W.AL_AMU * C.AMU, W.AR_AMU * C.AMU
    kT = C.K_B * 300.0
    v = np.stack([outs[1]["trace"][k] for k in ("vx", "vy", "vz")], axis=1).astype(np.float64)
    ke = 0.5 * m * np.sum(v * v, axis=1)
    assert abs(ke.mean() / (1.5 * kT) - 1) < 0.03
    mr = m * M / (m + M)
    n_gas = C.gas_density(0.5, 300.0)
    nu_eq = n_gas * 2 * math.sqrt(math.pi) * (3.6e-10) ** 2 * math.sqrt(2 * kT / mr) * (273.0 / 300.0) ** 0.3
    dt = outs[1]["trace"]["tof_s"].astype(np.float64).sum() - outs[0]["trace"]["tof_s"].astype(np.float64).sum()
    rate = (outs[1]["collisions"] - outs[0]["collisions"]) / dt
    assert abs(rate / nu_eq - 1) < 0.02


def test_sputter_yield_count_matches_oracle(pm):
    p = W.discharge_small(seed=7)
    case = pm.Case(p)
    case.step(2000)
    d = case.sample_diagnostics()
    target = d["iedf"][0]
    assert target.sum() > 0
    for Y, table in ((1.0, None), (0.7, None), (2.4, None), (None, ([0.0, 50.0, 400.0], [0.0, 0.4, 2.2]))):
        src = case.inject_sputtered(yield_const=Y if Y is not None else 0.0, table=table, seed=9, job_id=4)
        want = T.sputtered_count(target, Y if table is None else table, seed=9, job_id=4)
        assert src["n_emitted"] == want
        assert src["n_impacts"] == int(target.sum())
    # re-sputtering: the substrate's impacts with their own draws
    substrate = d["iedf"][1]
    assert substrate.sum() > 0
    src = case.inject_sputtered(yield_const=1.3, seed=9, job_id=4, electrode=1)
    assert src["electrode"] == 1 and src["n_impacts"] == int(substrate.sum())
    assert src["n_emitted"] == T.sputtered_count(substrate, 1.3, seed=9, job_id=4, electrode=1)
    case.close()


def test_substrate_emission_matches_oracle_atom_by_atom(pm):
    """Re-sputtered atoms leave the substrate into -x: the same atoms reach the same
    walls after the same events as in the oracle."""
    n = 20000
    src, tp = W.sputter_transport(p_pa=0.5, n_atoms=n)
    src["electrode"] = 1
    g = pm.run_test_particles(src, tp, trace=True)
    o = T.run(src, tp, trace=True)
    gt, ot = g["trace"], o["trace"]
    same = (gt["wall"] == ot["wall"]) & (gt["events"].astype(np.int64) == ot["events"])
    assert 1 - same.mean() <= 0.01
    s = same & (ot["wall"] == T.WALL_TARGET)
    assert s.sum() > n // 2
    assert np.all(np.abs(gt["tof_s"][s] - ot["tof"][s]) <= 1e-4 * ot["tof"][s])
    assert g["n_target"] > g["n_substrate"]


def test_coupled_source_to_flight(pm):
    """One-way coupling: the atoms sputtered by a discharge's target impacts are flown."""
    p = W.discharge_small(seed=8)
    case = pm.Case(p)
    case.step(2000)
    src = case.inject_sputtered(yield_const=1.0, seed=5, job_id=6)
    assert src["n_atoms"] == src["n_impacts"] > 0 and src["flux_m2s"] > 0
    _, tp = W.sputter_transport(p_pa=p["p_pa"])
    tp["gap_m"] = p["gap_m"]
    g = pm.run_test_particles(src, tp)
    assert g["n_substrate"] + g["n_target"] + g["n_unfinished"] == src["n_atoms"]
    assert g["deposition_flux"] == pytest.approx(g["eta"] * src["flux_m2s"])
    case.close()


def test_live_injection_adds_up_to_the_window(pm):
    """Live coupling: the atoms injected after every RF cycle from the impacts
    that cycle recorded, and flown at once, are exactly the atoms of one
    injection and flight over the whole window (same ids, counts and integer
    tallies); each cycle's count equals the oracle's count of its new impacts."""
    p = W.discharge_small(seed=8)
    _, tp = W.sputter_transport(p_pa=p["p_pa"])
    tp["gap_m"] = p["gap_m"]
    kw = dict(yield_const=0.6, seed=5, job_id=6)
    live, whole = pm.Case(p), pm.Case(p)
    for c in (live, whole):
        c.step(1500)
        c.sample_diagnostics(reset=True)
    job = pm.TestParticleJob(tp)
    ints = ("n_substrate", "n_target", "n_unfinished", "events", "collisions", "overflow")
    hists = ("e_hist", "theta_hist", "tof_hist")
    acc = {k: 0 for k in ints}
    acc.update({k: 0 for k in hists + ("time_s", "disp_m", "e_sum_substrate")})
    prev = np.zeros(live.n_ebins, dtype=np.int64)
    n_em = 0
    for _ in range(4):
        live.step_rf_cycles(1)
        rec = live.sample_diagnostics()["iedf"][0].astype(np.int64)
        src = live.inject_sputtered(since_last=True, **kw)
        assert src["first_atom"] == n_em
        assert src["n_impacts"] == int(rec.sum() - prev.sum())
        assert src["n_emitted"] == T.sputtered_count(rec, 0.6, seed=5, job_id=6, taken=prev)
        prev = rec
        n_em += src["n_emitted"]
        if src["n_atoms"] > 0:
            r = job.run(src)
            for k in acc:
                acc[k] = acc[k] + r[k]
    assert n_em > 0
    whole.step_rf_cycles(4)
    src = whole.inject_sputtered(**kw)
    assert src["n_emitted"] == n_em and src["first_atom"] == 0
    assert src["n_impacts"] == int(prev.sum())
    r = job.run(src)
    for k in ints:
        assert acc[k] == r[k], k
    for k in hists:
        assert np.array_equal(acc[k], r[k]), k
    for k in ("time_s", "disp_m"):
        assert np.allclose(acc[k], r[k], rtol=1e-12, atol=1e-12 * np.max(np.abs(r[k]))), k
    assert acc["e_sum_substrate"] == pytest.approx(r["e_sum_substrate"], rel=1e-9)
    live.close()
    whole.close()


def test_zero_atoms_fly_nothing(pm):
    src, tp = W.sputter_transport(p_pa=0.5, n_atoms=0)
    g = pm.run_test_particles(src, tp)
    assert g["n_substrate"] == g["n_target"] == g["n_unfinished"] == g["events"] == 0
    assert not np.any(g["e_hist"]) and not np.any(g["time_s"]) and g["eta"] == 0.0


def test_few_atoms_fly_as_in_a_large_launch(pm):
    """One atom, a partial wavefront (63) and a little over four wavefronts (257):
    each atom's flight depends on its own id only, so these launches give, atom by
    atom, exactly what the same atoms give inside a launch of 5000, and the tallies
    count every atom once."""
    src, tp = W.sputter_transport(p_pa=2.0, n_atoms=5000)
    big = pm.run_test_particles(src, tp, trace=True)["trace"]
    for n in (1, 63, 257):
        g = pm.run_test_particles(dict(src, n_atoms=n), tp, trace=True)
        assert g["n_substrate"] + g["n_target"] + g["n_unfinished"] == n
        for k in ("wall", "events", "energy_ev", "tof_s", "theta_deg"):
            assert np.array_equal(g["trace"][k], big[k][:n]), (n, k)


@pytest.mark.parametrize("p_pa", [0.5, 5.0])
def test_full_size_flight_matches_oracle_on_sampled_atoms(pm, p_pa):
    """The benchmark's flights at full size (1e7 atoms at 0.5 Pa, 1e6 at 5 Pa, the
    launch the benchmark times): four runs of consecutive atoms spread over the
    id range, each flown by the oracle from its own ids, agree atom by atom to the
    per-atom bar; the tallies count every atom once."""
    n_full = 10_000_000 if p_pa < 1 else 1_000_000
    src, tp = W.sputter_transport(p_pa=p_pa, n_atoms=n_full)
    g = pm.run_test_particles(src, tp, trace=True)
    assert g["n_substrate"] + g["n_target"] + g["n_unfinished"] == n_full
    assert int(g["e_hist"].sum()) == g["n_substrate"]
    m = 400 if p_pa < 1 else 100
    for first in (0, n_full // 3, 2 * n_full // 3, n_full - m):
        print(f"atoms {first}..{first + m - 1} at {p_pa} Pa", flush=True)
        o = T.run(src, tp, n_atoms=m, first_id=first, trace=True)
        sub = {"trace": {k: v[first:first + m] for k, v in g["trace"].items()}}
        _compare_atoms(sub, o, max_mismatch=0.03)
