"""GPU PIC/MCC path against the oracle (runs on an MI355X).

Single steps from an identical state: cell indices, deposited charge and
collision decisions bit-exact; positions and velocities within 1e-5 relative in
FP32 (1e-11 in FP64).  Exempt, and counted, are the near-ties frozen before any
comparison: wall crossings within a few FP32 ulps of an electrode, process
selections whose oracle margin is below 2^-20 nu_max, and geometric-skip draws
within 1e-9 of an integer.
"""
import math

import numpy as np
import pytest

from oracle import constants as C
from oracle import philox as R
from oracle import pic as P
import workloads as W
from tests.gpu_helpers import assert_same, by_id, gpu_state_si, oracle_from_gpu, oracle_state, snapshot

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_04069_amd as mod
    return mod


def small_fp64():
    return W.discharge_small(seed=1)


def small_fp32():
    return W.discharge_small(seed=2, fp64=False)


def working_reduced():
    # the working-size grid (1024 cells, 300 V, 0.5 Pa, dt = T/2000) with 100k + 100k particles
    return W.discharge_working(np_each=100_000)


def small_circuit_fp64():
    # the paper's drive (Sec. III): two harmonics, Delta phi = 0, through a blocking capacitor
    p = W.discharge_small(seed=3)
    p.update(v2_volt=p["v0_volt"], phase2_rad=0.0, cb_f_m2=1e-8)
    return p


def small_circuit_fp32():
    p = small_circuit_fp64()
    p.update(fp64=False, seed=4)
    return p


CASES = {"small_fp64": small_fp64, "small_fp32": small_fp32, "working_1024_fp32": working_reduced,
         "small_circuit_fp64": small_circuit_fp64, "small_circuit_fp32": small_circuit_fp32}


def tols(p):
    return (1e-11, 1e-11) if p.get("fp64") else (1e-5, 1e-5)


def vth(p, s):
    T = p["te_ev"] if s == 0 else p["ti_ev"]
    m = C.M_E if s == 0 else C.M_AR
    return math.sqrt(T * C.E_CHARGE / m)


# ---------------------------------------------------------------- loading
@pytest.mark.parametrize("name", list(CASES))
def test_load_matches_oracle(pm, name):
    p = CASES[name]()
    case = pm.Case(p)
    orc = P.Discharge(p, wait_cap=P.WAIT_CAP)
    rtol, _ = tols(p)
    for s in (0, 1):
        gid, gx, gv, gn = gpu_state_si(case, s)
        oid, ox, ov, on = oracle_state(orc, s)
        assert np.array_equal(gid, oid)
        assert np.array_equal(gx, ox)                  # N * U is exact in both precisions
        scale = np.maximum(np.abs(ov), vth(p, s))
        assert np.all(np.abs(gv - ov) <= rtol * scale)
        Us = R.draw(oid, np.uint64(2 ** 64 - 1), R.tag(s, R.SKIP), p["seed"], p["case_id"])
        _, _, tie = P.skip(Us[:, 0], -1, orc.d["p_tot"][s])
        assert np.array_equal(gn[~tie], on[~tie])
    case.close()


@pytest.mark.parametrize("name", list(CASES))
def test_initial_fields_match_oracle(pm, name):
    p = CASES[name]()
    case = pm.Case(p)
    f = case.get_fields()
    orc = oracle_from_gpu(case, p)
    Qe, Qi, rho, V, Phi, E = orc.field(orc.step_index)
    assert np.array_equal(f["qe"], Qe) and np.array_equal(f["qi"], Qi)   # bit-exact charge
    assert np.max(np.abs(f["phi"] - Phi)) <= 1e-12 * max(np.max(np.abs(Phi)), 1.0)
    assert np.max(np.abs(f["E"] - E)) <= 1e-11 * np.max(np.abs(E))
    case.close()


# ---------------------------------------------------------------- one step
def compare_step(case, p, orc, rec, before, after, n_ties):
    """Compare the GPU state after one step with the oracle's, by particle id."""
    rtol, _ = tols(p)
    N = p["n_cells"]
    l = rec["step"]
    exempt = set()
    for s in (0, 1):
        # wall near-ties: pushed position within 4 FP32 ulps (at N) of an electrode
        xp = rec[f"pushed_xt_{s}"]
        near = (np.abs(xp) <= 4 * N * 2.0 ** -23) | (np.abs(xp - N) <= 4 * N * 2.0 ** -23)
        exempt |= set(rec[f"pushed_id_{s}"][near].tolist())
        if f"tie_{s}" in rec:
            cid = rec[f"cand_id_{s}"]
            tie = rec[f"tie_{s}"] | rec[f"skip_tie_{s}"]
            exempt |= set(cid[tie].tolist())
            if s == 0 and np.any(rec["tie_0"]):
                w0, w1, _, _ = R.philox4x64(cid[rec["tie_0"]], np.uint64(l), R.tag(0, R.CHILD), 0,
                                            p["seed"], p["case_id"])
                exempt |= set(w0.tolist()) | set(w1.tolist())
        if f"redraw_id_{s}" in rec:
            exempt |= set(rec[f"redraw_id_{s}"][rec[f"redraw_tie_{s}"]].tolist())
    n_ties["count"] += len(exempt)
    ex = np.array(sorted(exempt), dtype=np.uint64)
    for s in (0, 1):
        gid, gx, gv, gn = gpu_state_si(case, s)
        oid, ox, ov, on = oracle_state(orc, s)
        gk = ~np.isin(gid, ex)
        ok = ~np.isin(oid, ex)
        assert np.array_equal(gid[gk], oid[ok]), f"species {s}: surviving/born ids differ"
        gx, gv, gn = gx[gk], gv[gk], gn[gk]
        ox, ov, on = ox[ok], ov[ok], on[ok]
        assert np.array_equal(np.floor(gx), np.floor(ox)) or _cell_near_ties_only(gx, ox)
        assert np.all(np.abs(gx - ox) <= rtol * np.maximum(np.abs(ox), 1.0)), f"species {s}: positions"
        scale = np.maximum(np.linalg.norm(ov, axis=1), vth(p, s))[:, None]
        assert np.all(np.abs(gv - ov) <= rtol * scale), f"species {s}: velocities"
        assert np.array_equal(gn, on), f"species {s}: next candidate steps"
    # the deposited charge of step l+1, computed by the oracle from the GPU's positions
    f = case.get_fields()
    for s, key in ((0, "qe"), (1, "qi")):
        g = case.get_particles(s)
        assert np.array_equal(f[key], P.deposit(g["xt"], N)), f"charge of species {s}"
    # counters of the step
    d1 = after
    d0 = before
    acc = orc.acc
    for s in (0, 1):
        assert d1["candidates"][s] - d0["candidates"][s] == acc["candidates"][s] - rec["acc0"]["candidates"][s]


def _cell_near_ties_only(gx, ox):
    diff = np.floor(gx) != np.floor(ox)
    return bool(np.all(np.abs(ox[diff] - np.rint(ox[diff])) <= 2 * 2.0 ** -23 * np.maximum(np.abs(ox[diff]), 1)))


def run_single_steps(pm, p, warm_steps, reps):
    case = pm.Case(p)
    if warm_steps:
        case.step(warm_steps)
    n_ties = {"count": 0}
    n_cand = 0
    for _ in range(reps):
        orc = oracle_from_gpu(case, p)
        before = case.sample_diagnostics()
        acc0 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in orc.acc.items()}
        rec = orc.step(record=True)
        rec["acc0"] = acc0
        case.step(1)
        after = case.sample_diagnostics()
        compare_step(case, p, orc, rec, before, after, n_ties)
        n_cand += int(sum(len(rec.get(f"cand_id_{s}", [])) for s in (0, 1)))
    case.close()
    return n_ties["count"], n_cand


@pytest.mark.parametrize("name", list(CASES))
def test_single_steps_match_oracle(pm, name):
    p = CASES[name]()
    ties, cand = run_single_steps(pm, p, warm_steps=0, reps=4)
    assert cand > 0
    assert ties <= max(2, cand // 100)


@pytest.mark.parametrize("np_e,np_i", [(5001, 4999), (3000, 0)])
def test_ragged_and_ion_free_steps_match_oracle(pm, np_e, np_i):
    """Particle counts that leave ragged tiles, and a start with no ions at all
    (the species' slot range empty until ionisation creates ions)."""
    p = W.discharge_small(seed=14, fp64=False)
    p.update(np_e=np_e, np_i=np_i, capacity_e=4 * np_e, capacity_i=20000)
    ties, cand = run_single_steps(pm, p, warm_steps=0, reps=3)
    assert cand > 0
    assert ties <= max(2, cand // 100)


@pytest.mark.parametrize("n_cells,np_e,np_i", [(1, 400, 400), (2, 400, 400), (777, 5003, 4997), (64, 1, 0)])
def test_extreme_grids_and_counts_match_oracle(pm, n_cells, np_e, np_i):
    """The smallest grids (one cell: both nodes are electrodes and the field is
    the applied one plus the boundary charges' half-cell terms; two cells: one
    interior node), a grid of no power-of-two size, and a discharge of a single
    electron, each over single steps after 20 warm-up steps."""
    p = W.discharge_small(seed=16, fp64=False)
    p.update(n_cells=n_cells, np_e=np_e, np_i=np_i, capacity_e=max(4 * np_e, 256), capacity_i=4 * max(np_i, 100))
    ties, cand = run_single_steps(pm, p, warm_steps=20, reps=3)
    if np_e > 1:
        assert cand > 0
    assert ties <= max(2, cand // 100)


@pytest.mark.parametrize("mode", ["no_collisions", "zero_pressure", "no_self_field"])
def test_degenerate_modes_match_oracle(pm, mode):
    """The method's degenerate cases, single steps after 200 warm-up steps:
    collisions switched off, no gas at all (zero pressure: no collision
    schedule, every particle's next examination never), and charges that feel
    only the applied field (the particles' own field switched off)."""
    p = W.discharge_small(seed=15, fp64=False)
    if mode == "no_collisions":
        p["flags"] = P.NO_COLLISIONS
    elif mode == "zero_pressure":
        p["p_pa"] = 0.0
    else:
        p["flags"] = P.NO_SELF_FIELD
    ties, cand = run_single_steps(pm, p, warm_steps=200, reps=3)
    if mode == "no_self_field":
        assert cand > 0
    else:
        assert cand == 0
    assert ties <= max(2, cand // 100)


@pytest.mark.parametrize("name", ["small_fp64", "small_fp32", "small_circuit_fp64", "small_circuit_fp32"])
def test_single_steps_after_warmup_match_oracle(pm, name):
    p = CASES[name]()
    ties, cand = run_single_steps(pm, p, warm_steps=800, reps=6)
    assert cand > 0


@pytest.mark.parametrize("fp64", [False, True])
def test_cut_wait_examinations_match_oracle(pm, fp64):
    """Examinations at a cut wait take only a fresh wait (no collision test), and
    examination steps anywhere up to the cut survive the 15-bit code's wrap."""
    p = W.discharge_small(seed=7, fp64=fp64)
    case = pm.Case(p)
    case.step(5)
    l = int(case.sample_diagnostics()["step"])
    rng = np.random.default_rng(3)
    for s in (0, 1):
        g = case.get_particles(s)
        n = len(g["xt"])
        nx = g["next"].astype(np.int64)
        due = rng.uniform(size=n) < 0.5
        nx[due] = l | (1 << 31)                                   # due now, redraw only
        far = ~due & (rng.uniform(size=n) < 0.3)
        nx[far] = l + rng.integers(1, 32768, size=int(far.sum()))  # real, up to the cut
        g["next"] = nx.astype(np.uint32)
        case.set_particles(s, g)                                  # (the set sorts by cell)
        back = case.get_particles(s)
        assert np.array_equal(by_id(back["id"], back["next"])[1], by_id(g["id"], g["next"])[1])
    g = case.get_particles(0)
    g["next"][0] = l + 32768                                      # beyond the cut
    with pytest.raises(pm.PicMccError):
        case.set_particles(0, g)
    n_ties = {"count": 0}
    orc = oracle_from_gpu(case, p)
    assert orc.sp[0].redraw.sum() > 100 and orc.sp[1].redraw.sum() > 100
    before = case.sample_diagnostics()
    acc0 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in orc.acc.items()}
    rec = orc.step(record=True)
    rec["acc0"] = acc0
    case.step(1)
    after = case.sample_diagnostics()
    compare_step(case, p, orc, rec, before, after, n_ties)
    assert n_ties["count"] <= 2
    case.close()


def test_circuit_vacuum_divider(pm):
    """Without space charge the blocking capacitor and the gap divide the source:
    Phi_0 = (C_gap V(0) + C_B V(t) + e w n) / (C_gap + C_B) with n the net charges
    the driven electrode has absorbed (counted on the device), and the potential is
    linear across the gap."""
    p = W.discharge_small(seed=6, flags=P.NO_SELF_FIELD | P.NO_COLLISIONS)
    p.update(v0_volt=150.0, v2_volt=150.0, cb_f_m2=2e-10)
    case = pm.Case(p)
    d = P.derived(p)
    cg = C.EPS0 / p["gap_m"]
    V0 = P.voltage(p, 0)
    f = case.get_fields()
    assert abs(f["phi"][0] - V0) <= 1e-12 * abs(V0)
    assert abs(f["sigma_init"] - cg * V0) <= 1e-9 * abs(cg * V0)
    seen = set()
    for k in (1, 1, 2, 3, 5, 8, 13, 21, 34):
        case.step(k)
        l = int(case.sample_diagnostics()["step"])
        f = case.get_fields()
        n = int(f["n_absorbed_net"])
        seen.add(n)
        want = (cg * V0 + p["cb_f_m2"] * P.voltage(p, l) + C.E_CHARGE * d["w"] * n) / (cg + p["cb_f_m2"])
        assert abs(f["phi"][0] - want) <= 1e-11 * max(abs(want), 1.0), (l, f["phi"][0], want)
        x = np.arange(f["phi"].size) / (f["phi"].size - 1)
        assert np.allclose(f["phi"], want * (1 - x), rtol=0, atol=1e-10 * max(abs(want), 1.0))
    assert len(seen) > 1                          # particles did reach the driven electrode
    case.close()


def _beam_state(n, N, speed_cells, rng, step):
    dirs = rng.normal(size=(n, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    u = (speed_cells * dirs).astype(np.float32).astype(np.float64)
    xt = rng.uniform(0.25 * N, 0.75 * N, n).astype(np.float32).astype(np.float64)
    return dict(xt=xt, ux=u[:, 0], uy=u[:, 1], uz=u[:, 2],
                id=np.arange(n, dtype=np.uint64) + np.uint64(1000),
                next=np.full(n, step, dtype=np.uint32))


@pytest.mark.parametrize("fp64", [False, True])
def test_collision_kinematics_match_oracle(pm, fp64):
    """Every particle a candidate at 60 eV (electrons) and 100 eV (ions): elastic,
    excitation, ionisation (with births) and charge exchange all occur."""
    p = W.discharge_small(seed=5, fp64=fp64, flags=P.NO_SELF_FIELD)
    p.update(v0_volt=0.0, p_pa=10.0, capacity_e=60000, capacity_i=60000)
    case = pm.Case(p)
    info = case.info()
    N = p["n_cells"]
    rng = np.random.default_rng(11)
    ve = math.sqrt(2 * 60.0 * C.E_CHARGE / C.M_E) * info["dt"] / info["dx"]
    vi = math.sqrt(2 * 100.0 * C.E_CHARGE / C.M_AR) * info["dt"] / info["dx"]
    case.set_particles(0, _beam_state(20000, N, ve, rng, 0))
    case.set_particles(1, _beam_state(20000, N, vi, rng, 0))
    orc = oracle_from_gpu(case, p)
    before = case.sample_diagnostics()
    acc0 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in orc.acc.items()}
    rec = orc.step(record=True)
    rec["acc0"] = acc0
    case.step(1)
    after = case.sample_diagnostics()
    n_ties = {"count": 0}
    compare_step(case, p, orc, rec, before, after, n_ties)
    proc = rec["proc_0"]
    assert np.count_nonzero(proc == P.P_ION) > 100 and np.count_nonzero(proc == P.P_EXC) > 100
    assert np.count_nonzero(rec["proc_1"] == P.P_CX) > 1000
    dc = after["collisions"] - before["collisions"]
    oc = orc.acc["collisions"] - acc0["collisions"]
    assert np.all(np.abs(dc - oc) <= n_ties["count"])
    assert after["births"] - before["births"] == orc.acc["births"] - acc0["births"] or n_ties["count"] > 0
    case.close()


# ---------------------------------------------------------------- determinism
@pytest.mark.parametrize("fp64", [False, True])
def test_checkpoint_round_trip_resumes_bit_exact(pm, fp64):
    """Save and restore in mid-window: 600 steps straight equal 300 steps, every
    particle read back to the host and written again (re-sorted, re-deposited,
    the field re-solved), then 300 more.  With the blocking capacitor, phase bins
    and flux profiles, so that the circuit's state and every running sum carry
    over; random numbers are keyed by (id, step), so nothing else is needed."""
    p = small_circuit_fp64()
    p.update(fp64=int(fp64), n_phase=4, flux_profiles=1)
    straight = pm.Case(p)
    straight.step(600)
    ref = snapshot(straight)
    ref_ph = [straight.sample_phase(b) for b in range(4)]
    resumed = pm.Case(p)
    resumed.step(300)
    saved = [resumed.get_particles(s) for s in (0, 1)]
    for s in (0, 1):
        resumed.set_particles(s, saved[s])
    resumed.step(300)
    assert_same(ref, snapshot(resumed))
    for b in range(4):
        got = resumed.sample_phase(b)
        for k in ("ne", "ni", "phi", "gamma_e", "gamma_i", "n_steps", "n_flux_samples"):
            assert np.array_equal(np.asarray(got[k]), np.asarray(ref_ph[b][k])), (b, k)
    straight.close()
    resumed.close()


@pytest.mark.parametrize("fp64", [False, True])
def test_checkpoint_restores_into_a_new_case(pm, fp64):
    """pm_save_checkpoint / pm_load_checkpoint: a fresh case of the same
    parameters, loaded with the state of a case saved after 300 steps (in mid
    RF cycle and mid averaging window), then run 500 steps (one RF cycle of 400
    from the graph, then 100 single steps), equals 800 steps straight bit for bit, as does
    the saved case itself; a checkpoint is refused by a case of other parameters
    and when cut short, with the case unchanged."""
    p = small_circuit_fp64()
    p.update(fp64=int(fp64), n_phase=4, flux_profiles=1, sort_interval=20)
    straight = pm.Case(p)
    straight.step(800)
    ref = snapshot(straight)
    ref_ph = [straight.sample_phase(b) for b in range(4)]
    saved = pm.Case(p)
    saved.step(300)
    buf = saved.save_checkpoint()
    fresh = pm.Case(dict(p, sort_interval=25))       # the sort interval is no part of the state
    fresh.step(7)                                    # whatever it held is replaced
    fresh.load_checkpoint(buf)
    for c in (saved, fresh):
        c.step_rf_cycles(1)
        c.step(100)
        assert_same(ref, snapshot(c))
        for b in range(4):
            got = c.sample_phase(b)
            for k in ("ne", "ni", "phi", "gamma_e", "gamma_i", "n_steps", "n_flux_samples"):
                assert np.array_equal(np.asarray(got[k]), np.asarray(ref_ph[b][k])), (b, k)
    other = pm.Case(dict(p, seed=p["seed"] + 1))
    before = snapshot(other)
    for bad in (lambda: other.load_checkpoint(buf), lambda: fresh.load_checkpoint(buf[:-1])):
        with pytest.raises(pm.PicMccError):
            bad()
    assert_same(before, snapshot(other))
    for c in (straight, saved, fresh, other):
        c.close()


_RESUME_CHILD = """
import sys, numpy as np
sys.path.insert(0, sys.argv[1])
import paper_1607_04069_amd as pm
from tests.test_gpu_pic import small_circuit_fp64
p = small_circuit_fp64()
p.update(fp64=0, n_phase=4, flux_profiles=1)
c = pm.Case(p)
c.load_checkpoint(np.fromfile(sys.argv[2], dtype=np.uint8))
c.step(300)
out = {}
for s in (0, 1):
    g = c.get_particles(s)
    o = np.argsort(g["id"])
    for k, v in g.items():
        out[f"{k}_{s}"] = v[o]
d = c.sample_diagnostics()
for k in ("ne", "ni", "phi", "iedf"):
    out[k] = d[k]
np.savez(sys.argv[3], **out)
"""


def test_checkpoint_resumes_in_another_process(pm, tmp_path):
    """A checkpoint written to a file by this process and loaded by a fresh
    process into a case of its own arena resumes exactly as this process does."""
    import subprocess
    import sys
    import os
    p = small_circuit_fp64()
    p.update(fp64=0, n_phase=4, flux_profiles=1)
    c = pm.Case(p)
    c.step(300)
    path = tmp_path / "case.ckpt"
    c.save_checkpoint().tofile(path)
    c.step(300)
    ref = snapshot(c)
    c.close()
    out = tmp_path / "child.npz"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", _RESUME_CHILD, root, str(path), str(out)],
                       capture_output=True, text=True, timeout=180, cwd=root)
    assert r.returncode == 0, r.stderr[-2000:]
    got = np.load(out)
    for s in (0, 1):
        for k in ref[0][s]:
            assert np.array_equal(got[f"{k}_{s}"], ref[0][s][k]), (s, k)
    for k in ("ne", "ni", "phi", "iedf"):
        assert np.array_equal(got[k], ref[2][k]), k


def test_sort_interval_graph_and_rerun_are_bit_identical(pm):
    p = W.discharge_small(seed=3, fp64=False)
    runs = []
    for K, graph in ((25, True), (0, False), (1, False), (25, True)):
        q = dict(p, sort_interval=K)
        case = pm.Case(q)
        if graph:
            case.step_rf_cycles(2)
        else:
            case.step(2 * p["steps_per_cycle"])
        runs.append(snapshot(case))
        case.close()
    for r in runs[1:]:
        assert_same(runs[0], r)


def test_diagnostics_window_matches_oracle(pm):
    """Averages of a one-step window from an identical state: densities from the
    integer charge sums, the potential to 1e-12, counts exactly."""
    p = W.discharge_small(seed=4)
    case = pm.Case(p)
    case.step(200)
    case.sample_diagnostics(reset=True)
    orc = oracle_from_gpu(case, p)
    orc.reset_diagnostics()
    rec = orc.step(record=True)
    case.step(1)
    g = case.sample_diagnostics()
    o = orc.sample_diagnostics()
    assert g["avg_steps"] == o["avg_steps"] == 1
    # ion impacts by energy and angle: equal but for impacts within 1e-4 of a bin
    # edge (FP32 on the GPU, FP64 in the oracle)
    near = 0
    if "lost_ion_E" in rec:
        for v in (rec["lost_ion_E"], rec["lost_ion_theta"] / 0.25):
            near += int(np.sum(np.abs(v - np.rint(v)) < 1e-4 * np.maximum(v, 1.0)))
    assert int(np.abs(g["iead"].astype(np.int64) - o["iead"]).sum()) <= 2 * near
    assert int(g["iead"].sum()) == int(o["iead"].sum())
    for k in ("ne", "ni"):
        assert np.allclose(g[k], o[k], rtol=1e-14, atol=0)
    assert np.max(np.abs(g["phi"] - o["phi"])) <= 1e-12 * max(np.max(np.abs(o["phi"])), 1.0)
    assert g["particle_steps"] == o["particle_steps"]
    assert np.array_equal(g["candidates"], o["candidates"])
    case.close()


# ---------------------------------------------------------------- failures
def test_capacity_exhaustion_is_sticky(pm):
    p = W.discharge_small(seed=6, fp64=False, flags=P.NO_SELF_FIELD)
    p.update(v0_volt=0.0, p_pa=10.0, capacity_e=5000, capacity_i=5000)
    case = pm.Case(p)
    info = case.info()
    ve = math.sqrt(2 * 60.0 * C.E_CHARGE / C.M_E) * info["dt"] / info["dx"]
    case.set_particles(0, _beam_state(5000, p["n_cells"], ve, np.random.default_rng(1), 0))
    case.step(1)
    with pytest.raises(pm.PicMccError) as e:
        case.sample_diagnostics()
    assert e.value.status == -4
    with pytest.raises(pm.PicMccError) as e2:
        case.step(1)
    assert e2.value.status == -6
    case.close()


def test_particle_count_query_and_null_arrays(pm):
    """pm_get_particles with no room returns PM_EINVAL and the live count; with
    room but a null array, PM_EINVAL; the case is untouched either way."""
    import ctypes as C
    case = pm.Case(W.discharge_small(seed=8, fp64=False))
    before = snapshot(case)
    pp = pm.pm_particles(n=0, capacity=0)
    assert pm.pm_get_particles(case.h, 0, C.byref(pp), None) == -1
    assert pp.n == len(before[0][0]["id"])
    pp = pm.pm_particles(n=0, capacity=10 ** 6)
    assert pm.pm_get_particles(case.h, 1, C.byref(pp), None) == -1
    assert_same(before, snapshot(case))
    case.close()


def test_stability_warnings_follow_the_limits(pm):
    """The limits of 'Limitations and Constraints' (Sec. IV.A), reported at init as
    warning bits: the cell against the Debye length (bit 1), omega_p dt against
    0.2 (bit 2) and at least 20 electrons per cell (bit 4), each computed here
    from its definition."""
    cases = [W.discharge_small(seed=5, fp64=False), W.discharge_working(np_each=100_000),
             dict(W.discharge_small(seed=5, fp64=False), np_e=1, np_i=0, capacity_e=256, capacity_i=400),
             dict(W.discharge_small(seed=5, fp64=False), n0_m3=1e13, steps_per_cycle=4000)]
    seen = set()
    for p in cases:
        lam_d = math.sqrt(C.EPS0 * p["te_ev"] / (p["n0_m3"] * C.E_CHARGE))
        w_p = math.sqrt(p["n0_m3"] * C.E_CHARGE ** 2 / (C.EPS0 * C.M_E))
        dx, dt = p["gap_m"] / p["n_cells"], 1.0 / (p["freq_hz"] * p["steps_per_cycle"])
        want = (1 if dx > lam_d else 0) | (2 if w_p * dt > 0.2 else 0) | (4 if p["np_e"] / p["n_cells"] < 20 else 0)
        case = pm.Case(p)
        assert int(case.sample_diagnostics()["warnings"]) == want, (p["n_cells"], p["np_e"], want)
        seen.add(want)
        case.close()
    assert len(seen) >= 3


def test_sort_cadence_counts_steps_across_calls(pm):
    """Dead slots are compacted by the cell sort, and births append past the last
    slot meanwhile.  A strongly ionising case with electron slots for 1.2 times
    its initial electrons outgrows them within 1200 steps when it never sorts;
    stepped one step per call with a sort interval of 25 it must keep sorting (the
    interval counts steps across calls) and stay within its slots."""
    p = W.discharge(0.025, 64, 500.0, 1000, 10.0, 2000, 1e15, seed=3, case_id=1)
    p.update(capacity_e=2400, capacity_i=8000)
    never = pm.Case(dict(p, sort_interval=0))
    never.step(1200)
    with pytest.raises(pm.PicMccError) as e:
        never.sample_diagnostics()
    assert e.value.status == -4
    never.close()
    case = pm.Case(dict(p, sort_interval=25))
    for _ in range(1200):
        case.step(1)
    d = case.sample_diagnostics()
    assert d["status"] == 0 and d["step"] == 1200
    assert d["births"] > 500 and d["n_e"] <= 2400
    case.close()


def test_sorts_of_a_population_that_outgrows_its_load(pm):
    """A sort launches one workgroup per 2048 initially loaded particles and
    grid-strides over whatever the slot range holds by then: a strongly ionising
    case (30 Pa, 1000 V) whose 1000 electrons grow several times over, sorted
    every 25 steps or every step by its one sort workgroup, holds bit for bit
    what it holds unsorted (sort interval 0, slots to spare)."""
    p = W.discharge(0.025, 64, 1000.0, 1000, 30.0, 1000, 1e14, seed=4, case_id=1)
    p.update(capacity_e=60000, capacity_i=60000, fp64=False)
    runs = []
    for K in (0, 25, 1):
        c = pm.Case(dict(p, sort_interval=K))
        c.step(1500)
        runs.append(snapshot(c))
        n_e = int(c.sample_diagnostics()["n_e"])
        c.close()
    assert n_e > 3 * 1000, n_e
    for r in runs[1:]:
        assert_same(runs[0], r)


def test_electrical_asymmetry_self_bias(pm):
    """The paper's drive V0 [cos(wt + dphi) + cos(2wt)] through a blocking
    capacitor (Sec. III, Sec. V): a geometrically symmetric discharge builds a DC
    self-bias (the time-averaged potential of the driven electrode) whose sign
    follows the phase -- negative at dphi = 0, positive at dphi = pi/2, where the
    waveform is the dphi = 0 one turned upside down."""
    bias = {}
    for dphi in (0.0, math.pi / 2):
        p = W.discharge_small(seed=8, fp64=False)
        p.update(v2_volt=p["v0_volt"], phase_rad=dphi, phase2_rad=0.0, cb_f_m2=5e-9)
        case = pm.Case(p)
        case.step_rf_cycles(150)
        case.sample_diagnostics(reset=True)
        case.step_rf_cycles(50)
        d = case.sample_diagnostics()
        assert d["status"] == 0
        bias[dphi] = float(d["phi"][0])
        case.close()
    V0 = W.discharge_small()["v0_volt"]
    assert bias[0.0] < -0.1 * V0 and bias[math.pi / 2] > 0.1 * V0, bias


def _peak_and_width(h, skip=20):
    """Energy of the highest bin above the lowest `skip` eV and the full width at
    half of it (1 eV bins)."""
    h = np.asarray(h, dtype=float)
    b = int(np.argmax(h[skip:])) + skip
    lo = hi = b
    while lo > 0 and h[lo] >= h[b] / 2:
        lo -= 1
    while hi < len(h) - 1 and h[hi] >= h[b] / 2:
        hi += 1
    return b + 0.5, float(hi - lo)


def test_paper_case_self_bias_and_ion_energies(pm):
    """The example discharge of Sec. III (75 mm, Ar 0.5 Pa 650 K, V0 [cos(wt) +
    cos(2wt)] with V0 = 300 V, blocking capacitor) shows the features Sec. V
    reports: a large negative DC self-bias from the electrically asymmetric drive
    (the paper: about 225 V), ions reaching the target with much more energy than
    the substrate (sheath drops of about 350 V and 125 V), narrow ion energy peaks
    (the width-to-peak ratio near 0.1 of hypothesis A), impacts within about a
    degree of the normal, and an ionisation degree below 1e-4 (hypothesis B).  The
    cross sections here are analytic stand-ins, so each check is qualitative, with
    margin; averages over RF cycles 400-600."""
    from oracle import constants as C
    p = W.discharge_paper()
    case = pm.Case(p)
    case.step_rf_cycles(400)
    case.sample_diagnostics(reset=True)
    case.step_rf_cycles(200)
    d = case.sample_diagnostics()
    assert d["status"] == 0
    bias = float(d["phi"][0])
    e_t, e_s = d["mean_ion_energy"]
    (pk_t, w_t), (pk_s, w_s) = (_peak_and_width(d["iedf"][el]) for el in (0, 1))
    med = []
    for el in (0, 1):
        cum = np.cumsum(d["iadf"][el]) / max(d["iadf"][el].sum(), 1)
        med.append(0.25 * (np.searchsorted(cum, 0.5) + 1))
    ion_deg = float(d["ni"].max()) / C.gas_density(p["p_pa"], p["t_gas_k"])
    print(f"paper case: bias {bias:.1f} V; mean ion energy target {e_t:.1f} eV, substrate {e_s:.1f} eV; "
          f"peaks {pk_t:.0f} / {pk_s:.0f} eV, width/peak {w_t / pk_t:.3f} / {w_s / pk_s:.3f}; "
          f"median angle {med[0]:.2f} / {med[1]:.2f} deg; n_i/n_Ar {ion_deg:.1e}")
    assert bias < -0.3 * p["v0_volt"], bias
    assert e_t > 1.5 * e_s > 75.0, (e_t, e_s)
    assert pk_t > 2.0 * pk_s > 150.0, (pk_t, pk_s)
    assert w_t / pk_t < 0.3 and w_s / pk_s < 0.3, (w_t, pk_t, w_s, pk_s)
    assert max(med) < 2.0, med
    assert ion_deg < 1e-4, ion_deg
    # the joint energy-angle histogram (Fig. 7): its marginals are the 1 eV and
    # 0.25 degree histograms grouped by 4, and at the target the ions of the
    # high-energy peak arrive within a couple of degrees of the normal
    iead = d["iead"].astype(np.int64)
    nb = d["iedf"].shape[1]
    for el in (0, 1):
        e_marg = np.concatenate([d["iedf"][el].astype(np.int64), np.zeros(-(-nb // 4) * 4 - nb, np.int64)])
        assert np.array_equal(iead[el].sum(axis=1), e_marg.reshape(-1, 4).sum(axis=1))
        assert np.array_equal(iead[el].sum(axis=0), d["iadf"][el].astype(np.int64).reshape(-1, 4).sum(axis=1))
    top = iead[0][int(0.8 * pk_t) // 4:]
    assert top[:, :2].sum() >= 0.9 * top.sum(), (top[:, :2].sum(), top.sum())
    case.close()
