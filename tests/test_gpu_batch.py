"""Batched stepping against each case alone (runs on an MI355X).

A batch advances independent cases with one launch per time step.  Each case
draws its random numbers from (seed, case_id, particle id, step) and sums its
charge in integers, so its state -- particles compared by id, the grid, the
diagnostics -- must be bit-identical whether it ran alone or in a batch, with
any number of workgroups and any neighbours.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import assert_same, snapshot

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_04069_amd as mod
    return mod


def mixed_cases(fp64=False):
    """Three unlike cases sharing N_t = 400 and the sort interval: different grids,
    sizes, voltages, pressures and seeds."""
    return [W.discharge_small(seed=11, fp64=fp64),
            W.discharge(0.04, 128, 250.0, 400, 3.0, 20000, 4e15, seed=11, case_id=201, fp64=fp64),
            W.discharge(0.03, 256, 80.0, 400, 8.0, 8000, 2e15, seed=12, case_id=202, fp64=fp64)]


def _alone(pm, ps, run):
    out = []
    for p in ps:
        c = pm.Case(p)
        run(c)
        out.append(snapshot(c))
        c.close()
    return out


@pytest.mark.parametrize("fp64", [False, True])
def test_batch_steps_match_each_case_alone(pm, fp64):
    ps = mixed_cases(fp64)
    ref = _alone(pm, ps, lambda c: c.step(60))          # two sorts inside the call
    cases = [pm.Case(p) for p in ps]
    b = pm.Batch(cases)
    info = b.info()
    assert info["n_cases"] == 3 and sum(info["case_workgroups"]) <= info["step_workgroups"]
    assert min(info["case_workgroups"]) >= 1
    b.step(60)
    for c, r in zip(cases, ref):
        assert_same(r, snapshot(c))
    b.close()
    for c in cases:
        c.close()


def test_a_nan_fails_only_its_case(pm):
    """Failure detection: a NaN velocity written from the host into one case of a
    batch fails that case alone.  It reports PM_ENUMERIC at its next
    synchronising call and PM_ESTATE after, the batch refuses to step on, and its
    two neighbours hold exactly what they hold after the same steps alone."""
    ps = mixed_cases()
    ref = _alone(pm, [ps[0], ps[2]], lambda c: c.step(5))
    cases = [pm.Case(p) for p in ps]
    g = cases[1].get_particles(0)
    g["ux"][17] = np.nan
    cases[1].set_particles(0, g)
    b = pm.Batch(cases)
    b.step(5)
    for c, r in zip((cases[0], cases[2]), ref):
        assert_same(r, snapshot(c))
    with pytest.raises(pm.PicMccError) as e:
        cases[1].sample_diagnostics()
    assert e.value.status == -5
    with pytest.raises(pm.PicMccError) as e2:
        cases[1].step(1)
    assert e2.value.status == -6
    with pytest.raises(pm.PicMccError) as e3:
        b.step(1)
    assert e3.value.status == -6
    b.close()
    for c in cases:
        c.close()


def test_a_batch_member_rewound_from_a_checkpoint(pm):
    """A member of a batch rewound to a checkpoint taken 100 steps earlier steps on
    with its neighbours (each case keeps its own step count), and after 100 more
    batched steps it equals the same case run 200 steps alone; the neighbours,
    now 100 steps ahead of it, equal their own 300-step runs alone."""
    ps = mixed_cases()
    ref = _alone(pm, ps, lambda c: c.step(300))
    ref_back = _alone(pm, [ps[1]], lambda c: c.step(200))[0]
    cases = [pm.Case(p) for p in ps]
    b = pm.Batch(cases)
    b.step(100)
    saved = cases[1].save_checkpoint()
    b.step(100)
    cases[1].load_checkpoint(saved)
    b.step(100)
    assert_same(ref_back, snapshot(cases[1]))
    for i in (0, 2):
        assert_same(ref[i], snapshot(cases[i]))
    b.close()
    for c in cases:
        c.close()


def extreme_cases():
    """A one-cell grid, the largest grid, a single electron and a 777-cell grid,
    all on the small discharge's clock (N_t = 400)."""
    out = []
    for k, (n_cells, np_e, np_i) in enumerate(((1, 400, 400), (1024, 3000, 3000), (64, 1, 0), (777, 5003, 4997))):
        p = W.discharge_small(seed=17, fp64=False)
        p.update(n_cells=n_cells, np_e=np_e, np_i=np_i, case_id=301 + k,
                 capacity_e=max(4 * np_e, 256), capacity_i=4 * max(np_i, 100))
        out.append(p)
    return out


def test_batch_of_extreme_cases_matches_alone(pm):
    ps = extreme_cases()
    ref = _alone(pm, ps, lambda c: c.step(60))
    cases = [pm.Case(p) for p in ps]
    b = pm.Batch(cases)
    b.step(60)
    for c, r in zip(cases, ref):
        assert_same(r, snapshot(c))
    b.close()
    for c in cases:
        c.close()


@pytest.mark.parametrize("lanes", [1, 3])
def test_batch_graph_then_alone_steps_match(pm, lanes):
    """An RF cycle of the batch from its graph (the lanes forked from and joined
    into the caller's stream), then each case continues alone."""
    ps = mixed_cases()
    ref = _alone(pm, ps, lambda c: c.step(430))
    cases = [pm.Case(p) for p in ps]
    b = pm.Batch(cases)
    b.set_launch_shape(lanes=lanes)
    assert b.launch_shape()["lanes"] == lanes
    b.step_rf_cycles(1)
    for c in cases:
        c.step(30)
    for c, r in zip(cases, ref):
        assert_same(r, snapshot(c))
    b.close()
    for c in cases:
        c.close()


def test_batch_order_and_neighbours_do_not_matter(pm):
    ps = mixed_cases()
    a = [pm.Case(p) for p in ps]
    b = [pm.Case(p) for p in reversed(ps)]
    ba, bb = pm.Batch(a), pm.Batch(b[:2])        # case 0 of ps is absent from the second batch
    ba.step(50)
    bb.step(50)
    sa = [snapshot(c) for c in a]
    sb = [snapshot(c) for c in b[:2]]
    assert_same(sa[2], sb[0])
    assert_same(sa[1], sb[1])
    for x in (ba, bb):
        x.close()
    for c in a + b:
        c.close()


def test_batch_rejects_unlike_or_repeated_cases(pm):
    p32 = W.discharge_small(seed=1, fp64=False)
    p64 = W.discharge_small(seed=1, fp64=True)
    c32, c64 = pm.Case(p32), pm.Case(p64)
    c25 = pm.Case(dict(p32, sort_interval=10, case_id=9))
    for group in ([c32, c64], [c32, c32]):
        with pytest.raises(pm.PicMccError):
            pm.Batch(group)
    b = pm.Batch([c32, c25])                 # cases of unlike sort intervals may share a batch
    for bad in (dict(unroll=4), dict(waves=2), dict(deposit_mode=2), dict(sort_interval=-1), dict(lanes=5)):
        with pytest.raises(pm.PicMccError):
            b.set_launch_shape(**bad)
    b.close()
    # a batch of one is the plain case
    ref = _alone(pm, [p32], lambda c: c.step(30))[0]
    one = pm.Batch([c32])
    one.step(30)
    assert_same(ref, snapshot(c32))
    one.close()
    for c in (c32, c64, c25):
        c.close()


def test_batch_of_sweep_cases_matches_alone(pm):
    """Eight of the sweep's cases (N from 128 to 1024, 20k-500k particles per
    species, 0.5-10 Pa) for 30 steps, batched and alone."""
    ps = W.sweep_cases()[:8]
    ref = _alone(pm, ps, lambda c: c.step(30))
    cases = [pm.Case(p) for p in ps]
    b = pm.Batch(cases)
    b.step(30)
    for c, r in zip(cases, ref):
        assert_same(r, snapshot(c))
    n = np.array(b.info()["case_workgroups"])
    assert np.all(n >= 1)
    b.close()
    for c in cases:
        c.close()


SHAPES = [dict(unroll=16), dict(waves=6), dict(deposit_mode=0), dict(deposit_mode=1), dict(work_groups=3),
          dict(sort_interval=7, unroll=16, waves=6), dict(lanes=2), dict(lanes=4, waves=6, work_groups=5)]


def test_launch_shapes_change_nothing_but_speed(pm):
    """Every launch shape of a case, and of a batch, gives the same state."""
    ps = mixed_cases()
    ref = _alone(pm, ps, lambda c: c.step(40))
    for sh in SHAPES:
        c = pm.Case(ps[1])
        c.set_launch_shape(**sh)
        got = c.launch_shape()
        assert all(got[k] == v for k, v in sh.items() if k not in ("work_groups", "lanes"))
        assert got["lanes"] == 1                   # a case has one lane
        c.step(40)
        assert_same(ref[1], snapshot(c))
        c.close()
    for sh in SHAPES:
        cases = [pm.Case(p) for p in ps]
        b = pm.Batch(cases)
        b.set_launch_shape(**dict(sh, work_groups=sh.get("work_groups", 0) * 4))
        b.step(40)
        for c, r in zip(cases, ref):
            assert_same(r, snapshot(c))
        b.close()
        for c in cases:
            c.close()


def test_graph_follows_a_new_shape(pm):
    p = mixed_cases()[0]
    ref = _alone(pm, [p], lambda c: c.step(800))[0]
    c = pm.Case(p)
    c.step_rf_cycles(1)
    c.set_launch_shape(unroll=16, waves=6, work_groups=2)
    c.step_rf_cycles(1)
    assert_same(ref, snapshot(c))
    c.close()


def test_slot_workgroups_take_over_when_a_share_overflows(pm):
    """One working workgroup for 200k particles: a workgroup walks at most 65532
    slots, so the workgroups that only hold slots take the rest.  The state must
    equal the default launch's."""
    p = W.discharge_working(np_each=100_000)
    ref = _alone(pm, [p], lambda c: c.step(30))[0]
    c = pm.Case(p)
    c.set_launch_shape(work_groups=1, sort_interval=7)
    assert c.launch_shape()["work_groups"] == 1
    c.step(30)
    assert_same(ref, snapshot(c))
    c.close()
    cases = [pm.Case(p), pm.Case(W.discharge_small(seed=11, fp64=False))]
    b = pm.Batch(cases)
    b.set_launch_shape(work_groups=2, lanes=2)
    b.step(30)
    assert_same(ref, snapshot(cases[0]))
    b.close()
    for x in cases:
        x.close()


def test_full_sweep_step_matches_oracle_on_sampled_cases(pm):
    """The benchmark's workload at its full size and launch shape: all 64 sweep
    cases (about 1.5e7 particles) in one batch with the tuned shape, one RF cycle
    from the graph, then one more batched step checked against the oracle on four
    cases spread over the sizes (each sampled case whole: the oracle takes the
    GPU's state before the step and steps it), to the single-step bar."""
    from oracle import pic as P
    from paper_1607_04069_amd import autotune
    from tests.gpu_helpers import oracle_from_gpu
    from tests.test_gpu_pic import compare_step
    ps = W.sweep_cases()
    cases = [pm.Case(p) for p in ps]
    b = pm.Batch(cases)
    autotune.tune(b, ps, use_cache=True)
    b.step_rf_cycles(1)
    order = sorted(range(len(ps)), key=lambda i: ps[i]["np_e"])
    pick = [order[k] for k in (0, len(ps) // 3, 2 * len(ps) // 3, len(ps) - 1)]
    pre = {}
    for i in pick:
        print(f"sampled case {i}: {ps[i]['np_e']} particles per species, {ps[i]['n_cells']} cells", flush=True)
        orc = oracle_from_gpu(cases[i], ps[i])
        before = cases[i].sample_diagnostics()
        acc0 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in orc.acc.items()}
        rec = orc.step(record=True)
        rec["acc0"] = acc0
        pre[i] = (orc, rec, before)
    b.step(1)
    n_ties = {"count": 0}
    n_cand = 0
    for i in pick:
        orc, rec, before = pre[i]
        compare_step(cases[i], ps[i], orc, rec, before, cases[i].sample_diagnostics(), n_ties)
        n_cand += int(sum(len(rec.get(f"cand_id_{s}", [])) for s in (0, 1)))
    assert n_cand > 0
    assert n_ties["count"] <= max(2, n_cand // 100)
    b.close()
    for c in cases:
        c.close()


def test_slotted_batch_members_come_and_go(pm):
    """A slotted batch keeps one RF-cycle graph while cases join and leave its
    slots; each case still computes exactly what it computes alone for the
    number of cycles it was a member."""
    ps = mixed_cases()
    cycles = {0: 3, 1: 2, 2: 2}
    ref = [_alone(pm, [p], lambda c, k=cycles[i]: c.step_rf_cycles(k))[0] for i, p in enumerate(ps)]
    cases = [pm.Case(p) for p in ps]
    b = pm.SlotBatch(3, 400, max_cells=256)
    b.set_launch_shape(lanes=2)
    b.step_rf_cycles(1)                      # an empty batch steps nothing
    b.set_slot(1, cases[0])
    b.step_rf_cycles(1)                      # case 0: 1
    b.set_slot(0, cases[1])
    b.step_rf_cycles(1)                      # case 0: 2, case 1: 1
    b.set_slot(2, cases[2])
    b.step_rf_cycles(1)                      # case 0: 3, case 1: 2, case 2: 1
    b.set_slot(1, None)
    b.set_slot(0, None)
    info = b.info()
    assert info["n_cases"] == 3 and info["case_workgroups"][0] == info["case_workgroups"][1] == 0
    b.step_rf_cycles(1)                      # case 2: 2
    for c, r in zip(cases, ref):
        assert_same(r, snapshot(c))
    with pytest.raises(pm.PicMccError):
        b.set_slot(0, cases[2])              # already in slot 2
    b.close()
    for c in cases:
        c.close()
