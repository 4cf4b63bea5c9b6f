"""The served stream (continuous batching) against each request alone (runs on an
MI355X).  A discharge served in the mix -- admitted while others run, batched
with whatever is resident, retired on its own schedule -- must return exactly
what it returns alone; a test-particle job run beside the discharges must
return exactly its tallies alone."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_04069_amd as mod
    return mod


def small_discharge(i, rng):
    n_cells = int(rng.choice([64, 128]))
    v0 = rng.uniform(80.0, 200.0)
    p_pa = math.exp(rng.uniform(math.log(1.0), math.log(5.0)))
    np_each = int(rng.uniform(3000, 8000))
    return W.discharge(0.03, n_cells, v0, 400, p_pa, np_each, 2e15, case_id=500 + i)


def small_tpm(i, rng):
    src, tp = W.sputter_transport(p_pa=rng.uniform(0.5, 3.0), n_atoms=20000, job_id=500 + i)
    return {"src": src, "tp": tp}


def test_served_results_equal_alone(pm):
    from paper_1607_04069_amd import serve
    reqs = serve.poisson_stream(12, 40.0, small_discharge, small_tpm, seed=11)
    kinds = [r.kind for r in reqs]
    assert "tpm" in kinds and kinds.count("discharge") >= 4
    srv = serve.Server(pm, cycles_budget=3, max_slots=3)
    summary = srv.run(reqs)
    assert summary["discharge_count"] == kinds.count("discharge")
    assert 0 < summary["latency_p50_s"] <= summary["latency_p99_s"]
    for r in reqs:
        assert r.done >= r.arrival and r.result is not None
        if r.kind == "discharge":
            ref = serve.run_alone(pm, r.params, 3)
            assert r.result["step"] == ref["step"] == 3 * 400
            for k in ("ne", "ni", "phi", "iedf", "iadf", "collisions", "absorbed", "avg_steps"):
                assert np.array_equal(np.asarray(r.result[k]), np.asarray(ref[k])), (r.rid, k)
        else:
            ref = pm.run_test_particles(r.params["src"], r.params["tp"])
            for k in ("n_substrate", "n_target", "events", "collisions"):
                assert r.result[k] == ref[k], (r.rid, k)
            assert np.array_equal(r.result["e_hist"], ref["e_hist"])


def test_admission_respects_slots_and_memory(pm):
    from paper_1607_04069_amd import serve
    reqs = serve.poisson_stream(6, 1000.0, small_discharge, small_tpm, tpm_fraction=0.0, seed=12)
    seen = []
    srv = serve.Server(pm, cycles_budget=2, max_slots=2, log=seen.append)
    srv.run(reqs)
    sizes = [int(s.split("batch of ")[1].split()[0]) for s in seen if "batch of " in s]
    assert max(sizes) == 2
    assert any("6 of 6 discharges done" in s for s in seen)
    # a memory budget of the largest case of the stream admits one case at a time
    reqs = serve.poisson_stream(4, 1000.0, small_discharge, small_tpm, tpm_fraction=0.0, seed=13)
    fp = max(srv._footprint(r.params) for r in reqs)
    seen.clear()
    srv = serve.Server(pm, cycles_budget=2, max_slots=8, hbm_budget_bytes=fp, log=seen.append)
    srv.run(reqs)
    admitted = [s for s in seen if "batch of " in s]
    assert admitted and all(int(s.split("batch of ")[1].split()[0]) == 1 for s in admitted)
    # a request that the whole budget cannot hold is refused, not queued forever
    reqs = serve.poisson_stream(4, 1000.0, small_discharge, small_tpm, tpm_fraction=0.0, seed=13)
    fps = [srv._footprint(r.params) for r in reqs]
    summ = serve.Server(pm, cycles_budget=2, max_slots=8, hbm_budget_bytes=min(fps)).run(reqs)
    refused = [r for r, f in zip(reqs, fps) if f > min(fps)]
    assert refused and summ["failed"] == len(refused)
    assert all("does not fit" in r.result["error"] for r in refused)
    assert all("error" not in r.result for r, f in zip(reqs, fps) if f == min(fps))


def test_a_failed_case_leaves_the_stream_running(pm):
    """A case that runs out of particle slots (hot electrons in dense gas, every
    slot in use from the start) fails while served; it leaves the batch with its
    error and the other requests of the stream still return what they return
    alone."""
    from paper_1607_04069_amd import serve
    from oracle import pic as P

    def make(i, rng):
        if i == 1:
            p = W.discharge(0.03, 64, 100.0, 400, 10.0, 3000, 2e15, case_id=599, flags=P.NO_SELF_FIELD,
                            capacity_factor=1)
            p["te_ev"] = 60.0
            return p
        return small_discharge(i, rng)

    reqs = serve.poisson_stream(4, 1000.0, make, small_tpm, tpm_fraction=0.0, seed=21)
    summ = serve.Server(pm, cycles_budget=2, max_slots=4).run(reqs)
    assert summ["failed"] == 1
    bad = [r for r in reqs if r.rid == 1][0]
    assert "error" in bad.result and "PM_ECAPACITY" in bad.result["error"]
    for r in reqs:
        if r.rid == 1:
            continue
        ref = serve.run_alone(pm, r.params, 2)
        for k in ("ne", "ni", "phi", "iedf", "flux"):
            assert np.array_equal(np.asarray(r.result[k]), np.asarray(ref[k])), (r.rid, k)
