"""Launch-shape autotuner: host logic on the CPU (signature and cache), and on an
MI355X a tuning run that leaves a valid shape and is then served from the cache."""
import json

import pytest

import workloads as W


def test_signature_separates_workloads():
    from paper_1607_04069_amd import autotune as A
    a = W.sweep_cases(8)
    assert A.signature(a) == A.signature(list(reversed(a)))          # order-free
    assert A.signature(a) != A.signature(a[:7])
    b = [dict(p, fp64=1) for p in a]
    assert A.signature(a) != A.signature(b)
    c = [dict(p, np_e=p["np_e"] * 4, np_i=p["np_i"] * 4) for p in a]
    assert A.signature(a) != A.signature(c)


def test_cache_round_trip(tmp_path, monkeypatch):
    from paper_1607_04069_amd import autotune as A
    path = tmp_path / "shapes.json"
    monkeypatch.setenv(A.CACHE_ENV, str(path))
    shape = dict(unroll=8, waves=6, work_groups=2048, deposit_mode=1, sort_interval=25)
    A._store("dev|batch|x", shape, 1.0e11)
    A._store("dev|case|y", dict(shape, unroll=16), 5.0e10)
    data = json.loads(path.read_text())
    assert data["dev|batch|x"]["shape"] == shape
    assert A._load()["dev|case|y"]["shape"]["unroll"] == 16


@pytest.mark.gpu
def test_tune_small_batch_then_cache(tmp_path, monkeypatch):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_04069_amd as pm
    from paper_1607_04069_amd import autotune as A
    monkeypatch.setenv(A.CACHE_ENV, str(tmp_path / "shapes.json"))
    ps = W.sweep_cases(4)
    cases = [pm.Case(p) for p in ps]
    b = pm.Batch(cases)
    shape, rate, src = A.tune(b, ps, steps=25)
    assert src == "timed" and rate > 0
    assert shape["unroll"] in (8, 16) and shape["waves"] in (0, 6) and shape["work_groups"] >= 1
    assert b.launch_shape() == shape
    b.set_launch_shape(unroll=8, waves=0, work_groups=0)
    shape2, _, src2 = A.tune(b, ps)
    assert src2 == "cache" and shape2["unroll"] == shape["unroll"] and shape2["waves"] == shape["waves"]
    b.close()
    for c in cases:
        c.close()
