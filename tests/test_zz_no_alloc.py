"""The test-particle entry point that allocates nothing (runs on an MI355X).

pm_run_test_particles_static keeps its tallies in the library's per-GPU static
scratch instead of a caller's arena.  Called through the C interface, it must
return exactly what pm_run_test_particles returns for the same arguments --
counts, histograms, energy sums and the density and mean-velocity profiles --
on two calls in a row, the second smaller than the first (so that nothing of
the first call's tallies may survive in the shared scratch), and it must not
grow torch's device memory.
"""
import ctypes as C

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


def _same(a, b):
    assert set(a) == set(b)
    for k in a:
        if isinstance(a[k], np.ndarray):
            assert np.array_equal(a[k], b[k]), k
        else:
            assert a[k] == b[k], (k, a[k], b[k])


def test_static_scratch_equals_the_arena_form(pm):
    import torch
    calls = ((2.0, 200_000, 100, 200), (0.5, 30_000, 40, 120))      # the second call is smaller
    for p_pa, n_atoms, n_xbins, n_ebins in calls:
        src, tp = W.sputter_transport(p_pa=p_pa, n_atoms=n_atoms)
        src["flux_m2s"] = 3.0e18
        tp.update(n_xbins=n_xbins, n_ebins=n_ebins, n_tbins=n_ebins)
        print(f"static scratch: {p_pa} Pa, {n_atoms} atoms, {n_xbins} cells", flush=True)
        ref = pm.run_test_particles(src, tp)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        got = pm.run_test_particles_static(src, tp)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        _same(got, ref)
        assert got["n_substrate"] + got["n_target"] + got["n_unfinished"] == n_atoms
        assert np.all(got["density_m3"] > 0)


def test_static_scratch_rejects_what_does_not_fit(pm):
    src, tp = W.sputter_transport(n_atoms=10)
    tp.update(n_ebins=200_000)                # 1.6 MB of energy bins
    res = pm.pm_tp_result()
    st = pm.pm_run_test_particles_static(C.byref(pm.tp_params(tp)), C.byref(pm.tp_source(src)), None,
                                         C.byref(res))
    assert st == -2                           # PM_ENOSPACE
