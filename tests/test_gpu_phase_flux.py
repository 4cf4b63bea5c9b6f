"""Phase-resolved averages and flux profiles (Sec. IV averaging, Fig. 8) on the
GPU against the oracle.

A window of single steps: before each step the oracle takes the GPU's own state
and runs that step, and its per-step sums are added up on the host, so the
expected window holds exactly what the GPU's steps started from.  Densities
come from integer charge sums (equal to 1e-14); the potential to 1e-12 of its
scale; the flux profiles carry one rounding of the fixed-point weight per
particle (2^-33 of the particle's velocity) and of its 2^-40 velocity unit,
checked to 1e-8 of the profile's largest value.
"""
import numpy as np
import pytest

from oracle import pic as P
import workloads as W
from tests.gpu_helpers import oracle_from_gpu

pytestmark = pytest.mark.gpu

SUM_KEYS = ("sumQ", "sumPhi", "sumQ_phase", "sumPhi_phase", "n_phase", "sumF", "n_flux")


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_04069_amd as mod
    return mod


def _params(fp64, seed):
    p = W.discharge_small(seed=seed, fp64=fp64)
    p.update(n_phase=100, flux_profiles=1)       # 4 steps per bin at N_t = 400
    return p


def _expected_window(case, p, n_steps):
    """Step the case n_steps times; the oracle's sums of the same steps, each
    taken from the GPU's state before the step."""
    tot = P.Discharge(p, load=False)
    for _ in range(n_steps):
        orc = oracle_from_gpu(case, p)
        orc.step()
        for k in SUM_KEYS:
            tot.acc[k] = tot.acc[k] + orc.acc[k]
        tot.acc["n_steps"] += orc.acc["n_steps"]
        case.step(1)
    return tot


def _compare(g, o, label):
    for k in ("ne", "ni"):
        assert np.allclose(g[k], o[k], rtol=1e-14, atol=0), (label, k)
    assert np.max(np.abs(g["phi"] - o["phi"])) <= 1e-12 * max(np.max(np.abs(o["phi"])), 1.0), label
    for key, dens in (("e", o["ne"]), ("i", o["ni"])):
        go, gg = o["gamma_" + key], g["gamma_" + key]
        tol = 1e-8 * max(np.max(np.abs(go)), 1.0)
        assert np.max(np.abs(gg - go)) <= tol, (label, key, np.max(np.abs(gg - go)), tol)
        held = dens > 0
        assert np.all(g["u_" + key][~held] == 0), (label, key)
        assert np.all(np.abs(g["u_" + key][held] - o["u_" + key][held]) <= tol / dens[held]
                      + 1e-12 * np.abs(o["u_" + key][held])), (label, key)


@pytest.mark.parametrize("fp64", [True, False])
def test_phase_bins_and_flux_window_match_oracle(pm, fp64):
    p = _params(fp64, seed=21 if fp64 else 22)
    case = pm.Case(p)
    case.step(198)
    case.sample_diagnostics(reset=True)
    print(f"phase/flux window, fp64={fp64}", flush=True)
    tot = _expected_window(case, p, 10)             # steps 198..207: bins 49, 50, 51
    for b in (49, 50, 51, 52, 0):
        g = case.sample_phase(b)
        o = tot.sample_phase(b)
        assert g["n_steps"] == o["n_steps"] and g["n_flux_samples"] == o["n_flux_samples"], b
        assert g["status"] == 0
        _compare(g, o, f"bin {b}")
    assert [case.sample_phase(b)["n_steps"] for b in (49, 50, 51, 52)] == [2, 4, 4, 0]
    g = case.sample_diagnostics()
    o = tot.sample_diagnostics()
    assert g["avg_steps"] == o["avg_steps"] == 10
    _compare(g, o, "window")
    case.close()


def test_flux_sums_are_order_free_across_launch_paths(pm):
    """Integer flux and phase sums: stepping one RF period as single launches or as
    the captured graph gives bit-identical profiles."""
    p = _params(False, seed=23)
    out = []
    for graph in (False, True):
        case = pm.Case(p)
        case.sample_diagnostics(reset=True)
        if graph:
            case.step_rf_cycles(1)
        else:
            case.step(p["steps_per_cycle"])
        d = case.sample_diagnostics()
        ph = case.sample_phase(37)
        out.append((d, ph))
        case.close()
    (d0, p0), (d1, p1) = out
    for k in ("ne", "ni", "phi", "gamma_e", "gamma_i", "u_e", "u_i"):
        assert np.array_equal(d0[k], d1[k]), k
        assert np.array_equal(p0[k], p1[k]), k
    assert p0["n_steps"] == p0["n_flux_samples"] == 4
    assert np.any(d0["gamma_i"] != 0)


def test_phase_and_flux_interface_errors(pm):
    p = _params(False, seed=24)
    case = pm.Case(p)
    for bad in (-1, 100):
        with pytest.raises(pm.PicMccError):
            case.sample_phase(bad)
    with pytest.raises(pm.PicMccError):
        pm.Batch([case])                             # flux samples need the single-case steps
    plain = pm.Case(W.discharge_small(seed=25, fp64=False))
    with pytest.raises(pm.PicMccError):
        plain.sample_phase(0)                        # no phase bins kept
    d = plain.sample_diagnostics()
    assert np.all(d["gamma_e"] == 0) and np.all(d["u_i"] == 0)
    plain.close()
    case.close()


@pytest.mark.parametrize("n_phase", [1, 128])
def test_one_bin_is_the_window_and_bins_partition_it(pm, n_phase):
    """With one phase bin that bin is the window, bit for bit; with the most bins
    (128, which do not divide N_t = 400) every bin of a whole period holds 3 or 4
    steps as floor((l mod N_t) n_phase / N_t) assigns them, and the bins weighted
    by their steps give the window's averages."""
    p = dict(W.discharge_small(seed=26, fp64=False), n_phase=n_phase, flux_profiles=1)
    Nt = p["steps_per_cycle"]
    case = pm.Case(p)
    case.step(123)
    case.sample_diagnostics(reset=True)
    case.step(Nt)
    d = case.sample_diagnostics()
    keys = ("ne", "ni", "phi", "gamma_e", "gamma_i")
    if n_phase == 1:
        b = case.sample_phase(0)
        assert b["n_steps"] == b["n_flux_samples"] == d["avg_steps"] == Nt
        for k in keys:
            assert np.array_equal(b[k], d[k]), k
    else:
        want = np.bincount((np.arange(Nt) * n_phase) // Nt, minlength=n_phase)
        acc = {k: np.zeros_like(d[k]) for k in keys}
        for i in range(n_phase):
            b = case.sample_phase(i)
            assert b["n_steps"] == b["n_flux_samples"] == want[i], i
            for k in keys:
                acc[k] += b[k] * b["n_steps"]
        for k in keys:
            scale = max(np.max(np.abs(d[k])), 1.0)
            assert np.max(np.abs(acc[k] / Nt - d[k])) <= 1e-12 * scale, k
    case.close()
