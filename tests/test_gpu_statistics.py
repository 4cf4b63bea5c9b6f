"""Long-run statistical parity, GPU vs oracle (runs on an MI355X).

Past a few hundred steps the GPU run and the oracle are different realisations
of the same stochastic process (rounding differences grow chaotically), so they
are compared statistically.  The oracle's runs are stored as two pools of seeds
per workload (tests/golden/, written by make_discharge_stats.py from the oracle
alone); the GPU runs the seeds of pool A -- all of them in one batch -- over the
same warm-up and averaging window, and its pooled time-averaged density
profiles, ion energy distributions at both electrodes (Kolmogorov-Smirnov
distance), mean ion energies, wall fluxes and, behind a blocking capacitor, the
DC self-bias must each come within 3 % of the oracle's pool A.  The oracle's
own distance between its pools A and B and its standard error (from the
seeds' scatter) are printed beside each; test_golden_stats.py checks on the CPU
that the standard errors are at most 1 %.

Workloads: the small discharge (64 cells, 5k + 5k, 1 Pa, 100 V; in FP64 and in
FP32), the same with the paper's drive (two harmonics through a blocking
capacitor), the working-size discharge (1M + 1M, 1024 cells, 0.5 Pa, 300 V;
20 RF cycles), and the batched sweep's two corners (10 Pa at 500 V, 0.5 Pa at
50 V; 256 cells, 5e4 + 5e4).
"""
import numpy as np
import pytest

from tests import golden_stats as G

pytestmark = pytest.mark.gpu

CASES = [("small", True), ("small", False), ("small_eae", False), ("working", False), ("corner_hi", False),
         ("corner_lo", False)]


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_04069_amd as mod
    return mod


def _gpu_pool(pm, pool, fp64):
    """The pool's seeds on the GPU, batched, over the pool's warm-up and window."""
    params = [dict(p, fp64=int(fp64)) for p in pool["params"]]
    nt = params[0]["steps_per_cycle"]
    warm, window = int(pool["warm"]), int(pool["window"])
    assert warm % nt == 0 and window % nt == 0
    cases = [pm.Case(p) for p in params]
    batch = pm.Batch(cases) if len(cases) > 1 else None
    stepper = batch if batch is not None else cases[0]
    stepper.step_rf_cycles(warm // nt)
    for c in cases:
        c.sample_diagnostics(reset=True)
    stepper.step_rf_cycles(window // nt)
    out = [c.sample_diagnostics() for c in cases]
    if batch is not None:
        batch.close()
    for c in cases:
        c.close()
    for o in out:
        assert o["status"] == 0 and o["avg_steps"] == window
    return out


@pytest.mark.parametrize("name,fp64", CASES, ids=[f"{n}-{'fp64' if f else 'fp32'}" for n, f in CASES])
def test_long_run_statistics_match_oracle(pm, name, fp64):
    a, b = G.load_pool(name, "A"), G.load_pool(name, "B")
    if a is None or b is None:
        pytest.skip(f"oracle statistics for {name} not generated")
    assert str(a["oracle_sha256"]) == G.oracle_sha256(), "statistics written by another oracle"
    print(f"{name} fp64={fp64}: {len(a['seeds'])} seeds, warm {int(a['warm'])}, window {int(a['window'])}",
          flush=True)
    g = G.pooled(_gpu_pool(pm, a, fp64))
    bias = a["params"][0].get("cb_f_m2", 0.0) > 0
    d = G.distances(g, G.pooled(a), self_bias=bias)
    spread = G.distances(G.pooled(b), G.pooled(a), self_bias=bias)
    noise = G.noise(a, self_bias=bias) if len(a["seeds"]) >= 4 else spread
    for k in d:
        print(f"  {k}: GPU-oracle {d[k]:.4f} (oracle: pool-to-pool {spread[k]:.4f}, standard error {noise[k]:.4f})")
    bad = {k: v for k, v in d.items() if v > G.TOL}
    assert not bad, bad
