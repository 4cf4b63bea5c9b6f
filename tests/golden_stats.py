"""Pooled long-run statistics of discharge runs and their distances (Sec. IV:
time averages over a window once the run has settled).

A pool is several seeds of one workload, each averaged over the same window;
its statistics are the seeds' pooled averages: the mean density profiles, the
summed ion impact energy histograms, the impact-weighted mean ion energy, the
mean wall fluxes and the mean driven-electrode potential (the DC self-bias
behind a blocking capacitor).  Two pools are compared by
  * density: the largest difference of the profiles, each averaged over 16
    equal spatial bins, relative to the profile's peak, per species;
  * ion energy distribution: the Kolmogorov-Smirnov distance of the pooled
    histograms at each electrode;
  * mean ion energy and wall flux (per species and electrode): relative
    differences;
  * DC self-bias: relative difference.
The stored oracle pools are written by tests/golden/make_discharge_stats.py,
which calls only the oracle.
"""
import glob
import hashlib
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_FILES = ("constants.py", "philox.py", "pic.py", "xsec.py")
BINS = 16
TOL = 0.03          # the stated bar on every metric
NOISE_BAR = 0.01    # the largest standard error of an oracle pool's metric (bootstrap over its seeds)


def oracle_sha256():
    h = hashlib.sha256()
    for f in ORACLE_FILES:
        with open(os.path.join(ROOT, "oracle", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def load_pool(name, which):
    path = os.path.join(GOLDEN, f"discharge_{name}_pool{which}.npz")
    if not os.path.exists(path):
        return None
    z = np.load(path)
    d = {k: z[k] for k in z.files}
    d["params"] = [json.loads(str(s)) for s in d["params"]]
    return d


def available(names):
    return [n for n in names if glob.glob(os.path.join(GOLDEN, f"discharge_{n}_poolA.npz"))
            and glob.glob(os.path.join(GOLDEN, f"discharge_{n}_poolB.npz"))]


def _coarse(n, bins=BINS):
    k = (len(n) - 1) // bins
    return np.array([n[i * k:(i + 1) * k + 1].mean() for i in range(bins)])


def pooled(runs):
    """Pooled statistics of per-seed results (a stored pool, or a list of dicts)."""
    if isinstance(runs, dict):
        get = lambda k: np.asarray(runs[k])
    else:
        get = lambda k: np.stack([np.asarray(r[k]) for r in runs])
    absorbed = get("absorbed").astype(np.float64)                 # [seed][species][electrode]
    energy = get("mean_ion_energy") * absorbed[:, 1, :]           # impact energy sums per electrode
    n_imp = absorbed[:, 1, :].sum(axis=0)
    return {"ne": get("ne").mean(axis=0), "ni": get("ni").mean(axis=0),
            "iedf": get("iedf").astype(np.float64).sum(axis=0),
            "mean_ion_energy": np.where(n_imp > 0, energy.sum(axis=0) / np.maximum(n_imp, 1), 0.0),
            "flux": get("flux").mean(axis=0), "phi0": float(get("phi")[:, 0].mean()),
            "impacts": n_imp}


def ks(h1, h2):
    c1 = np.cumsum(h1) / max(h1.sum(), 1)
    c2 = np.cumsum(h2) / max(h2.sum(), 1)
    return float(np.max(np.abs(c1 - c2)))


def distances(a, b, self_bias=False):
    """Every metric's distance of pool a from pool b (relative to b)."""
    d = {}
    for k in ("ne", "ni"):
        ca, cb = _coarse(a[k]), _coarse(b[k])
        d[f"profile_{k}"] = float(np.max(np.abs(ca - cb)) / np.max(cb))
    for el in (0, 1):
        if b["impacts"][el] > 0:
            d[f"iedf_ks_{el}"] = ks(a["iedf"][el], b["iedf"][el])
            d[f"mean_energy_{el}"] = float(abs(a["mean_ion_energy"][el] / b["mean_ion_energy"][el] - 1))
    for s in (0, 1):
        for el in (0, 1):
            if b["flux"][s][el] > 0:
                d[f"flux_{s}{el}"] = float(abs(a["flux"][s][el] / b["flux"][s][el] - 1))
    if self_bias:
        d["self_bias"] = float(abs(a["phi0"] / b["phi0"] - 1))
    return d


def subset(pool, idx):
    """The pool restricted to (or resampled at) the given seed indices."""
    out = {}
    for k, v in pool.items():
        if isinstance(v, np.ndarray) and v.ndim >= 1 and len(v) == len(pool["seeds"]):
            out[k] = v[idx]
    return out


def noise(pool, self_bias=False, n_boot=200, seed=0):
    """Each metric's noise level: the root-mean-square distance of the pooled
    statistics of seeds resampled with replacement from the pooled statistics of
    the pool itself (the standard error of the pool's value, estimated from the
    seed-to-seed scatter; for the KS distance the typical distance)."""
    rng = np.random.default_rng(seed)
    n = len(pool["seeds"])
    ref = pooled(pool)
    acc = {}
    for _ in range(n_boot):
        d = distances(pooled(subset(pool, rng.integers(0, n, n))), ref, self_bias)
        for k, v in d.items():
            acc.setdefault(k, []).append(v * v)
    return {k: float(np.sqrt(np.mean(v))) for k, v in acc.items()}
