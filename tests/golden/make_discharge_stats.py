"""Write the oracle's long-run discharge statistics used by the statistical parity
tests.  Calls only oracle/ and workloads/ (CPU, FP64).

    python tests/golden/make_discharge_stats.py [name ...] [--workers N]

A workload runs as two pools of seeds, A and B.  For each seed: `warm` steps
from the initial load, then the averages are reset and `window` steps are
averaged (Sec. IV: time averages over an adequate period).  Each pool is stored
as tests/golden/discharge_<name>_pool<A|B>.npz with the per-seed time-averaged
densities, potential, ion impact energy histograms, wall fluxes and counters,
the case parameters (JSON) and the SHA-256 of the oracle's discharge sources, so
that a test can refuse statistics written by another oracle.  The GPU runs the
seeds of pool A; pool B measures the oracle's own pool-to-pool spread.

The oracle takes its plain geometric waits between collision checks (no cut).
The workload `wait_cut` instead runs the same seeds with and without the cut
of the GPU's examination schedule (waits longer than WAIT_CAP steps redrawn at
the cut), at the ions' collision probability of the working-size discharge,
long enough for the cut to act many times.
"""
import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor, as_completed

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import pic as P  # noqa: E402

ORACLE_FILES = ("constants.py", "philox.py", "pic.py", "xsec.py")


def oracle_sha256():
    """SHA-256 over the oracle's discharge sources (what a stored value depends on)."""
    h = hashlib.sha256()
    for f in ORACLE_FILES:
        with open(os.path.join(ROOT, "oracle", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _eae(seed):
    # the small case with the paper's drive: two harmonics (delta phi = 0) through a
    # blocking capacitor of 5e-9 F/m^2 (DC self-bias)
    return dict(W.discharge_small(seed=seed), v2_volt=100.0, phase_rad=0.0, phase2_rad=0.0, cb_f_m2=5e-9)


def _corner(p_pa, v0, case_id):
    # corners of the batched sweep's ranges: 40 mm, 256 cells, 5e4 + 5e4, dt = T_rf / 1000
    return lambda seed: W.discharge(0.04, 256, v0, 1000, p_pa, 50_000, 4e15, seed=seed, case_id=case_id)


def _wait_cut_case(seed):
    # the ions' collision probability of the working-size discharge (0.5 Pa, 300 V,
    # dt = T_rf / 2000: P_i = 1.35e-4, so 1.2 % of their waits exceed WAIT_CAP)
    # on 128 cells with 1e4 + 1e4 particles
    return W.discharge(0.04, 128, 300.0, 2000, 0.5, 10_000, 4e15, seed=seed, case_id=6)


K_SMALL = 128
RUNS = {
    # 64 cells, 5k + 5k: 40 RF cycles to settle, averages over the next 20 (8000 steps);
    # 128 seeds per pool keep the pooled statistics' standard errors below 1 %
    "small": dict(make=lambda seed: W.discharge_small(seed=seed),
                  pools=(range(1, 1 + K_SMALL), range(1001, 1001 + K_SMALL)), warm=16000, window=8000),
    "small_eae": dict(make=_eae, pools=(range(101, 101 + K_SMALL), range(1101, 1101 + K_SMALL)),
                      warm=16000, window=8000),
    # the working-size discharge, 1M + 1M on 1024 cells: 20 RF cycles, averages over the last 10
    "working": dict(make=lambda seed: W.discharge_working(seed=seed), pools=((1607,), (1608,)),
                    warm=20000, window=20000),
    # the batched sweep's extremes: 10 Pa at 500 V (nu_max dt = 0.36 for electrons) and
    # 0.5 Pa at 50 V; 20 RF cycles to settle, averages over the next 30; the electrons'
    # wall fluxes are the noisiest metric (36 and 24 seeds bring them below 1 %)
    "corner_hi": dict(make=_corner(10.0, 500.0, 7), pools=(range(1, 37), range(1001, 1037)),
                      warm=20000, window=30000),
    "corner_lo": dict(make=_corner(0.5, 50.0, 8), pools=(range(1, 25), range(1001, 1025)),
                      warm=20000, window=30000),
    # the cut against the plain waits: the same seeds, pool A cut, pool B plain
    "wait_cut": dict(make=_wait_cut_case, pools=(range(1, 7), range(1, 7)), warm=40000, window=60000,
                     wait_caps=(P.WAIT_CAP, None)),
}

KEYS = ("ne", "ni", "phi", "iedf", "flux", "absorbed", "mean_ion_energy", "collisions", "candidates",
        "n_e", "n_i", "step", "avg_steps", "particle_steps", "redraws")


def run_one(args):
    name, pool, seed = args
    spec = RUNS[name]
    p = spec["make"](seed)
    cap = spec.get("wait_caps", (None, None))[pool]
    t0 = time.time()
    d = P.Discharge(p, wait_cap=cap)
    d.run(spec["warm"])
    d.reset_diagnostics()
    d.run(spec["window"])
    o = d.sample_diagnostics()
    return name, pool, seed, {k: np.asarray(o[k]) for k in KEYS}, json.dumps(p, sort_keys=True), time.time() - t0


def _stored(name, pool, sha):
    """Seeds already stored for a pool by this oracle: {seed: (results, params JSON)}."""
    path = os.path.join(HERE, f"discharge_{name}_pool{'AB'[pool]}.npz")
    if not os.path.exists(path):
        return {}
    z = np.load(path)
    spec = RUNS[name]
    if str(z["oracle_sha256"]) != sha or int(z["warm"]) != spec["warm"] or int(z["window"]) != spec["window"]:
        return {}
    return {int(sd): ({k: z[k][i] for k in KEYS}, str(z["params"][i])) for i, sd in enumerate(z["seeds"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*")
    ap.add_argument("--workers", type=int, default=6)
    ap.add_argument("--extend", action="store_true", help="keep the seeds a pool already holds, run the rest")
    a = ap.parse_args()
    names = a.names or list(RUNS)
    sha = oracle_sha256()
    kept = {(n, k): (_stored(n, k, sha) if a.extend else {}) for n in names for k in range(2)}
    jobs = [(n, k, s) for n in names for k, pool in enumerate(RUNS[n]["pools"]) for s in pool
            if s not in kept[(n, k)]]
    # the longest runs first
    jobs.sort(key=lambda j: -RUNS[j[0]]["make"](j[2])["np_e"] * (RUNS[j[0]]["warm"] + RUNS[j[0]]["window"]))
    got = {key: [(sd, o, pj) for sd, (o, pj) in kept[key].items()
                 if sd in RUNS[key[0]]["pools"][key[1]]] for key in kept}
    with ProcessPoolExecutor(max_workers=max(1, min(a.workers, len(jobs)))) as ex:
        for fut in as_completed([ex.submit(run_one, j) for j in jobs]):
            name, pool, seed, o, pj, dt = fut.result()
            print(f"{name} pool {'AB'[pool]} seed {seed}: {dt:.0f} s", flush=True)
            got.setdefault((name, pool), []).append((seed, o, pj))
            spec = RUNS[name]
            if len(got[(name, pool)]) == len(spec["pools"][pool]):
                runs = sorted(got[(name, pool)], key=lambda r: r[0])
                out = {k: np.stack([r[1][k] for r in runs]) for k in KEYS}
                path = os.path.join(HERE, f"discharge_{name}_pool{'AB'[pool]}.npz")
                cap = spec.get("wait_caps", (None, None))[pool]
                np.savez_compressed(path, seeds=np.array([r[0] for r in runs]),
                                    params=np.array([r[2] for r in runs]), warm=spec["warm"],
                                    window=spec["window"], wait_cap=-1 if cap is None else cap,
                                    oracle_sha256=sha, **out)
                print("wrote", os.path.basename(path), flush=True)


if __name__ == "__main__":
    main()
