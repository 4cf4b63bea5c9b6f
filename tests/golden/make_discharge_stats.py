"""Write the oracle's long-run discharge statistics used by the GPU statistical
parity test.  Calls only oracle/ and workloads/ (CPU, FP64).

    python tests/golden/make_discharge_stats.py [name ...]

For each workload and seed: run `warm` steps from the initial load, reset the
averages, run `window` steps, and store the time-averaged densities, potential,
ion energy/angle histograms, wall fluxes and counters in
tests/golden/discharge_<name>_seed<seed>.npz.  Three seeds per workload give the
oracle's own seed-to-seed spread.
"""
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import pic as P  # noqa: E402

RUNS = {
    # 64 cells, 5k + 5k: 40 RF cycles to settle, averages over the next 10 (4000 steps)
    "small": dict(make=lambda seed: W.discharge_small(seed=seed), seeds=(1, 2, 3), warm=16000, window=4000),
    # the small case with the paper's drive: two harmonics (delta phi = 0) through a
    # blocking capacitor of 5e-9 F/m^2 (DC self-bias)
    "small_eae": dict(make=lambda seed: dict(W.discharge_small(seed=seed), v2_volt=100.0, phase_rad=0.0,
                                             phase2_rad=0.0, cb_f_m2=5e-9),
                      seeds=(11, 12, 13), warm=16000, window=4000),
    # 1024 cells, 100k + 100k at the working-size conditions: averages over cycles 3-6
    "working100k": dict(make=lambda seed: W.discharge_working(seed=seed, np_each=100_000),
                        seeds=(1607, 1608, 1609), warm=6000, window=6000),
}


def run_one(args):
    name, seed = args
    spec = RUNS[name]
    p = spec["make"](seed)
    t0 = time.time()
    d = P.Discharge(p)
    d.run(spec["warm"])
    d.reset_diagnostics()
    d.run(spec["window"])
    o = d.sample_diagnostics()
    path = os.path.join(HERE, f"discharge_{name}_seed{seed}.npz")
    np.savez(path, ne=o["ne"], ni=o["ni"], phi=o["phi"], iedf=o["iedf"], iadf=o["iadf"],
             flux=o["flux"], absorbed=o["absorbed"], mean_ion_energy=o["mean_ion_energy"],
             collisions=o["collisions"], n_e=o["n_e"], n_i=o["n_i"], step=o["step"],
             avg_steps=o["avg_steps"], warm=spec["warm"], window=spec["window"], seed=seed)
    return f"{name} seed {seed}: {time.time() - t0:.0f} s -> {os.path.basename(path)}"


if __name__ == "__main__":
    names = sys.argv[1:] or list(RUNS)
    jobs = [(n, s) for n in names for s in RUNS[n]["seeds"]]
    with ProcessPoolExecutor(max_workers=min(6, len(jobs))) as ex:
        for msg in ex.map(run_one, jobs):
            print(msg, flush=True)
