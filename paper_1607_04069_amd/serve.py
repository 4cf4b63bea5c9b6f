"""Served stream: continuous batching of discharge cases and test-particle jobs.

Requests arrive as a seeded Poisson process.  A discharge request is admitted
when a slot is free and its device footprint (pm_case_footprint) fits in what
is left of the HBM budget; it is then loaded on the device and joins the
running batch at the next chunk boundary.  Every resident case advances in the
same launches, one RF cycle per chunk (a replay of the batch's RF-cycle graph,
recaptured when the set of resident cases changes).  A case is done after its
RF-cycle budget; its time averages cover the last fifth of its cycles (the
averaging window is reset at that cycle boundary).  It is then read out and
retired, which frees its slot and memory for the queue.  Test-particle jobs run
on a second stream from a worker thread, overlapping the discharge chunks.

Each case's result depends only on its own parameters and the number of steps
it ran, never on its neighbours in the batch, so a case served in the mix
returns exactly what it returns alone (``run_alone``).
"""
import collections
import dataclasses
import math
import threading
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    kind: str                 # "discharge" or "tpm"
    arrival: float            # seconds after the start of the stream
    params: dict              # discharge parameters, or {"src": ..., "tp": ...}
    admitted: float = math.nan
    done: float = math.nan
    result: dict = None

    @property
    def latency(self):
        return self.done - self.arrival


def poisson_stream(n, rate_hz, make_discharge, make_tpm, tpm_fraction=0.5, seed=1607):
    """n requests with exponential inter-arrival times (mean 1/rate_hz); each is
    a test-particle job with probability tpm_fraction, else a discharge case."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_hz)
        if rng.uniform() < tpm_fraction:
            out.append(Request(i, "tpm", t, make_tpm(i, rng)))
        else:
            out.append(Request(i, "discharge", t, make_discharge(i, rng)))
    return out


def _window_start(budget):
    return budget - max(1, budget // 5)


def _result(case):
    d = case.sample_diagnostics()
    return {k: d[k] for k in ("ne", "ni", "phi", "iedf", "iadf", "flux", "mean_ion_energy", "step",
                              "avg_steps", "particle_steps", "collisions", "absorbed")}


def run_alone(pm, params, budget):
    """One discharge case alone, with the served schedule: budget RF cycles, the
    averaging window reset after the first 4/5 of them."""
    c = pm.Case(params)
    w = _window_start(budget)
    c.step_rf_cycles(w)
    c.sample_diagnostics(reset=True)
    c.step_rf_cycles(budget - w)
    r = _result(c)
    c.close()
    return r


def run_tpm(pm, job):
    return pm.run_test_particles(job["src"], job["tp"])


class Server:
    """Serve a list of requests in (scaled) real time on the current device."""

    def __init__(self, pm, cycles_budget=200, max_slots=64, hbm_budget_bytes=64 << 30, shape=None,
                 log=None):
        self.pm = pm
        self.budget = int(cycles_budget)
        self.max_slots = int(max_slots)
        self.hbm_budget = int(hbm_budget_bytes)
        self.shape = shape            # launch shape for every batch (None: the library default)
        self.log = log or (lambda s: None)

    def _footprint(self, params):
        import ctypes as C
        cp = self.pm.case_params(params)
        return int(self.pm.pm_case_footprint(C.byref(cp)))

    def run(self, requests):
        import torch
        pm = self.pm
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending = collections.deque(r for r in reqs if r.kind == "discharge")
        resident = []                 # [request, case, cycles_done, footprint]
        used = 0
        batch = None
        dirty = True
        particle_steps = 0
        tpm_events = 0
        tpm_lock = threading.Lock()
        tpm_stream = torch.cuda.Stream()
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        tpm_list = [r for r in reqs if r.kind == "tpm"]
        dev = torch.cuda.current_device()

        def tpm_worker():
            # jobs start at their arrival (or when the previous job ends)
            nonlocal tpm_events
            torch.cuda.set_device(dev)
            with torch.cuda.stream(tpm_stream):
                for r in tpm_list:
                    time.sleep(max(0.0, r.arrival - now()))
                    r.admitted = now()
                    res = pm.run_test_particles(r.params["src"], r.params["tp"], stream=tpm_stream)
                    r.done = now()
                    r.result = res
                    with tpm_lock:
                        tpm_events += res["events"]

        worker = threading.Thread(target=tpm_worker, daemon=True)
        worker.start()
        n_done = 0
        n_dis = len(reqs) - len(tpm_list)
        while n_done < n_dis:
            t = now()
            # admission by slot and footprint, in arrival order
            while pending and pending[0].arrival <= t and len(resident) < self.max_slots:
                fp = self._footprint(pending[0].params)
                if used + fp > self.hbm_budget and resident:
                    break
                r = pending.popleft()
                r.admitted = t
                c = pm.Case(r.params)
                resident.append([r, c, 0, fp])
                used += fp
                dirty = True
            if not resident:
                time.sleep(max(0.0, min(pending[0].arrival - t, 0.05)))
                continue
            if dirty:
                if batch is not None:
                    batch.close()
                batch = pm.Batch([e[1] for e in resident])
                if self.shape:
                    batch.set_launch_shape(**self.shape)
                dirty = False
                self.log(f"{now():8.2f}s batch of {len(resident)} cases")
            batch.step_rf_cycles(1)
            torch.cuda.current_stream().synchronize()
            t_end = now()
            retire = []
            for e in resident:
                e[2] += 1
                if e[2] == _window_start(self.budget):
                    # the step counters restart with the averaging window
                    particle_steps += e[1].sample_diagnostics(reset=True)["particle_steps"]
                if e[2] == self.budget:
                    retire.append(e)
            for e in retire:
                r, c = e[0], e[1]
                r.result = _result(c)
                particle_steps += r.result["particle_steps"]
                r.done = t_end
                resident.remove(e)
                used -= e[3]
                n_done += 1
                dirty = True
            if retire:
                batch.close()
                batch = None
                for e in retire:
                    e[1].close()
        worker.join()
        torch.cuda.synchronize()
        wall = now()
        if batch is not None:
            batch.close()
        lat = {k: np.array([r.latency for r in reqs if r.kind == k]) for k in ("discharge", "tpm")}
        summary = {"wall_s": wall, "requests": len(reqs), "discharge_particle_steps": particle_steps,
                   "tpm_events": tpm_events,
                   "particle_steps_per_s": (particle_steps + tpm_events) / wall,
                   "discharge_particle_steps_per_s": particle_steps / wall}
        for k, v in lat.items():
            if len(v):
                summary[f"{k}_latency_p50_s"] = float(np.percentile(v, 50))
                summary[f"{k}_latency_p99_s"] = float(np.percentile(v, 99))
                summary[f"{k}_count"] = int(len(v))
        allv = np.concatenate([v for v in lat.values() if len(v)])
        summary["latency_p50_s"] = float(np.percentile(allv, 50))
        summary["latency_p99_s"] = float(np.percentile(allv, 99))
        return summary
