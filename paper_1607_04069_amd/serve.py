"""Served stream: continuous batching of discharge cases and test-particle jobs.

Requests arrive as a seeded Poisson process.  A discharge request is admitted
when a slot of the slotted batch is free and its device footprint
(pm_case_footprint) fits in what is left of the HBM budget; it is then loaded
on the device and joins the running batch at the next chunk boundary
(pm_batch_set_slot rewrites the batch's device tables; the RF-cycle graph,
captured once for the slot table, is kept).  Every resident case advances in
the same launches, one RF cycle per chunk.  A case is done after its RF-cycle
budget; its time averages cover the last fifth of its cycles (the averaging
window is reset at that cycle boundary).  It is then read out and its slot
emptied, which frees the slot and its memory for the queue.

Test-particle jobs are admitted against the same HBM budget (their tally arena,
pm_tp_footprint) and run on a few worker streams beside the discharge chunks,
so several jobs and the batch share the device at once.

A request whose footprint the whole budget cannot hold (or whose parameters the
library rejects) is refused at arrival with an error; a case that fails while
served (slots exhausted, a NaN) leaves the batch with its error.  Neither stops
the stream.

Each case's result depends only on its own parameters and the number of steps
it ran, never on its neighbours in the batch, so a case served in the mix
returns exactly what it returns alone (``run_alone``).
"""
import collections
import ctypes
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


def case_footprint(pm, params):
    cp = pm.case_params(params)
    return int(pm.pm_case_footprint(ctypes.byref(cp)))


def tpm_footprint(pm, job):
    tp = pm.tp_params(job["tp"])
    return int(pm.pm_tp_footprint(ctypes.byref(tp)))


class _Budget:
    """Device bytes in use by admitted requests, shared by the discharge loop and
    the test-particle workers."""

    def __init__(self, limit):
        self.limit = int(limit)
        self.used = 0
        self.lock = threading.Lock()

    def take(self, nbytes):
        """Reserve nbytes if they fit in what is left."""
        with self.lock:
            if self.used + nbytes <= self.limit:
                self.used += nbytes
                return True
            return False

    def never_fits(self, nbytes):
        """A request that the whole budget cannot hold (or whose parameters the
        library rejects: footprint 0) is refused rather than queued forever."""
        return nbytes == 0 or nbytes > self.limit

    def give(self, nbytes):
        with self.lock:
            self.used -= nbytes


class Server:
    """Serve a list of requests in real time on the current device.

    cycles_budget: RF cycles per discharge; max_slots: discharge slots of the
    batch; hbm_budget_bytes: device bytes all admitted requests may hold;
    tpm_workers: test-particle jobs that may run at once (one stream each);
    shape: launch shape of the batch (None: the library's default)."""

    def __init__(self, pm, cycles_budget=200, max_slots=64, hbm_budget_bytes=64 << 30, shape=None,
                 tpm_workers=4, log=None):
        self.pm = pm
        self.budget = int(cycles_budget)
        self.max_slots = int(max_slots)
        self.hbm_budget = int(hbm_budget_bytes)
        self.shape = shape
        self.tpm_workers = int(tpm_workers)
        self.log = log or (lambda s: None)

    def _footprint(self, params):
        return case_footprint(self.pm, params)

    def run(self, requests):
        import torch
        pm = self.pm
        reqs = sorted(requests, key=lambda r: r.arrival)
        dis = [r for r in reqs if r.kind == "discharge"]
        tpm_list = [r for r in reqs if r.kind == "tpm"]
        budget = _Budget(self.hbm_budget)
        dev = torch.cuda.current_device()
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        # ---- test-particle jobs: a shared queue in arrival order, several workers
        tpm_queue = collections.deque(tpm_list)
        tpm_lock = threading.Lock()
        tpm_events = [0]

        def tpm_worker():
            torch.cuda.set_device(dev)
            stream = torch.cuda.Stream()
            while True:
                with tpm_lock:
                    if not tpm_queue:
                        return
                    r = tpm_queue[0]
                    wait = r.arrival - now()
                    fp = tpm_footprint(pm, r.params)
                    if wait <= 0 and budget.never_fits(fp):
                        tpm_queue.popleft()
                        r.admitted = r.done = now()
                        r.result = {"error": f"footprint {fp} B does not fit the budget", "events": 0}
                        continue
                    if wait > 0 or not budget.take(fp):
                        r = None
                    else:
                        tpm_queue.popleft()
                if r is None:
                    time.sleep(min(max(wait, 0.0), 0.01) if wait > 0 else 0.002)
                    continue
                r.admitted = now()
                try:
                    res = pm.run_test_particles(r.params["src"], r.params["tp"], stream=stream)
                except pm.PicMccError as e:          # rejected or failed: reported, not retried
                    res = {"error": str(e), "events": 0}
                finally:
                    budget.give(fp)
                r.done = now()
                r.result = res
                with tpm_lock:
                    tpm_events[0] += res["events"]

        workers = [threading.Thread(target=tpm_worker, daemon=True) for _ in range(self.tpm_workers)]
        for w in workers:
            w.start()

        # ---- discharge cases: a slotted batch, one RF cycle per chunk
        batch = None
        particle_steps = 0
        busy = 0.0
        chunks = 0
        if dis:
            nt = dis[0].params["steps_per_cycle"]
            assert all(r.params["steps_per_cycle"] == nt for r in dis), "one RF-cycle length per stream"
            fp64 = bool(dis[0].params.get("fp64", 0))
            max_cells = max(int(r.params["n_cells"]) for r in dis)
            batch = pm.SlotBatch(self.max_slots, nt, max_cells=max_cells, fp64=fp64)
            if self.shape:
                batch.set_launch_shape(**self.shape)
        pending = collections.deque(dis)
        free = list(range(self.max_slots))[::-1]
        resident = {}                 # slot -> [request, case, cycles done, footprint]
        n_done = 0
        while n_done < len(dis):
            t = now()
            changed = False
            # admission by slot and footprint, in arrival order
            while pending and pending[0].arrival <= t and free:
                fp = self._footprint(pending[0].params)
                if budget.never_fits(fp):
                    r = pending.popleft()
                    r.admitted = r.done = t
                    r.result = {"error": f"footprint {fp} B does not fit the budget"}
                    n_done += 1
                    continue
                if not budget.take(fp):
                    break
                r = pending.popleft()
                r.admitted = t
                try:
                    c = pm.Case(r.params)
                except pm.PicMccError as err:
                    budget.give(fp)
                    r.done = t
                    r.result = {"error": str(err)}
                    n_done += 1
                    continue
                slot = free.pop()
                batch.set_slot(slot, c)
                resident[slot] = [r, c, 0, fp]
                changed = True
            if changed:
                self.log(f"{now():8.2f}s batch of {len(resident)} cases")
            if not resident:
                if pending:
                    time.sleep(max(0.0, min(pending[0].arrival - t, 0.05)))
                continue
            t_chunk = time.perf_counter()
            batch.step_rf_cycles(1)
            torch.cuda.current_stream().synchronize()
            busy += time.perf_counter() - t_chunk
            chunks += 1
            t_end = now()
            for slot in list(resident):
                e = resident[slot]
                e[2] += 1
                r, c = e[0], e[1]
                try:
                    if e[2] == _window_start(self.budget):
                        # the step counters restart with the averaging window
                        particle_steps += c.sample_diagnostics(reset=True)["particle_steps"]
                    if e[2] == self.budget:
                        r.result = _result(c)
                        particle_steps += r.result["particle_steps"]
                except pm.PicMccError as err:
                    # a case that failed (slots exhausted, a NaN) leaves with its error;
                    # the others go on
                    r.result = {"error": str(err)}
                    e[2] = self.budget
                if e[2] == self.budget:
                    r.done = t_end
                    batch.set_slot(slot, None)
                    c.close()
                    budget.give(e[3])
                    del resident[slot]
                    free.append(slot)
                    n_done += 1
                    if n_done % 25 == 0 or n_done == len(dis):
                        self.log(f"{t_end:8.2f}s {n_done} of {len(dis)} discharges done")
        for w in workers:
            w.join()
        torch.cuda.synchronize()
        wall = now()
        if batch is not None:
            batch.close()
        lat = {k: np.array([r.latency for r in reqs if r.kind == k]) for k in ("discharge", "tpm")}
        summary = {"wall_s": wall, "requests": len(reqs), "discharge_particle_steps": particle_steps,
                   "failed": sum(1 for r in reqs if isinstance(r.result, dict) and "error" in r.result),
                   "tpm_events": tpm_events[0],
                   "particle_steps_per_s": (particle_steps + tpm_events[0]) / wall,
                   "discharge_particle_steps_per_s": particle_steps / wall,
                   "batch_busy_s": busy, "chunks": chunks,
                   "discharge_particle_steps_per_busy_s": particle_steps / busy if busy > 0 else 0.0}
        if dis:
            span = max(dis[-1].arrival - dis[0].arrival, 1e-9)
            offered = sum((r.params["np_e"] + r.params["np_i"]) * self.budget * r.params["steps_per_cycle"]
                          for r in dis)
            summary["offered_discharge_particle_steps_per_s"] = offered / span
        for k, v in lat.items():
            if len(v):
                summary[f"{k}_latency_p50_s"] = float(np.percentile(v, 50))
                summary[f"{k}_latency_p99_s"] = float(np.percentile(v, 99))
                summary[f"{k}_count"] = int(len(v))
        allv = np.concatenate([v for v in lat.values() if len(v)])
        summary["latency_p50_s"] = float(np.percentile(allv, 50))
        summary["latency_p99_s"] = float(np.percentile(allv, 99))
        return summary
