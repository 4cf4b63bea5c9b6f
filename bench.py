"""Throughput of the PIC/MCC hot path on one MI355X: batched vs plain.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--retune]

Headline workload (synthetic, seeded): the batched parameter sweep -- 64
independent argon discharges, 40 mm gap, pressure log-uniform on 0.5-10 Pa,
voltage uniform on 50-500 V, 128/256/512/1024 cells, 20k-500k particles per
species, 13.56 MHz, dt = T_rf/1000, FP32 particles, int64 charge, FP64 Poisson.
One bench step is one RF cycle (1000 time steps) of all 64 cases, replayed from
the batch's HIP graph; inputs are resident in HBM before the timed region.  Each
case runs 200 RF cycles (--case-cycles): by default 2 warm-up cycles and the
other 198 timed, so the rate covers the whole run as the discharges settle (their
live particles fall to about half); with fewer timed steps, untimed cycles
before the warm-up make the timed ones the last of the 200.
The push and collision kernels are first timed alone (single steps, HIP events)
from the seeded initial load, for the roofline.

Beside it, measured after the timed region: the same 64 cases stepped one case
at a time (each from its own RF-cycle graph), the plain single working-size
discharge (1024 cells, 1M e + 1M Ar+, 300 V, 0.5 Pa, dt = T_rf/2000), and the
sputtered-atom flight (1e7 Al atoms at 0.5 and 5 Pa).  Prints one JSON line.
"""
import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (batched vs plain) at oracle-matched stats; p50/p99 case latency"
HBM_PEAK_GBS = 8000.0
PROBE = 100


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=198, help="timed RF cycles of the batch")
    ap.add_argument("--warmup", type=int, default=2, help="untimed RF cycles of the batch")
    ap.add_argument("--kernel-probe", type=int, default=PROBE, help="single batch steps timed one by one")
    ap.add_argument("--case-cycles", type=int, default=200,
                    help="RF cycles of a sweep case: the timed cycles are the last of them (the untimed "
                         "cycles before the warm-up settle the discharges)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-side", action="store_true", help="skip the plain and test-particle legs")
    ap.add_argument("--retune", action="store_true", help="time the launch shapes instead of the cached choice")
    ap.add_argument("--serve-requests", type=int, default=48, help="requests of the served-stream leg (0: skip)")
    ap.add_argument("--serve-cycles", type=int, default=200, help="RF-cycle budget of a served discharge")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the served stream (after the batched sweep that sets its capacity)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB (counter calibration)")
    ap.add_argument("--probe", choices=("push", "flight"), default=None,
                    help="for counter passes: only the push/collision probe (single batch steps) or only "
                         "the atom flights, with plain launches and no graph; prints one JSON line")
    ap.add_argument("--sweep-cases", type=int, default=64,
                    help="cases of the push probe's sweep (128: twice the working set, the 64-case "
                         "shape with its workgroups doubled)")
    return ap.parse_args()


def kernel_probe(batch, cases, n):
    """Average durations of the push and collision kernels over n single steps,
    each launch bracketed by HIP events on the stream it runs on (one lane, so
    every launch has the device to itself), and the work per step."""
    shape = batch.launch_shape()
    batch.set_launch_shape(lanes=1)
    d0 = [c.sample_diagnostics() for c in cases]
    push_ms, mcc_ms = batch.time_kernels(n)
    d1 = [c.sample_diagnostics() for c in cases]
    batch.set_launch_shape(**shape)
    ps = sum(y["particle_steps"] - x["particle_steps"] for x, y in zip(d0, d1))
    cand = sum(int(sum(y["candidates"]) - sum(x["candidates"])) for x, y in zip(d0, d1))
    return push_ms, mcc_ms, ps / n, cand / n


def flight_probe(pm, W, torch):
    """The atom flights alone (1e7 atoms at 0.5 and 5 Pa, each after a warm-up
    of 1e5): no discharge, no graph."""
    out = {"probe": "flight"}
    for p_pa in (0.5, 5.0):
        src, tp = W.sputter_transport(p_pa=p_pa)
        job = pm.TestParticleJob(tp)
        r0 = job.run(dict(src, n_atoms=100_000))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = job.run(src)
        torch.cuda.synchronize()
        out[f"tpm_{p_pa:g}pa"] = {"warmup_atoms": 100_000, "warmup_events": r0["events"],
                                  "atoms": src["n_atoms"], "events": r["events"],
                                  "seconds": time.perf_counter() - t0}
    return out


def copy_probe(mb, torch):
    """A device copy of mb MiB: the counters' reading for bytes of known size."""
    n = mb * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n}), flush=True)


def measured_traffic(probe_launches):
    """HBM bytes per probe launch of the batched step kernel from the committed
    counter passes (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's
    reading for a copy of known size), or None when the kernel source changed."""
    path = os.path.join(ROOT, "profiles", "k_step_batch_traffic.json")
    src = os.path.join(ROOT, "paper_1607_04069_amd", "csrc", "pic_kernels.hip")
    try:
        with open(path) as f:
            t = json.load(f)
        with open(src, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if t.get("source_sha256") != digest or t.get("probe_launches") != probe_launches:
        return None
    return t["bytes_per_launch"]


def _oracle_case(args):
    """One oracle case for a number of steps (a worker process)."""
    p, steps = args
    import oracle.pic as P
    d = P.Discharge(p)
    n = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        n += len(d.sp[0]) + len(d.sp[1])
        d.step()
    return n, time.perf_counter() - t0


def cpu_baseline(params, steps):
    """The oracle on a sample of the sweep: every fourth case, run as independent
    processes on the host's cores (the cases are independent)."""
    sample = params[::4]
    cores = max(1, min(len(sample), len(os.sched_getaffinity(0)), 16))
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_case, [(p, steps) for p in sample], chunksize=1)
    wall = time.perf_counter() - t0
    n = sum(r[0] for r in res)
    busy = sum(r[1] for r in res)
    return n / wall, cores, len(sample), n, wall, n / busy


def cpu_single_core(W):
    """The oracle on one core for the other workloads: the small and the working
    discharge (a few hundred and ten steps from their load) and the atom flight at
    0.5 Pa (2e4 atoms) and 5 Pa (2e3 atoms)."""
    import oracle.pic as P
    import oracle.tpm as T
    out = {}
    for name, p, steps in (("discharge_small", W.discharge_small(), 400), ("discharge_working", W.discharge_working(), 10)):
        d = P.Discharge(p)
        n = 0
        t0 = time.perf_counter()
        for _ in range(steps):
            n += len(d.sp[0]) + len(d.sp[1])
            d.step()
        out[f"{name}_particle_steps_per_s"] = n / (time.perf_counter() - t0)
    for p_pa, n_atoms in ((0.5, 20_000), (5.0, 2_000)):
        src, tp = W.sputter_transport(p_pa=p_pa, n_atoms=n_atoms)
        t0 = time.perf_counter()
        r = T.run(src, tp, n_atoms=n_atoms)
        dt = time.perf_counter() - t0
        out[f"tpm_{p_pa:g}pa_atoms_per_s"] = n_atoms / dt
        out[f"tpm_{p_pa:g}pa_events_per_s"] = r["events"] / dt
    return out


def serving_leg(pm, W, args, capacity):
    """The served stream: Poisson arrivals at 4/s, half discharges drawn as in the
    sweep (RF-cycle budget args.serve_cycles, averages over its last fifth), half
    test-particle jobs; the load factor is the discharges' offered particle-steps/s
    (initial particles x budget) over the batched sweep's measured rate, and
    served_over_capacity the live particle-steps advanced per second over it."""
    from paper_1607_04069_amd import serve
    reqs = serve.poisson_stream(args.serve_requests, 4.0, W.served_discharge, W.served_tpm)
    srv = serve.Server(pm, cycles_budget=args.serve_cycles, max_slots=64, tpm_workers=4,
                       shape=dict(unroll=8, waves=0, work_groups=0, deposit_mode=1, sort_interval=50, lanes=2),
                       log=lambda m: print(m, file=sys.stderr, flush=True))
    summ = srv.run(reqs)
    offered = summ.get("offered_discharge_particle_steps_per_s", 0.0)
    served = summ.get("discharge_particle_steps_per_s", 0.0)
    return {"requests": args.serve_requests, "arrivals_per_s": 4.0, "rf_cycles_per_case": args.serve_cycles,
            # offered: the cases' initial particles x budget steps per second of arrivals
            "load_factor": offered / capacity if capacity > 0 else None,
            # served: the live particle-steps actually advanced per second of the stream
            "served_over_capacity": served / capacity if capacity > 0 else None,
            "capacity_particle_steps_per_s": capacity, **summ}


def timed_cycles(obj, cases, k, torch):
    torch.cuda.synchronize()
    p0 = sum(c.sample_diagnostics()["particle_steps"] for c in cases)
    t0 = time.perf_counter()
    obj.step_rf_cycles(k)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    p1 = sum(c.sample_diagnostics()["particle_steps"] for c in cases)
    return p1 - p0, dt


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; independent cases and atom ranges "
                                   "would shard across GPUs, which is described but not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_1607_04069_amd as pm
    from paper_1607_04069_amd import autotune
    import workloads as W

    torch.cuda.set_device(0)
    if args.probe == "flight":
        print(json.dumps(flight_probe(pm, W, torch)), flush=True)
        if args.copy_probe_mb:
            copy_probe(args.copy_probe_mb, torch)
        return
    n_sweep = args.sweep_cases if args.probe == "push" else 64
    params = W.sweep_cases(n_sweep)
    cases = [pm.Case(p) for p in params]
    batch = pm.Batch(cases)
    if n_sweep == 64:
        shape, _, source = autotune.tune(batch, params, use_cache=not args.retune,
                                         log=(lambda m: print(m, file=sys.stderr, flush=True)) if args.retune
                                         else None)
    else:
        # the shape cached for the 64-case sweep (its first 64 cases are these'),
        # with as many particles per workgroup
        shape, _, source = autotune.tune(batch, params[:64], use_cache=True)
        if source != "cache":
            raise SystemExit("no cached launch shape for the 64-case sweep")
        batch.set_launch_shape(work_groups=shape["work_groups"] * n_sweep // 64)
        shape = batch.launch_shape()
    for c in cases:
        c.sample_diagnostics(reset=True)

    # The dominant kernel, the push, timed first from the seeded initial load (the
    # same launches in every run, so the counter passes of this command see them
    # too): per particle-step it must move x and v_x in and out in FP32 (16 B).
    # The collision kernel must move, per null-collision candidate, its list entry
    # in (slot, x and v_x: 12 B), its record in (v_y, v_z, id: 16 B) and its next
    # examination code out (2 B): 30 B.
    progress(f"kernel probe: {args.kernel_probe} single steps of {len(cases)} cases")
    k_ms, mcc_ms, ps_per_launch, cand_per_launch = kernel_probe(batch, cases, args.kernel_probe)
    if args.probe == "push":
        alg = 16.0 * ps_per_launch
        print(json.dumps({"probe": "push", "cases": n_sweep, "launch_shape": shape, "shape_source": source,
                          "probe_launches": args.kernel_probe, "push_ms": k_ms, "mcc_ms": mcc_ms,
                          "particle_steps_per_launch": ps_per_launch, "candidates_per_launch": cand_per_launch,
                          "push_alg_bytes_per_launch": alg, "push_alg_gbs": alg / (k_ms * 1e-3) / 1e9,
                          "push_frac": alg / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}), flush=True)
        batch.close()
        for c in cases:
            c.close()
        if args.copy_probe_mb:
            copy_probe(args.copy_probe_mb, torch)
        return
    alg_bytes = 16.0 * ps_per_launch
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.kernel_probe)

    settle = max(0, args.case_cycles - args.warmup - args.steps)
    progress(f"push {k_ms * 1e3:.1f} us, collisions {mcc_ms * 1e3:.1f} us; settling {settle} RF cycles")
    t_settle = time.perf_counter()
    batch.step_rf_cycles(settle)
    torch.cuda.synchronize()
    t_settle = time.perf_counter() - t_settle
    batch.step_rf_cycles(args.warmup)
    ps, elapsed = timed_cycles(batch, cases, args.steps, torch)
    value = ps / elapsed
    live = sum(int(c.sample_diagnostics()["n_e"] + c.sample_diagnostics()["n_i"]) for c in cases)

    side = {}
    probe128 = None
    if not args.no_side and not args.serve_only:
        # the same cases one at a time, each from its own RF-cycle graph
        for c in cases:
            c.step_rf_cycles(1)                     # capture each graph outside the timing
        torch.cuda.synchronize()
        p0 = sum(c.sample_diagnostics()["particle_steps"] for c in cases)
        t0 = time.perf_counter()
        for c in cases:
            c.step_rf_cycles(1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        p1 = sum(c.sample_diagnostics()["particle_steps"] for c in cases)
        side["plain_same_cases_particle_steps_per_s"] = (p1 - p0) / dt
        side["batched_over_plain"] = value / side["plain_same_cases_particle_steps_per_s"]
        batch.close()
        for c in cases:
            c.close()
        torch.cuda.empty_cache()
        progress(f"batched {value:.3e} particle-steps/s; plain {side['plain_same_cases_particle_steps_per_s']:.3e}")
        # the plain single working-size discharge
        pw = W.discharge_working()
        one = pm.Case(pw)
        autotune.tune(one, [pw], use_cache=not args.retune)
        one.step_rf_cycles(1)
        n1, d1 = timed_cycles(one, [one], 3, torch)
        side["single_case_particle_steps_per_s"] = n1 / d1
        side["single_case_push_ms"], side["single_case_collision_ms"] = one.time_kernels(50)
        side["single_case_shape"] = one.launch_shape()
        shape1 = one.launch_shape()
        one.close()
        # the same case with the paper's drive: two harmonics (delta phi = 0)
        # through a blocking capacitor
        pd = dict(pw, v2_volt=pw["v0_volt"], phase_rad=0.0, phase2_rad=0.0, cb_f_m2=1e-6)
        one = pm.Case(pd)
        one.set_launch_shape(**shape1)
        one.step_rf_cycles(1)
        one.sample_diagnostics(reset=True)
        n1, d1 = timed_cycles(one, [one], 3, torch)
        side["paper_drive_particle_steps_per_s"] = n1 / d1
        one.close()
        # the working case with 32 phase bins and the flux profiles sampled every
        # step (the extra read of x and v_x by k_flux)
        one = pm.Case(dict(pw, n_phase=32, flux_profiles=1))
        one.set_launch_shape(**shape1)
        one.step_rf_cycles(1)
        one.sample_diagnostics(reset=True)
        n1, d1 = timed_cycles(one, [one], 3, torch)
        side["phase_flux_particle_steps_per_s"] = n1 / d1
        side["phase_flux_over_single_case"] = (n1 / d1) / side["single_case_particle_steps_per_s"]
        one.close()
        progress("single working-size case done; atom flights")
        # the sputtered-atom flight
        for p_pa, law, dt_s in ((0.5, 0, 0.0), (5.0, 0, 0.0), (0.5, 1, 0.0), (0.5, 0, 1e-8)):
            src, tp = W.sputter_transport(p_pa=p_pa)
            tp.update(scatter=law, dt_s=dt_s)
            if dt_s:
                src["n_atoms"] = 1_000_000              # ~1e3 fixed steps per atom
                tp["e_max"] = 10 ** 7
            job = pm.TestParticleJob(tp)
            job.run(dict(src, n_atoms=100_000))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = job.run(src)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            side[f"tpm_{'m1_' if law else ''}{'fixed_dt_' if dt_s else ''}{p_pa:g}pa"] = {"atoms_per_s": src["n_atoms"] / dt, "events_per_s": r["events"] / dt,
                                       "events_per_atom": r["events"] / src["n_atoms"], "eta": r["eta"]}
        if args.serve_requests:
            progress(f"served stream: {args.serve_requests} requests")
            side["serving"] = serving_leg(pm, W, args, value)
        # the same push probe on twice the sweep (its first 64 cases and 64 more
        # from the same distribution, 3.5e7 particle-steps per launch: particle
        # streams well above the 256 MB Infinity Cache), in the 64-case shape
        # with its workgroups doubled
        progress("push probe on 128 sweep cases")
        p128 = W.sweep_cases(128)
        c128 = [pm.Case(p) for p in p128]
        b128 = pm.Batch(c128)
        b128.set_launch_shape(**dict(shape, work_groups=shape["work_groups"] * 2))
        k2, m2, ps2, cand2 = kernel_probe(b128, c128, args.kernel_probe)
        probe128 = {"cases": 128, "kernel_ms": k2, "particle_steps_per_launch": ps2,
                    "alg_bytes_per_launch": 16.0 * ps2, "achieved": 16.0 * ps2 / (k2 * 1e-3) / 1e9,
                    "frac": 16.0 * ps2 / (k2 * 1e-3) / 1e9 / HBM_PEAK_GBS, "collision_kernel_ms": m2,
                    "candidates_per_launch": cand2}
        b128.close()
        for c in c128:
            c.close()
        torch.cuda.empty_cache()
    else:
        batch.close()
        for c in cases:
            c.close()
        if args.serve_only and args.serve_requests:
            progress(f"served stream: {args.serve_requests} requests")
            side["serving"] = serving_leg(pm, W, args, value)

    out = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched sweep: 64 argon discharges (40 mm; 0.5-10 Pa log-uniform; 50-500 V; "
                               "128-1024 cells; 20k-500k particles per species), 13.56 MHz, dt = T_rf/1000; "
                               "step = 1 RF cycle of all 64 cases from one HIP graph; timed: the last cycles of each case's 200",
                   "case_rf_cycles": args.case_cycles,
                   "timed_rf_cycles": [settle + args.warmup + 1, settle + args.warmup + args.steps],
                   "settle_s": t_settle, "live_particles_end": live, "launch_shape": shape,
                   "shape_source": source, **side},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_step_batch (push)", "kernel_ms": k_ms, "alg_bytes_per_launch": alg_bytes,
                     "design_bytes_per_particle_step": 18.0,
                     "design_gbs": 18.0 * ps_per_launch / (k_ms * 1e-3) / 1e9,
                     "particle_steps_per_launch": ps_per_launch,
                     "above_infinity_cache": probe128,
                     "collision_kernel": {"kernel": "k_mcc_batch", "kernel_ms": mcc_ms,
                                          "candidates_per_launch": cand_per_launch,
                                          "alg_bytes_per_launch": 30.0 * cand_per_launch,
                                          "achieved_gbs": 30.0 * cand_per_launch / (mcc_ms * 1e-3) / 1e9,
                                          "bound": "hbm (gathered records share cache lines) and latency"}},
    }
    if not args.no_cpu_baseline:
        progress("oracle on the host cores")
        rate, cores, ncase, n, wall, per_core = cpu_baseline(params, 40)
        out["cpu_baseline"] = {"value": rate, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
                               "sample": f"40 PIC/MCC steps of every fourth sweep case ({ncase} cases) from "
                                         f"their initial load, one process per case on {cores} host cores "
                                         f"({n} particle-steps in {wall:.1f} s wall; {per_core:.3e} "
                                         "particle-steps/s per busy core; FP64 numpy)",
                               "single_core": cpu_single_core(W)}
    print(json.dumps(out), flush=True)
    if args.copy_probe_mb:
        copy_probe(args.copy_probe_mb, torch)


if __name__ == "__main__":
    main()
