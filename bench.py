"""Throughput of the PIC/MCC + test-particle hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (synthetic, seeded): the working-size discharge -- 40 mm gap, 1024
cells, 1M electrons + 1M Ar+, 300 V at 13.56 MHz, Ar 0.5 Pa 300 K, dt = T_rf/2000,
FP32 particles, int64 charge, FP64 Poisson -- coupled one way to the sputtered
Al atoms.  One bench step is one RF cycle: 2000 PIC/MCC time steps replayed from
a HIP graph, then the yield rule on that cycle's target ion impacts and the
collisional flight of the atoms they sputter.  Inputs are resident in HBM before
the timed region.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (batched vs plain) at oracle-matched stats; p50/p99 case latency"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40, help="timed RF cycles")
    ap.add_argument("--warmup", type=int, default=5, help="untimed RF cycles")
    ap.add_argument("--np-each", type=int, default=1_000_000)
    ap.add_argument("--kernel-probe", type=int, default=200, help="single steps timed one by one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=100)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB (counter calibration)")
    return ap.parse_args()


def kernel_probe(pm, case, n, torch):
    """Average duration of the fused step kernel: each launch bracketed by HIP
    events on the stream it is launched on."""
    st = torch.cuda.current_stream()
    times = []
    d0 = case.sample_diagnostics()
    for _ in range(n):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        case.step(1)
        b.record(st)
        times.append((a, b))
    torch.cuda.synchronize()
    d1 = case.sample_diagnostics()
    ms = [a.elapsed_time(b) for a, b in times]
    ps = d1["particle_steps"] - d0["particle_steps"]
    cand = int(sum(d1["candidates"]) - sum(d0["candidates"]))
    return sum(ms) / len(ms), ps / n, cand / n


def measured_traffic(probe_launches):
    """HBM bytes per probe launch of the step kernel from the committed counter
    passes (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's reading
    for a copy of known size), or None when the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "k_step_traffic.json")
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


def cpu_baseline(p, steps):
    import oracle.pic as P
    d = P.Discharge(p)
    n = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        n += len(d.sp[0]) + len(d.sp[1])
        d.step()
    dt = time.perf_counter() - t0
    return n / dt, n, dt


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is a design "
                                   "note (independent cases / atom ranges), not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_1607_04069_amd as pm
    import workloads as W

    p = W.discharge_working(np_each=args.np_each)
    src_tp, tp = W.sputter_transport(p_pa=p["p_pa"])
    tp["gap_m"] = p["gap_m"]
    torch.cuda.set_device(0)
    case = pm.Case(p)
    job = pm.TestParticleJob(tp)

    # The dominant kernel, timed first from the seeded initial load (the same
    # launches in every run, so rocprofv3 passes of this command see them too):
    # the fused step moves 16 B per particle-step (x and v_x read and written in
    # FP32) plus 24 B per null-collision candidate (v_y, v_z read + written, id).
    k_ms, ps_per_launch, cand_per_launch = kernel_probe(pm, case, args.kernel_probe, torch)
    alg_bytes = 16.0 * ps_per_launch + 24.0 * cand_per_launch
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    case.sample_diagnostics(reset=True)

    def one_cycle():
        case.step_rf_cycles(1)
        src = case.inject_sputtered(yield_const=1.0, u_s_ev=3.4, e_cut_ev=200.0, seed=1607, job_id=3)
        r = job.run(src)
        case.sample_diagnostics(reset=True)
        return r["events"]

    for _ in range(args.warmup):
        one_cycle()
    torch.cuda.synchronize()
    d0 = case.sample_diagnostics(reset=True)
    tp_events = 0
    pic_ps = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        case.step_rf_cycles(1)
        src = case.inject_sputtered(yield_const=1.0, u_s_ev=3.4, e_cut_ev=200.0, seed=1607, job_id=3)
        tp_events += job.run(src)["events"]
        pic_ps += case.sample_diagnostics(reset=True)["particle_steps"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = (pic_ps + tp_events) / elapsed

    d_end = case.sample_diagnostics()

    out = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "working-size discharge: 40 mm, 1024 cells, "
                               f"{args.np_each} e + {args.np_each} Ar+, 300 V 13.56 MHz, Ar 0.5 Pa 300 K, "
                               "dt = T_rf/2000; step = 1 RF cycle (2000 PIC/MCC steps) + sputter "
                               "source + Al flight (VHS, 0.5 Pa)",
                   "pic_particle_steps_per_s": pic_ps / elapsed,
                   "tpm_events_per_s": tp_events / elapsed,
                   "live_particles": [int(d_end["n_e"]), int(d_end["n_i"])]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.kernel_probe),
                     "kernel": "k_step", "kernel_ms": k_ms, "alg_bytes_per_launch": alg_bytes,
                     "particle_steps_per_launch": ps_per_launch},
    }
    if not args.no_cpu_baseline:
        rate, n, dt = cpu_baseline(p, args.cpu_steps)
        out["cpu_baseline"] = {"value": rate, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"{args.cpu_steps} PIC/MCC steps of the same discharge from its "
                                         f"initial load ({n} particle-steps in {dt:.1f} s, FP64 numpy, "
                                         "one thread)"}
    print(json.dumps(out), flush=True)
    case.close()
    if args.copy_probe_mb:
        n = args.copy_probe_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n}), flush=True)


if __name__ == "__main__":
    main()
