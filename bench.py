#!/usr/bin/env python3
"""Benchmark of the FMM evaluation pass on one MI355X.

One step = the whole path over one particle set already resident in HBM:
plan (root box, Morton keys, radix sort, leaves, cells, near lists, M2L
tiles) + evaluation (P2M, M2M, M2L, L2L, L2P, P2P, combine) + release.
Workload: N = 1,000,000 particles uniform in the unit cube, charges uniform
in [-1, 1), octree height 6, order 7 (seed 1002).

The headline runs the mixed-precision path when its relative L2 error
against the FP64 path on the same inputs is at most 1e-6 (checked here on
every run), else the FP64 path.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3}  # dense MFMA: FP64, FP32
GATE = 1e-6


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def m2l_source_hash():
    h = hashlib.sha256()
    for f in ("m2l.hip",):
        h.update(open(os.path.join(ROOT, "paper_1206_0115_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(workload, precision):
    """HBM bytes per M2L launch from the committed rocprofv3 counter summary,
    or None when it is absent or was taken on another version of the kernel."""
    path = os.path.join(ROOT, "profiles", "m2l_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d[workload][precision]
        if e.get("kernel_sha") != m2l_source_hash():
            return None
        return float(e["bytes_per_launch"])
    except Exception:
        return None


def cpu_baseline(kind, n, h, l, seed, budget_s):
    """The oracle (plan + FMM, all host cores) on a bounded sample of the
    workload.  The sample keeps the particle density and the leaf size: N/8
    particles with one level fewer (the same seeded generator).  When 8x that
    sample's time fits the budget, the full workload is timed instead."""
    import oracle
    from paper_1206_0115_amd import inputs

    def run(n_s, h_s):
        pos, q = inputs.make(kind, n_s, seed)
        t0 = time.perf_counter()
        tree = oracle.Tree(pos, h_s)
        tree.fmm(l, q)
        return time.perf_counter() - t0

    n_s, h_s = n // 8, h - 1
    dt = run(n_s, h_s)
    what = "density- and leaf-size-matched sample"
    if 9.0 * dt <= budget_s:
        n_s, h_s = n, h
        dt = run(n_s, h_s)
        what = "the full workload"
    return {"value": n_s / dt, "unit": "particles/s", "cores": oracle.get_threads(),
            "kind": "oracle",
            "sample": f"{what}: {kind} N={n_s} height={h_s} order={l} seed={seed}, "
                      f"plan+evaluate in {dt:.1f}s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cube1m_h6_p7")
    ap.add_argument("--precision", default="auto", choices=["auto", "fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=30.0)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print("bench.py measures one GPU only: this FMM build has no multi-GPU path "
                  f"(asked for --gpus {args.gpus}, WORLD_SIZE={world}).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1206_0115_amd import fmm, inputs

    fmm.lib()  # fails loudly if the HIP library is not built
    kind, n, h, l, seed = inputs.CONFIGS[args.workload]
    pos, q = inputs.make(kind, n, seed)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    pos_d = torch.from_numpy(pos).to(dev)
    q_d = torch.from_numpy(q).to(dev)
    phi = torch.empty(n, dtype=torch.float64, device=dev)
    frc = torch.empty(n, 3, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    # FP64 reference and the mixed path's error on the same inputs
    with torch.cuda.stream(stream):
        plan = fmm.Plan(pos_d, h, l, "fp64", stream=stream)
        p64, f64 = plan.evaluate(q_d, stream=stream)
        stream.synchronize()
        p64, f64 = p64.cpu().numpy(), f64.cpu().numpy()
        plan.set_precision("mixed")
        pm, fm = plan.evaluate(q_d, stream=stream)
        stream.synchronize()
        err_mixed = max(rel(pm.cpu().numpy(), p64), rel(fm.cpu().numpy(), f64))
        info = plan.info()
        plan.release()
    precision = args.precision
    if precision == "auto":
        precision = "mixed" if err_mixed <= GATE else "fp64"

    def run_steps(prec, steps, warmup):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps + warmup)]
        with torch.cuda.stream(stream):
            for e in ev:  # materialise the HIP events before handing them over
                for x in e:
                    x.record(stream)
            stream.synchronize()
            torch.cuda.synchronize()
            t0 = None
            for i, (s0, s1, m0, m1) in enumerate(ev):
                if i == warmup:
                    stream.synchronize()
                    t0 = time.perf_counter()
                fmm.set_m2l_timing_events(m0, m1)
                s0.record(stream)
                p = fmm.Plan(pos_d, h, l, prec, stream=stream)
                p.evaluate(q_d, phi, frc, stream=stream)
                s1.record(stream)
                p.release()
            stream.synchronize()
            t1 = time.perf_counter()
            fmm.set_m2l_timing_events(None, None)
        torch.cuda.synchronize()
        step_ms = np.array([a.elapsed_time(b) for a, b, _, _ in ev[warmup:]])
        m2l_ms = np.array([a.elapsed_time(b) for _, _, a, b in ev[warmup:]])
        return (t1 - t0) * 1e3 / steps, step_ms, m2l_ms

    def eval_only(prec, steps):
        with torch.cuda.stream(stream):
            p = fmm.Plan(pos_d, h, l, prec, stream=stream)
            p.evaluate(q_d, phi, frc, stream=stream)
            stream.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                p.evaluate(q_d, phi, frc, stream=stream)
            stream.synchronize()
            dt = (time.perf_counter() - t0) * 1e3 / steps
            p.release()
        return dt

    ms, step_ms, m2l_ms = run_steps(precision, args.steps, args.warmup)
    eval_ms = eval_only(precision, max(5, args.steps))
    other = "fp64" if precision == "mixed" else "mixed"
    ms_other, _, m2l_other = run_steps(other, max(3, args.steps // 4), 1)

    flops = 2.0 * float(l) ** 6 * info.far_pairs  # dense M2L, one launch
    m2l_s = float(np.mean(m2l_ms)) / 1e3
    achieved = flops / m2l_s / 1e12
    peak = PEAK_TFLOPS[precision]
    roof = {"bound": "mfma", "kernel": "m2l_kernel", "achieved": round(achieved, 2),
            "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
            "traffic": load_traffic(args.workload, precision),
            "flops_per_launch": flops, "far_pairs": int(info.far_pairs),
            "avg_launch_ms": round(m2l_s * 1e3, 4)}

    base = None
    if not args.no_cpu_baseline:
        base = cpu_baseline(kind, n, h, l, seed, args.cpu_budget)

    value = n / (ms / 1e3)
    out = {
        "metric": "particles/s (potential+force) at rel. L2 err <=1e-6 vs FP64; p50/p99 latency",
        "value": round(value, 1),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "kind": kind, "N": n, "height": h, "order": l,
                   "seed": seed, "precision": precision,
                   "step": "plan+evaluate+release, inputs resident in HBM"},
        "p50_ms": round(float(np.percentile(step_ms, 50)), 4),
        "p99_ms": round(float(np.percentile(step_ms, 99)), 4),
        "eval_only_ms": round(eval_ms, 4),
        "eval_only_particles_per_s": round(n / (eval_ms / 1e3), 1),
        "rel_l2_mixed_vs_fp64": err_mixed,
        "other_precision": {"precision": other, "ms_per_step": round(ms_other, 4),
                            "particles_per_s": round(n / (ms_other / 1e3), 1),
                            "m2l_avg_ms": round(float(np.mean(m2l_other)), 4)},
        "roofline": roof,
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
