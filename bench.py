#!/usr/bin/env python3
"""Benchmark of the FMM evaluation pass on one MI355X.

One step = the whole path over one particle set already resident in HBM:
plan (root box, Morton keys, radix sort, leaves, cells, near lists, M2L
tiles) + evaluation (P2M, M2M, M2L, L2L, L2P, P2P, combine) + release.

Headline workload: the largest configuration that fits one GPU, N = 30,000,000
particles uniform in the unit cube, charges uniform in [-1, 1), octree height
9, order 10 (seed 1005), in the compressed mixed mode (FP32 MFMA M2L on
Chebyshev-coefficient accumulators, FP32 near field).  Its dense FP64
evaluation does not fit in HBM, so the 1e-6 gate against FP64 is checked on
its density twin (468,750 particles, height 7, the same 1.79 particles per
leaf slot and the same order and tolerance), and the error against exact sums
is measured at 256 seeded targets of the 30M set itself (GPU direct sums).
The 1M-particle cube (height 6, order 7) and the 10M-particle sphere
(height 8, order 7) are reported beside it, every precision mode checked
against the dense FP64 path on the same inputs; a short serving leg runs a
Poisson request stream.  Prints one JSON line.
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

# MI355X published peaks: dense MFMA FP64 / FP32 (the FP64 / FP32 vector
# peaks are the same numbers), and HBM3E bandwidth
PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3}
HBM_GBPS = 8000.0
GATE = 1e-6
MODES = ["fp64", "mixed", "fp64_svd", "mixed_svd"]
HEADLINE = "cube30m_h9_p10"
# Workloads whose dense FP64 evaluation does not fit in HBM are checked
# against FP64 on their density twin: the same particles per leaf slot,
# order and M2L tolerance, two levels fewer.
TWIN = {"cube30m_h9_p10": "cube469k_h7_p10"}
# Compressed-M2L tolerance per workload (absent: the library default,
# 10^-order), chosen on the twin by the gate (inputs.SVD_TOL).
from paper_1206_0115_amd.inputs import SVD_TOL as HEADLINE_EPS  # noqa: E402
N_EXACT = 256  # seeded targets of the exact-sum check


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def m2l_source_hash():
    h = hashlib.sha256()
    for f in ("m2l.hip", "eval.hip"):
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
    workload that keeps its particle density, leaf occupancy and order: N/8^k
    particles of the same seeded generator with k levels fewer, starting
    from height 4 and growing by one level while 9 times the last time still
    fits the budget (the full workload if it does)."""
    import oracle
    from paper_1206_0115_amd import inputs

    def run(n_s, h_s):
        pos, q = inputs.make(kind, n_s, seed)
        t0 = time.perf_counter()
        tree = oracle.Tree(pos, h_s)
        tree.fmm(l, q)
        return time.perf_counter() - t0

    h_s = min(h, 4)
    n_s = max(1, n // 8 ** (h - h_s))
    dt = run(n_s, h_s)
    while h_s < h and 9.0 * dt <= budget_s:
        h_s += 1
        n_s = n // 8 ** (h - h_s)
        dt = run(n_s, h_s)
    # the median of three runs of the chosen sample
    times = [dt, run(n_s, h_s), run(n_s, h_s)]
    dt = float(np.median(times))
    what = "the full workload" if h_s == h else "density-, occupancy- and order-matched sample"
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": n_s / dt, "unit": "particles/s", "cores": oracle.get_threads(),
            "kind": "oracle", "cpu_model": model,
            "sample": f"{what}: {kind} N={n_s} height={h_s} order={l} seed={seed} "
                      f"(dense M2L, FP64), plan+evaluate in {dt:.1f}s (median of 3 runs: "
                      + ", ".join(f"{x:.1f}" for x in times) + " s)"}


def serve_height(pos, target=64.0):
    """Height whose non-empty leaves hold closest to `target` particles."""
    lo = pos.min(axis=0)
    L = float((pos.max(axis=0) - lo).max()) or 1.0
    best, best_d = 2, None
    for h in range(2, 9):
        side = 2 ** (h - 1)
        k = np.minimum(np.floor((pos - lo) / L * side), side - 1).astype(np.int64)
        occ = len(pos) / len(np.unique((k[:, 0] * side + k[:, 1]) * side + k[:, 2]))
        d = abs(np.log(occ) - np.log(target))
        if best_d is None or d < best_d:
            best, best_d = h, d
    return best


def serve_leg(n_requests, loads, budget_gb, prec, seed=1004):
    """Serving loop under a Poisson request stream: N log-uniform in
    [1e4, 2e6], cube or sphere 50/50, order in {3, 5, 7, 9}, height for about
    64 particles per leaf.  Latency p50/p99 and throughput at the given loads
    (rho = arrival rate x mean one-at-a-time service time), against the same
    requests run one at a time."""
    import torch

    from paper_1206_0115_amd import fmm, inputs

    fmm.lib()
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n_requests):
        n = int(np.exp(rng.uniform(np.log(1e4), np.log(2e6))))
        kind = "cube" if rng.random() < 0.5 else "sphere"
        l = int(rng.choice([3, 5, 7, 9]))
        pos, q = inputs.make(kind, n, 10_000 + i)
        h = serve_height(pos)
        reqs.append((torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda(), h, l, n))
    torch.cuda.synchronize()
    total_n = sum(r[4] for r in reqs)
    srv = fmm.Server(hbm_budget_bytes=int(budget_gb * (1 << 30)), max_active=32)

    # warm the operator caches (every order) and graphs
    warm = {}
    for r in reqs:
        warm.setdefault(r[3], r)
    for r in list(warm.values()) + reqs[:8]:
        srv.submit(r[0], r[1], r[2], r[3], prec).wait()
    # one at a time
    service = []
    for r in reqs:
        st = srv.submit(r[0], r[1], r[2], r[3], prec).wait()
        assert st.status == fmm.FMM_OK, fmm.last_error()
        service.append(st.done_s - st.submit_s)
    service = np.array(service)
    mean_s = float(service.mean())
    out = {"metric": "served particles/s (potential+force), p50/p99 latency",
           "unit": "particles/s", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "poisson_serving", "requests": len(reqs),
                      "N": "log-uniform [1e4, 2e6]", "orders": [3, 5, 7, 9],
                      "kinds": "cube/sphere 50/50", "leaf_target": 64,
                      "precision": prec, "budget_gb": budget_gb},
           "one_at_a_time": {"particles_per_s": round(total_n / float(service.sum()), 1),
                             "mean_service_ms": round(1e3 * mean_s, 3),
                             "p50_ms": round(1e3 * float(np.percentile(service, 50)), 3),
                             "p99_ms": round(1e3 * float(np.percentile(service, 99)), 3)},
           "loads": []}
    for rho in loads:
        lam = rho / mean_s
        gaps = rng.exponential(1.0 / lam, len(reqs))
        t0 = srv.now()
        arrivals = t0 + np.cumsum(gaps)
        tickets = []
        for r, ta in zip(reqs, arrivals):
            while srv.now() < ta:
                pass
            tickets.append(srv.submit(r[0], r[1], r[2], r[3], prec))
        sts = [t.wait() for t in tickets]
        assert all(s.status == fmm.FMM_OK for s in sts)
        lat = np.array([s.done_s - s.submit_s for s in sts])
        span = max(s.done_s for s in sts) - min(s.submit_s for s in sts)
        out["loads"].append({"rho": rho, "offered_req_per_s": round(lam, 2),
                             "particles_per_s": round(total_n / span, 1),
                             "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
                             "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3)})
    s = srv.stats()
    out["server"] = {k: int(getattr(s, k)) for k, _ in fmm.ServerStats._fields_}
    srv.close()
    out["value"] = max(x["particles_per_s"] for x in out["loads"])
    return out


def run_serve(args):
    out = serve_leg(args.requests, (0.5, 0.8, 0.95, 2.0), args.serve_budget_gb,
                    args.serve_precision)
    print(json.dumps(out), flush=True)


COPY_BYTES = 1 << 30  # the plain copy that calibrates the HBM counters


def probe_modes(workload):
    """The precision modes the traffic probe runs on a workload: all four
    where the dense FP64 evaluation fits, else the compressed mixed mode."""
    return ["mixed_svd"] if workload in TWIN else MODES


def run_near_probe(args):
    """Two evaluations of the workload with each near-field form (one-sided,
    then mutual), serial schedule, compressed mixed mode: the program that
    rocprofv3 runs to compare the two forms' kernels."""
    import torch

    from paper_1206_0115_amd import fmm, inputs

    kind, n, h, l, seed = inputs.CONFIGS[args.workload]
    pos, q = inputs.make(kind, n, seed)
    pos_d, q_d = torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda()
    p = fmm.Plan(pos_d, h, l, "mixed_svd", m2l_tolerance=HEADLINE_EPS.get(args.workload))
    p.set_schedule("serial")
    for near in ("one_sided", "mutual"):
        p.set_near(near)
        for _ in range(2):
            p.evaluate(q_d)
        torch.cuda.synchronize()
        print("probe", near, flush=True)
    p.release()


def run_traffic_probe(args):
    """One copy of COPY_BYTES (device to device) and then, for every
    precision mode of the workload, one plan + evaluation: the program that
    rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs to measure HBM traffic."""
    import torch

    from paper_1206_0115_amd import fmm, inputs

    fmm.lib()
    x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.neg(x, out=y)  # an elementwise kernel: reads and writes COPY_BYTES
    torch.cuda.synchronize()
    del x, y
    kind, n, h, l, seed = inputs.CONFIGS[args.workload]
    pos, q = inputs.make(kind, n, seed)
    pos_d, q_d = torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda()
    for m in probe_modes(args.workload):
        p = fmm.Plan(pos_d, h, l, m, m2l_tolerance=HEADLINE_EPS.get(args.workload))
        p.evaluate(q_d)
        torch.cuda.synchronize()
        p.release()
        print("probe", m, flush=True)


def ingest_traffic(args):
    """Turn the two counter CSVs of the traffic probe into
    profiles/m2l_traffic.json: per mode, the M2L launch's HBM bytes, with
    FETCH_SIZE and WRITE_SIZE each scaled so that the calibration copy reads
    exactly COPY_BYTES."""
    import csv

    def per_dispatch(path, counter):
        out = []
        for r in csv.DictReader(open(path)):
            if r.get("Counter_Name") == counter:
                out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
        out.sort()
        return out

    fetch = per_dispatch(args.ingest_traffic[0], "FETCH_SIZE")
    write = per_dispatch(args.ingest_traffic[1], "WRITE_SIZE")
    modes = probe_modes(args.workload)

    def scale_and_m2l(rows):
        # the elementwise negation of the COPY_BYTES buffer is the largest
        # elementwise dispatch for both counters
        cal = max(v for _, k, v in rows if "elementwise" in k)
        # one M2L launch per mode (the kernel the roofline times; the row
        # pass after it is a kernel of its own)
        m2l = [v for _, k, v in rows
               if "m2l_kernel" in k or "m2l_svd_kernel" in k or "m2l_svd_ws_kernel" in k]
        return COPY_BYTES / (cal * 1024.0), cal, m2l

    sf, calf, mf = scale_and_m2l(fetch)
    sw, calw, mw = scale_and_m2l(write)
    if len(mf) != len(modes) or len(mw) != len(modes):
        raise SystemExit(f"expected {len(modes)} M2L dispatches, got {len(mf)}/{len(mw)}")
    path = os.path.join(ROOT, "profiles", "m2l_traffic.json")
    d = json.load(open(path)) if os.path.exists(path) else {}
    d[args.workload] = {}
    for m, fv, wv in zip(modes, mf, mw):
        d[args.workload][m] = {
            "fetch_kib_raw": fv, "write_kib_raw": wv,
            "fetch_scale": sf, "write_scale": sw,
            "copy_fetch_kib_raw": calf, "copy_write_kib_raw": calw,
            "bytes_per_launch": fv * 1024.0 * sf + wv * 1024.0 * sw,
            "kernel_sha": m2l_source_hash()}
    json.dump(d, open(path, "w"), indent=1)
    print(json.dumps(d[args.workload]))


class Bench:
    """The measurements of one workload on one stream."""

    def __init__(self, name, stream):
        import torch

        from paper_1206_0115_amd import fmm, inputs

        self.fmm, self.torch = fmm, torch
        self.name = name
        self.kind, self.n, self.h, self.l, self.seed = inputs.CONFIGS[name]
        self.eps = HEADLINE_EPS.get(name)
        pos, q = inputs.make(self.kind, self.n, self.seed)
        self.pos, self.q = pos, q
        dev = torch.device("cuda:0")
        self.stream = stream
        self.pos_d = torch.from_numpy(pos).to(dev)
        self.q_d = torch.from_numpy(q).to(dev)
        self.phi = torch.empty(self.n, dtype=torch.float64, device=dev)
        self.frc = torch.empty(self.n, 3, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()

    def plan(self, prec, kernel="inv_r"):
        return self.fmm.Plan(self.pos_d, self.h, self.l, prec, stream=self.stream,
                             kernel=kernel, m2l_tolerance=self.eps)

    def new_events(self, k):
        ev = [self.torch.cuda.Event(enable_timing=True) for _ in range(k)]
        for x in ev:  # materialise the HIP events before handing them over
            x.record(self.stream)
        return ev

    def check_modes(self, quick_steps):
        """Every mode against the dense FP64 path on the same inputs, and a
        short timing of each."""
        torch, s = self.torch, self.stream
        out, infos = {}, {}
        with torch.cuda.stream(s):
            plan = self.plan("fp64")
            p64, f64 = plan.evaluate(self.q_d, stream=s)
            s.synchronize()
            p64, f64 = p64.cpu().numpy(), f64.cpu().numpy()
            for m in MODES:
                plan.set_precision(m)
                pm, fm = plan.evaluate(self.q_d, stream=s)
                s.synchronize()
                e_phi, e_f = rel(pm.cpu().numpy(), p64), rel(fm.cpu().numpy(), f64)
                out[m] = {"rel_l2_vs_fp64": max(e_phi, e_f), "phi": e_phi, "F": e_f,
                          "within_gate": max(e_phi, e_f) <= GATE,
                          "m2l_split": plan.m2l_split()}
                infos[m] = plan.info()
            self.svd = plan.svd_info()
            plan.release()
        for m in MODES:
            ms, _, m2l_ms = self.run_steps(m, quick_steps, 1)
            out[m].update({"ms_per_step": round(ms, 4),
                           "particles_per_s": round(self.n / (ms / 1e3), 1),
                           "m2l_avg_ms": round(float(np.mean(m2l_ms)), 4),
                           "m2l_flops": float(infos[m].m2l_flops)})
        return out

    def run_steps(self, prec, steps, warmup):
        """Plan + evaluate + release per step on the default (forked)
        schedule; the M2L launch bracketed by HIP events in every step."""
        torch, fmm, s = self.torch, self.fmm, self.stream
        with torch.cuda.stream(s):
            ev = [self.new_events(4) for _ in range(steps + warmup)]
            s.synchronize()
            torch.cuda.synchronize()
            t0 = None
            for i, (s0, s1, m0, m1) in enumerate(ev):
                if i == warmup:
                    s.synchronize()
                    t0 = time.perf_counter()
                fmm.set_m2l_timing_events(m0, m1)
                s0.record(s)
                p = self.plan(prec)
                p.evaluate(self.q_d, self.phi, self.frc, stream=s)
                s1.record(s)
                if i == 0:
                    self.info = p.info()
                    self.split = p.m2l_split()
                    self.step_svd = p.svd_info() if prec.endswith("svd") else None
                p.release()
            s.synchronize()
            t1 = time.perf_counter()
            fmm.set_m2l_timing_events(None, None)
        torch.cuda.synchronize()
        step_ms = np.array([a.elapsed_time(b) for a, b, _, _ in ev[warmup:]])
        m2l_ms = np.array([a.elapsed_time(b) for _, _, a, b in ev[warmup:]])
        return (t1 - t0) * 1e3 / steps, step_ms, m2l_ms

    def eval_only(self, prec, steps):
        torch, s = self.torch, self.stream
        with torch.cuda.stream(s):
            p = self.plan(prec)
            p.evaluate(self.q_d, self.phi, self.frc, stream=s)
            s.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                p.evaluate(self.q_d, self.phi, self.frc, stream=s)
            s.synchronize()
            dt = (time.perf_counter() - t0) * 1e3 / steps
            p.release()
        return dt

    def schedule_times(self, prec, steps):
        """Evaluate-only ms per step for each schedule, eager and replayed
        from the plan's captured graph."""
        torch, s = self.torch, self.stream
        out = {}
        with torch.cuda.stream(s):
            p = self.plan(prec)
            for sched in ("serial", "forked", "pipelined"):
                for graph in (False, True):
                    p.set_schedule(sched)
                    p.set_graph(graph)
                    p.evaluate(self.q_d, self.phi, self.frc, stream=s)
                    s.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(steps):
                        p.evaluate(self.q_d, self.phi, self.frc, stream=s)
                    s.synchronize()
                    out[sched + ("+graph" if graph else "")] = round(
                        (time.perf_counter() - t0) * 1e3 / steps, 4)
            p.release()
        return out

    def step_times(self, prec, reps):
        """Average duration of each bulk operator's kernel, every operator on
        one stream (serial schedule, so no kernel shares the GPU)."""
        torch, fmm, s = self.torch, self.fmm, self.stream
        with torch.cuda.stream(s):
            p = self.plan(prec)
            # the steps this plan runs (the events are recorded once when
            # made, so a step that never runs would time as zero)
            names = ["p2p"]
            if self.h >= 3:
                names += ["m2l", "p2m", "l2p"]
                if p.m2l_split() > 1:
                    names.append("loc_sum")
            if self.h >= 4:
                names += ["m2m", "l2l"]
            p.set_schedule("serial")
            p.evaluate(self.q_d, self.phi, self.frc, stream=s)
            ev = [self.new_events(2 * len(names)) for _ in range(reps)]
            s.synchronize()
            for e in ev:
                for k, name in enumerate(names):
                    fmm.set_step_timing_events(name, e[2 * k], e[2 * k + 1])
                p.evaluate(self.q_d, self.phi, self.frc, stream=s)
            s.synchronize()
            for name in names:
                fmm.set_step_timing_events(name, None, None)
            p.release()
        return {name: float(np.mean([e[2 * k].elapsed_time(e[2 * k + 1]) for e in ev]))
                for k, name in enumerate(names)}

    def near_forms(self, prec, reps):
        """The near field's two forms (one-sided; mutual, Sec. 5's reduction
        form) on this workload and mode: the average time of the near-field
        launches (serial schedule, HIP events around them), and the mutual
        form's output against the one-sided one's."""
        torch, fmm, s = self.torch, self.fmm, self.stream
        out, res = {}, {}
        with torch.cuda.stream(s):
            p = self.plan(prec)
            p.set_schedule("serial")
            for near in ("one_sided", "mutual"):
                p.set_near(near)
                p.evaluate(self.q_d, self.phi, self.frc, stream=s)
                ev = [self.new_events(2) for _ in range(reps)]
                s.synchronize()
                for e in ev:
                    fmm.set_step_timing_events("p2p", e[0], e[1])
                    p.evaluate(self.q_d, self.phi, self.frc, stream=s)
                s.synchronize()
                fmm.set_step_timing_events("p2p", None, None)
                res[near] = (self.phi.cpu().numpy(), self.frc.cpu().numpy())
                out[near + "_ms"] = round(float(np.mean([e[0].elapsed_time(e[1]) for e in ev])), 4)
            p.release()
        out["mutual_speedup"] = round(out["one_sided_ms"] / out["mutual_ms"], 3)
        out["mutual_vs_one_sided_rel_l2"] = max(rel(res["mutual"][0], res["one_sided"][0]),
                                                rel(res["mutual"][1], res["one_sided"][1]))
        return out

    def exact_error(self, count):
        """Error of the last evaluation's output against exact sums (GPU
        direct summation over all sources) at `count` seeded targets."""
        torch, s = self.torch, self.stream
        idx = np.sort(np.random.default_rng(self.seed).choice(self.n, count, replace=False))
        with torch.cuda.stream(s):
            pe, fe = self.fmm.direct_sampled(self.pos_d, self.q_d,
                                             torch.from_numpy(idx).cuda(), stream=s)
            s.synchronize()
        pe, fe = pe.cpu().numpy(), fe.cpu().numpy()
        phi = self.phi.cpu().numpy()[idx]
        frc = self.frc.cpu().numpy()[idx]
        return {"targets": count, "phi": rel(phi, pe), "F": rel(frc, fe)}

    def kernels(self, prec, reps):
        st = self.step_times(prec, reps)
        inf, n, l3 = self.info, self.n, self.l ** 3
        flops = float(inf.m2l_flops)
        peak = PEAK_TFLOPS["mixed" if prec.startswith("mixed") else "fp64"]
        p2p_flops = 20.0 * float(inf.near_pairs)
        p2m_bytes = 32.0 * n + 8.0 * l3 * float(inf.n_leaf)
        l2p_bytes = 64.0 * n + 8.0 * l3 * float(inf.n_leaf)
        h = self.h
        # three 1-D passes of l^4 FMAs per cell: M2M and L2L per child cell
        # below level 2, the coefficient rows per cell of levels >= 2
        trans = 6.0 * self.l ** 4
        children = float(sum(inf.ncell[lv] for lv in range(3, h)))
        rows = float(sum(inf.ncell[lv] for lv in range(2, h)))

        def rate(work, ms, pk, unit, bound, what):
            if ms is None:
                return None
            a = work / (ms / 1e3) / (1e12 if unit == "TFLOP/s" else 1e9)
            return {"bound": bound, "avg_ms": round(ms, 4), "achieved": round(a, 2),
                    "peak": pk, "unit": unit, "frac": round(a / pk, 4),
                    "work_per_launch": work, "work": what}

        out = {
            "m2l": rate(flops, st.get("m2l"), peak, "TFLOP/s", "mfma", "algorithmic flops"),
            "p2p": rate(p2p_flops, st.get("p2p"), peak, "TFLOP/s", "valu",
                        "20 flops per directed near pair"),
            "p2m": rate(p2m_bytes, st.get("p2m"), HBM_GBPS, "GB/s", "hbm",
                        "32 B per particle read + l^3 x 8 B per leaf written"),
            "l2p": rate(l2p_bytes, st.get("l2p"), HBM_GBPS, "GB/s", "hbm",
                        "64 B per particle read and written + l^3 x 8 B per leaf read"),
            "m2m": rate(trans * children, st.get("m2m"), PEAK_TFLOPS["fp64"], "TFLOP/s", "alu",
                        "6 l^4 FP64 flops per child cell, all levels"),
            "l2l": rate(trans * children, st.get("l2l"), PEAK_TFLOPS["fp64"], "TFLOP/s", "alu",
                        "6 l^4 FP64 flops per child cell, all levels"),
            "loc_sum": rate(8.0 * self.l ** 3 * rows * (getattr(self, "split", 1) + 1),
                            st.get("loc_sum"), HBM_GBPS, "GB/s", "hbm",
                            "l^3 x 8 B per part and cell of levels >= 2 read, the cell's row written"),
        }
        return {k: v for k, v in out.items() if v is not None}

    def second_kernel(self, prec, steps):
        """The 1/r^2 kernel on the same workload and mode: plan + evaluate +
        release per step, and its error against its own FP64 evaluation."""
        torch, s = self.torch, self.stream
        with torch.cuda.stream(s):
            ref = self.plan("fp64", kernel="inv_r2")
            pr, fr = ref.evaluate(self.q_d, stream=s)
            s.synchronize()
            pr, fr = pr.cpu().numpy(), fr.cpu().numpy()
            ref.release()
            p = self.plan(prec, kernel="inv_r2")
            pm, fm = p.evaluate(self.q_d, stream=s)
            s.synchronize()
            err = max(rel(pm.cpu().numpy(), pr), rel(fm.cpu().numpy(), fr))
            p.release()
            for i in range(steps + 1):
                if i == 1:
                    s.synchronize()
                    t0 = time.perf_counter()
                p = self.plan(prec, kernel="inv_r2")
                p.evaluate(self.q_d, self.phi, self.frc, stream=s)
                p.release()
            s.synchronize()
            dt = (time.perf_counter() - t0) * 1e3 / steps
        return {"kernel": "1/r^2", "precision": prec, "ms_per_step": round(dt, 4),
                "particles_per_s": round(self.n / (dt / 1e3), 1), "rel_l2_vs_fp64": err}

    def release(self):
        del self.pos_d, self.q_d, self.phi, self.frc
        self.torch.cuda.synchronize()
        self.torch.cuda.empty_cache()
        self.fmm.trim_cache()


def side_config(name, stream, steps):
    """A workload reported beside the headline: every mode against FP64 on
    it, the fastest mode within the gate timed, its error against exact sums."""
    b = Bench(name, stream)
    modes = b.check_modes(max(3, steps // 4))
    ok = [m for m in MODES if modes[m]["within_gate"]]
    prec = min(ok, key=lambda m: modes[m]["ms_per_step"])
    ms, step_ms, m2l_ms = b.run_steps(prec, steps, 2)
    out = {"kind": b.kind, "N": b.n, "height": b.h, "order": b.l, "seed": b.seed,
           "precision": prec, "m2l_svd_tolerance": b.svd.eps,
           "ms_per_step": round(ms, 4), "particles_per_s": round(b.n / (ms / 1e3), 1),
           "p50_ms": round(float(np.percentile(step_ms, 50)), 4),
           "p99_ms": round(float(np.percentile(step_ms, 99)), 4),
           "eval_only_ms": round(b.eval_only(prec, max(5, steps)), 4),
           "rel_l2_vs_fp64": modes[prec]["rel_l2_vs_fp64"],
           "rel_l2_vs_exact": b.exact_error(N_EXACT), "modes": modes,
           "kernels": b.kernels(prec, 5),
           "eval_only_ms_by_schedule": b.schedule_times(prec, max(5, steps)),
           "near_field_forms": b.near_forms(prec, 5)}
    if name == "cube1m_h6_p7":
        out["second_kernel"] = b.second_kernel(prec, max(5, steps // 2))
    b.release()
    return out


def summarize_counters(paths):
    """Every counter of every kernel in rocprofv3 --pmc CSVs (one or more
    passes), as a markdown table: the value of each dispatch in dispatch
    order (or the mean over more than 8).  Kernel names are shortened to
    their function name and template arguments."""
    import csv
    import re
    acc = {}
    for path in paths:
        for r in csv.DictReader(open(path)):
            name = r.get("Kernel_Name", "")
            m = re.match(r"(?:void )?(?:fmm::)?([A-Za-z0-9_]+(?:<[^>(]*>)?)", name)
            k = m.group(1) if m else name[:60]
            c = r.get("Counter_Name")
            acc.setdefault((k, c), []).append(float(r["Counter_Value"]))
    counters = sorted({c for _, c in acc})
    kernels = sorted({k for k, _ in acc})
    lines = ["| kernel | " + " | ".join(counters) + " |",
             "|---|" + "---|" * len(counters)]
    for k in kernels:
        cells = []
        for c in counters:
            v = acc.get((k, c))
            # up to 8 dispatches: each value in dispatch order; else the mean
            if not v:
                cells.append("")
            elif len(v) <= 8:
                cells.append(" / ".join(f"{x:.4g}" for x in v))
            else:
                cells.append(f"mean {np.mean(v):.4g} of {len(v)}")
        lines.append(f"| {k} | " + " | ".join(cells) + " |")
    print("\n".join(lines))


def summarize_trace(path, top, only=None):
    """Per-(kernel, grid) dispatch count and mean / total duration from a
    rocprofv3 --kernel-trace CSV, as a markdown table of the `top` kernels by
    total time.  The grid separates launches of one kernel over different
    workloads (a headline workload and its twin).  `only`: a regular
    expression; the overlap of queues then counts only the kernels whose
    names match it (e.g. the evaluation kernels of serving batches)."""
    import csv
    import re
    acc = {}
    for r in csv.DictReader(open(path)):
        name = r.get("Kernel_Name", "")
        m = re.match(r"(?:void )?(?:fmm::)?([A-Za-z0-9_]+(?:<[^>(]*>)?)", name)
        k = m.group(1) if m else name[:60]
        grid = "x".join(r.get(f"Grid_Size_{d}", "?") for d in "XYZ")
        dt = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
        acc.setdefault((k, grid), []).append(dt)
    rows = sorted(acc.items(), key=lambda kv: -sum(kv[1]))[:top]
    print("| kernel | grid (threads) | dispatches | mean ms | total ms |")
    print("|---|---|---|---|---|")
    for (k, grid), v in rows:
        print(f"| {k} | {grid} | {len(v)} | {np.mean(v):.4f} | {np.sum(v):.2f} |")
    # time during which kernels of two or more hardware queues ran at once
    spans = {}
    for r in csv.DictReader(open(path)):
        if only and not re.search(only, r.get("Kernel_Name", "")):
            continue
        qid = r.get("Queue_Id") or r.get("Stream_Id") or "?"
        spans.setdefault(qid, []).append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    ev = []
    for qid, v in spans.items():
        for a, b in v:
            ev += [(a, 1, qid), (b, -1, qid)]
    ev.sort(key=lambda e: (e[0], e[1]))
    active, busy, both, last = {}, 0, 0, None
    for t, d, qid in ev:
        if last is not None:
            n = sum(1 for c in active.values() if c > 0)
            if n >= 1:
                busy += t - last
            if n >= 2:
                both += t - last
        active[qid] = active.get(qid, 0) + d
        last = t
    print(f"\n{'kernels matching ' + only + ': ' if only else ''}"
          f"queues with kernels: {len(spans)}; time with a kernel running "
          f"{busy * 1e-6:.2f} ms, with kernels of two or more queues at once "
          f"{both * 1e-6:.2f} ms")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=HEADLINE)
    ap.add_argument("--precision", default="auto", choices=["auto"] + MODES)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-side", action="store_true",
                    help="only the headline workload (no side configurations, no serving leg)")
    ap.add_argument("--cpu-budget", type=float, default=30.0)
    ap.add_argument("--serve", action="store_true",
                    help="benchmark the serving loop instead (Poisson request stream)")
    ap.add_argument("--near-probe", action="store_true",
                    help="evaluate --workload with each near-field form (for rocprofv3)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="the program to run under rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE")
    ap.add_argument("--ingest-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/m2l_traffic.json from the two counter CSVs")
    ap.add_argument("--summarize-counters", nargs="+", metavar="CSV",
                    help="print per-kernel counter means from rocprofv3 --pmc CSVs")
    ap.add_argument("--trace-only", metavar="REGEX",
                    help="with --summarize-trace: count queue overlap over matching kernels only")
    ap.add_argument("--summarize-trace", metavar="CSV",
                    help="print per-kernel durations from a rocprofv3 --kernel-trace CSV")
    ap.add_argument("--requests", type=int, default=500)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-precision", default="mixed_svd", choices=MODES)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print("bench.py measures one GPU only: this FMM build has no multi-GPU path "
                  f"(asked for --gpus {args.gpus}, WORLD_SIZE={world}).", file=sys.stderr)
        sys.exit(2)

    if args.summarize_trace:
        summarize_trace(args.summarize_trace, 25, args.trace_only)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return
    if args.ingest_traffic:
        ingest_traffic(args)
        return
    if args.near_probe:
        run_near_probe(args)
        return
    if args.traffic_probe:
        run_traffic_probe(args)
        return
    if args.serve:
        run_serve(args)
        return

    import torch

    from paper_1206_0115_amd import fmm

    fmm.lib()  # fails loudly if the HIP library is not built
    stream = torch.cuda.Stream(device=torch.device("cuda:0"))
    name = args.workload
    twin = TWIN.get(name)
    log = lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True)

    # the gate: every mode against dense FP64, on the workload or its twin
    log(f"modes against FP64 on {twin or name}")
    g = Bench(twin or name, stream)
    gate = g.check_modes(3)
    g.release()
    ok = [m for m in MODES if gate[m]["within_gate"]]
    if args.precision != "auto":
        precision = args.precision
    elif twin:
        # at the twin's size every mode runs; at the full size only the
        # compressed ones are practical (dense order-10 M2L: 5e15 flops)
        precision = min([m for m in ok if m.endswith("svd")],
                        key=lambda m: gate[m]["ms_per_step"])
    else:
        precision = min(ok, key=lambda m: gate[m]["ms_per_step"])

    log(f"headline {name} {precision}: {args.warmup} + {args.steps} steps")
    b = Bench(name, stream)
    ms, step_ms, m2l_ms = b.run_steps(precision, args.steps, args.warmup)
    exact = b.exact_error(N_EXACT)
    log(f"headline {ms:.1f} ms per step; eval only")
    eval_ms = b.eval_only(precision, 3 if b.n > 10_000_000 else max(5, args.steps))
    log("kernels (serial schedule)")
    kernels = b.kernels(precision, 2 if b.n > 10_000_000 else 10)
    inf = b.info
    flops = float(inf.m2l_flops)
    m2l_s = float(np.mean(m2l_ms)) / 1e3
    achieved = flops / m2l_s / 1e12
    peak = PEAK_TFLOPS["mixed" if precision.startswith("mixed") else "fp64"]
    roof = {"bound": "mfma",
            "kernel": "m2l_svd_ws_kernel" if precision.endswith("svd") else "m2l_kernel",
            "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": load_traffic(name, precision),
            "flops_per_launch": flops, "far_pairs": int(inf.far_pairs),
            "m2l_split": b.split, "avg_launch_ms": round(m2l_s * 1e3, 4)}
    sv = b.step_svd
    kind, n, h, l, seed = b.kind, b.n, b.h, b.l, b.seed
    b.release()

    side, serving = {}, None
    if not args.no_side:
        for cfg in ("cube1m_h6_p7", "sphere10m_h8_p7"):
            log(f"side configuration {cfg}")
            side[cfg] = side_config(cfg, stream, args.steps)
        log("serving leg")
        serving = serve_leg(60, (0.8,), 64.0, "mixed_svd")

    base = None
    if not args.no_cpu_baseline:
        log("cpu baseline")
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
        "dtype": "f32+f64" if precision.startswith("mixed") else "f64",
        "data": "synthetic",
        "config": {"workload": name, "kind": kind, "N": n, "height": h, "order": l,
                   "seed": seed, "precision": precision,
                   "m2l_svd_tolerance": sv.eps if sv else None,
                   "step": "plan+evaluate+release, inputs resident in HBM",
                   "schedule": "forked (near field beside the far chain)"},
        "p50_ms": round(float(np.percentile(step_ms, 50)), 4),
        "p99_ms": round(float(np.percentile(step_ms, 99)), 4),
        "eval_only_ms": round(eval_ms, 4),
        "eval_only_particles_per_s": round(n / (eval_ms / 1e3), 1),
        "rel_l2_vs_fp64": gate[precision]["rel_l2_vs_fp64"],
        "gate_checked_on": twin or name,
        "rel_l2_vs_exact": exact,
        "modes": gate,
        "svd_weighted_rank": round(sv.weighted_rank, 3) if sv else None,
        "roofline": roof,
        "kernels": kernels,
        "configs": side,
        "serving": serving,
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
