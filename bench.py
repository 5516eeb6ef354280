#!/usr/bin/env python3
"""Benchmark: full spectral Ewald evaluation of the periodic Stokeslet sum on one MI355X.

One step = one ``ewald_eval`` (bin/sort, P2P, P2G, FFT+CNV+IFFT, G2P+self+sum+unsort)
over device-resident synthetic inputs.  Prints ONE JSON line on stdout.

Default workload "c2": N = 1e6 uniform in the unit cube, forces N(0,1) mean-removed,
tol 1e-8, 128^3 grid, FP64.  The window support is derived from tol (the Gaussian window
needs P = 16 for 1e-8; ``--P 12`` runs the configured support and reports its error).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particles/s full Stokeslet Ewald eval at 1e-6 rel err; P2G GB/s; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
FP32_VECTOR_TFLOPS = 157.3
FP64_MFMA_PEAK_TFLOPS = 78.6  # dense FP64 matrix (v_mfma_f64_16x16x4f64), the same rate as the vector FMA
FP32_MFMA_PEAK_TFLOPS = 157.3  # dense FP32 matrix (v_mfma_f32_16x16x4f32: G2P with an FP32 grid)
# algorithmic cost of one (target, source) pair inside r_c (documented in the design notes):
# 39 add/mul (FMA = 2) of the G^N f formula + 7 per special function (rsqrt, exp, erfc).
# Counted per ordered pair, whatever the kernel executes (the symmetric kernel evaluates the
# shared coefficients once per unordered pair).
P2P_FLOPS_PER_PAIR = 60.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "c2_fp64_p2p_traffic.json")
P2P_SOURCES = ("p2p.hip", "internal.h", "screening.h")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def p2p_pairs_uniform(n, box, r_c):
    """Expected number of ordered pairs within r_c for n uniform points (periodic)."""
    V = box[0] * box[1] * box[2]
    return n * (n - 1) / V * (4.0 / 3.0) * math.pi * r_c**3


def stage_roofline(stages, n, ncell, P, real, pairs, alu_peak_tflops):
    """Per-stage algorithmic work (see the design notes), achieved rate and fraction of the binding roof.

    sort: bytes N (24 + 48 + 64 + 16) + 12 per cell; P2P: 60 flop per pair in r_c; P2G and G2P: 7 flop per
    (particle, stencil point), bytes 64 per record + one pass over the 3-component grid (+ 72 per particle
    written/gathered by G2P; G2P runs on the FP64 matrix cores, or the FP32 ones with an FP32 grid,
    priced against that peak);
    FFT+CNV+IFFT: five passes, each reading and writing the 3-component grid.
    """
    out = {}

    def put(name, ms, flops=None, nbytes=None, bound="hbm"):
        if ms <= 0:
            return
        e = {"ms": ms}
        if flops is not None:
            e["TFLOPs"] = flops / (ms * 1e-3) / 1e12
        if nbytes is not None:
            e["GBs"] = nbytes / (ms * 1e-3) / 1e9
        e["bound"] = bound
        if bound == "alu":
            e["frac"] = e["TFLOPs"] / alu_peak_tflops
        elif bound == "mfma":  # FP32 matrix instructions with an FP32 grid, else FP64
            e["frac"] = e["TFLOPs"] / (FP32_MFMA_PEAK_TFLOPS if real == 4 else FP64_MFMA_PEAK_TFLOPS)
        else:
            e["frac"] = e["GBs"] / HBM_PEAK_GBS
        out[name] = e

    grid_bytes = 3 * ncell * real
    put("sort", stages["sort"], nbytes=n * (24 + 48 + 64 + 16) + 12 * ncell)
    if pairs:
        put("p2p", stages["p2p"], flops=pairs * P2P_FLOPS_PER_PAIR, bound="alu")
    put("p2g", stages["p2g"], flops=7.0 * n * P**3, nbytes=64 * n + grid_bytes, bound="alu")
    put("fgc", stages["fgc"], nbytes=5 * 2 * grid_bytes)
    put("g2p", stages["g2p"], flops=7.0 * n * P**3, nbytes=grid_bytes + (64 + 72) * n, bound="mfma")
    return out


def kernel_source_hash():
    """SHA-256 of the P2P kernel's sources with comments and blank space removed (a change of
    comments alone leaves the counters valid)."""
    import hashlib
    import re

    h = hashlib.sha256()
    for name in P2P_SOURCES:
        with open(os.path.join(ROOT, "paper_2606_19059_amd", "csrc", name)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE runs, scaled by a plain copy's readings), or None when the summary is absent,
    names another kernel, or was taken from different kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel") != kernel or t.get("source_sha256") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def timed_evals(plan, x, f, steps, warmup):
    """Median device ms of `steps` evaluations (stage timers of the plan)."""
    import torch

    ws = plan.workspace(x.shape[1], x.device)
    u = torch.empty_like(x)
    for _ in range(warmup):
        plan.eval(x, f, out=u, workspace=ws)
    torch.cuda.synchronize()
    tot = []
    for _ in range(steps):
        plan.eval(x, f, out=u, workspace=ws)
        torch.cuda.synchronize()
        tot.append(plan.stage_ms()["total"])
    return float(np.median(tot)), u


def config_leg(E, name, steps, warmup, n_targets, dev):
    """One benchmark configuration, timed as the main workload: median device ms of `steps`
    evaluations, per-stage times and rooflines (P2P priced on the exact pair count), the
    sampled error against the classical oracle, and for FP32 bulk the whole-N error against
    the FP64 GPU path at a tighter tolerance on the same grid."""
    import torch

    import oracle
    from paper_2606_19059_amd import workloads as W

    wl = W.WORKLOADS[name]
    x_np, f_np = wl.make()
    x = torch.from_numpy(x_np).to(dev)
    f = torch.from_numpy(f_np).to(dev)
    plan = E.Plan(wl.box, wl.tol, grid=wl.grid, precision=wl.precision, n_max=wl.n, timers=True)
    info = plan.info
    ws = plan.workspace(wl.n, dev)
    u = torch.empty_like(x)
    for _ in range(warmup):
        plan.eval(x, f, out=u, workspace=ws)
    torch.cuda.synchronize()
    acc = {k: 0.0 for k in E.STAGES}
    tot = []
    for _ in range(steps):
        plan.eval(x, f, out=u, workspace=ws)
        torch.cuda.synchronize()
        st = plan.stage_ms()
        tot.append(st["total"])
        for k in st:
            acc[k] += st[k] / steps
    ms = float(np.median(tot))
    pairs = plan.count_pairs(x, f, workspace=ws)
    real = 8 if wl.precision == "fp64" else 4
    ncell = info["grid"][0] * info["grid"][1] * info["grid"][2]
    peak = FP64_VECTOR_TFLOPS if wl.precision == "fp64" else FP32_VECTOR_TFLOPS
    out = {
        "workload": "%s: N=%d %s in box %s, tol %g, grid %s, P=%d (Gaussian, derived from tol), %s"
                    % (wl.name, wl.n, wl.dist, "x".join("%g" % b for b in wl.box), wl.tol,
                       "x".join(str(m) for m in info["grid"]), info["P"], wl.precision),
        "ms_median": ms, "particles_per_s": wl.n / (ms * 1e-3), "stage_ms": acc,
        "ordered_pairs_in_rc": pairs, "xi": info["xi"], "r_c": info["r_c"], "P": info["P"],
        "stage_roofline": stage_roofline(acc, wl.n, ncell, info["P"], real, pairs, peak),
    }
    u_np = u.cpu().numpy()
    if n_targets >= wl.n:
        ref = oracle.ewald_sum(x_np, f_np, wl.box)
        out["rel_err_oracle"] = oracle.rel_err(u_np, ref)
        out["oracle_targets"] = "all %d" % wl.n
    else:
        tgt = W.sample_targets(wl.n, n_targets, seed=100 + int(name[1:]))
        out["rel_err_oracle"] = oracle.rel_err(u_np[:, tgt], oracle.ewald_sum(x_np, f_np, wl.box, targets=tgt))
        out["oracle_targets"] = "%d seeded" % n_targets
    if wl.precision == "fp32":
        p64 = E.Plan(wl.box, min(wl.tol, 1e-8), grid=wl.grid, precision="fp64", n_max=wl.n)
        u64 = p64.eval(x, f)
        out["rel_err_vs_fp64_path_all_n"] = float((torch.linalg.norm(u - u64) / torch.linalg.norm(u64)).item())
        del p64, u64
    del plan, ws, u, x, f
    torch.cuda.empty_cache()
    return out


def serving_leg(n_requests):
    """Stream of independent suspensions (N log-uniform in [1e3, 1e6], cubic or 1x1x2 box,
    uniform or blobs, tol in {1e-4, 1e-6, 1e-8}), served from one device arena: saturated
    throughput with every request waiting at t = 0 on 4 slots and on 1 slot (the device
    clock's concurrency of the evaluations beside it), then Poisson arrivals at 0.5, 0.8 and
    0.95 of the 4-slot rate for p50/p99 latency, and once more at 0.8 under an 8 GiB budget
    (admission waits for memory)."""
    import torch

    from paper_2606_19059_amd import serve
    from paper_2606_19059_amd import workloads as W

    jobs = serve.make_jobs(W.serving_stream(n_requests, rate_per_s=0.0, seed=5))

    def reset(arrivals):
        for j, a in zip(jobs, arrivals):
            j.arrival = float(a)
            j.admitted = j.done = float("nan")
            j.slot = -1
            j.bypassed = 0

    def poisson(rate, seed):
        return np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, len(jobs)))

    def keep(r):
        return {k: r[k] for k in ("p50_ms", "p99_ms", "particles_per_s", "concurrency", "small_p50_ms") if k in r}

    srv = serve.Server(n_slots=4, hbm_budget=32 << 30)
    srv.run(jobs[: min(8, len(jobs))])  # plans and tables become resident
    torch.cuda.synchronize()
    reset(np.zeros(len(jobs)))
    sat = serve.summarize(srv.run(jobs))
    rate = sat["requests"] / sat["wall_s"]
    one = serve.Server(n_slots=1, hbm_budget=32 << 30)
    one.plans = srv.plans
    reset(np.zeros(len(jobs)))
    sat1 = serve.summarize(one.run(jobs))
    del one
    loads = {}
    for k, frac in enumerate((0.5, 0.8, 0.95)):
        reset(poisson(frac * rate, 50 + k))
        loads["%.2f" % frac] = keep(serve.summarize(srv.run(jobs)))
    # small requests only (N log-uniform in [1e3, 1e4]), all waiting: evaluated one by one on the
    # 4 streams, and grouped by plan into batched evaluations (ewald_eval_batch)
    sjobs = serve.make_jobs(W.serving_stream(256, rate_per_s=0.0, seed=7, n_lo=1e3, n_hi=1e4))
    small_rates = {}
    for batching in (False, True):
        sv = serve.Server(n_slots=4, hbm_budget=8 << 30, batching=batching)
        sv.plans = srv.plans
        sv.run(sjobs[:8])
        for j in sjobs:
            j.arrival, j.admitted, j.done, j.slot, j.bypassed = 0.0, float("nan"), float("nan"), -1, 0
        r = serve.summarize(sv.run(sjobs))
        small_rates["batched" if batching else "one_by_one"] = {
            "particles_per_s": r["particles_per_s"], "p50_ms": r["p50_ms"], "evaluations": sv.batches,
            "requests": r["requests"]}
        del sv
    del srv
    torch.cuda.empty_cache()
    small = serve.Server(n_slots=4, hbm_budget=8 << 30)
    reset(poisson(0.8 * rate, 60))
    r = serve.summarize(small.run(jobs))
    budget = dict(keep(r), budget_bytes=8 << 30, offered_load=0.8, max_in_flight_bytes=small.max_in_flight_bytes,
                  admissions_waiting_for_memory=small.memory_waits, bypasses=small.bypasses)
    return {
        "workload": "c5: %d requests, N log-uniform [1e3, 1e6], boxes 1^3 or 1x1x2, uniform or blobs, "
                    "tol in {1e-4, 1e-6, 1e-8} (FP32 bulk for tol >= 1e-6, FP64 below), inputs and results "
                    "in pinned host memory (copies included), one device arena, 4 streams" % n_requests,
        "saturated_particles_per_s": sat["particles_per_s"],
        "saturated_device_concurrency": sat["concurrency"],
        "saturated_1_slot_particles_per_s": sat1["particles_per_s"],
        "offered_load": 0.8,
        "p50_ms": loads["0.80"]["p50_ms"],
        "p99_ms": loads["0.80"]["p99_ms"],
        "particles_per_s": loads["0.80"]["particles_per_s"],
        "by_offered_load": loads,
        "hbm_budget_8GiB": budget,
        "small_requests_saturated": dict(small_rates, workload="256 requests, N log-uniform [1e3, 1e4], "
                                         "boxes 1^3 or 1x1x2, tol in {1e-4, 1e-6, 1e-8}, all waiting at t = 0"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--P", type=int, default=0, help="window support (0: derive from tol)")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="host time budget of the oracle sample (accuracy + CPU baseline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-plans", action="store_true",
                    help="skip the cost-model plan and Kaiser-Bessel legs")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests in the serving leg (Poisson stream of independent suspensions; 0: skip)")
    ap.add_argument("--entry", default="eval", choices=("eval", "overlap"),
                    help="entry point timed: ewald_eval, or ewald_eval_overlap (P2P on a second stream)")
    ap.add_argument("--compare-entries", action="store_true",
                    help="also time the other entry point (eval / overlap) on the same inputs")
    ap.add_argument("--configs", default="c1,c3,c4",
                    help="other benchmark configurations timed beside the main one (comma list; '' for none)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the evaluation is not sharded across "
              "GPUs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2606_19059_amd as E
    from paper_2606_19059_amd import workloads as W

    if args.copy_calibration_mib > 0:
        nb = args.copy_calibration_mib << 20
        src = torch.empty(nb, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: %d bytes read, %d bytes written by one copy kernel" % (nb, nb))
        del src, dst

    wl = W.WORKLOADS[args.config]
    precision = args.precision or wl.precision
    x_np, f_np = wl.make()
    dev = torch.device("cuda:0")
    x = torch.from_numpy(x_np).to(dev)
    f = torch.from_numpy(f_np).to(dev)
    plan = E.Plan(wl.box, wl.tol, grid=wl.grid, P=args.P or None, precision=precision, n_max=wl.n,
                  timers=True)
    info = plan.info
    log("plan:", json.dumps({k: info[k] for k in ("xi", "r_c", "grid", "P", "window_shape", "tile",
                                                   "stencil", "workspace_bytes")}))
    ws = plan.workspace(wl.n, dev)
    u = torch.empty_like(x)
    side = torch.cuda.Stream(device=dev)  # the near field's stream for the overlapped entry point

    def step(entry):
        if entry == "overlap":
            plan.eval_overlap(x, f, out=u, workspace=ws, near_stream=side)
        else:
            plan.eval(x, f, out=u, workspace=ws)

    for _ in range(args.warmup):
        step(args.entry)
    torch.cuda.synchronize()
    log("warmup done")

    stage_sum = {k: 0.0 for k in E.STAGES}
    step_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        step(args.entry)
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - ts) * 1e3)
        st = plan.stage_ms()
        for k in st:
            stage_sum[k] += st[k]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    stages = {k: v / args.steps for k, v in stage_sum.items()}
    log("stages (ms):", json.dumps({k: round(v, 4) for k, v in stages.items()}))
    # the other entry point on the same inputs (same results; P2P on one or two streams)
    other = "eval" if args.entry == "overlap" else "overlap"
    other_ms = None
    if args.compare_entries:
        for _ in range(2):
            step(other)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            step(other)
        torch.cuda.synchronize()
        other_ms = (time.perf_counter() - t1) * 1e3 / args.steps
        log("%s entry point: %.3f ms per step" % (other, other_ms))
        step(args.entry)
        torch.cuda.synchronize()

    # accuracy on sampled targets against the classical FP64 oracle (also the CPU baseline)
    rel_err = None
    cpu = None
    if args.cpu_seconds > 0 and not args.no_cpu_baseline:
        import oracle

        # a 64-target probe sizes the timed sample to at most about --cpu-seconds of host
        # work (its fixed cost, the structure factors over all sources, is charged per target)
        u_np = u.cpu().numpy()
        tc = time.perf_counter()
        oracle.ewald_sum(x_np, f_np, wl.box, targets=W.sample_targets(wl.n, 64, seed=100 + 2))
        probe_s = time.perf_counter() - tc
        n_tgt = int(max(64, min(4096, 64 * args.cpu_seconds / max(probe_s, 1e-3))))
        tgt = W.sample_targets(wl.n, n_tgt, seed=100 + 2)
        tc = time.perf_counter()
        ref = oracle.ewald_sum(x_np, f_np, wl.box, targets=tgt)
        cpu_s = time.perf_counter() - tc
        rel_err = oracle.rel_err(u_np[:, tgt], ref)
        cpu = {
            "value": len(tgt) / cpu_s,
            "unit": "particles/s",
            "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d seeded targets of the same N=%d evaluation (all sources; classical Ewald, "
                      "structure factor included), %.1f s" % (len(tgt), wl.n, cpu_s),
        }
        log("sampled rel err vs oracle: %.3e (tol %g); oracle %.2f s" % (rel_err, wl.tol, cpu_s))
        # the same oracle on one host core, on a smaller sample of the same targets
        threads = oracle.num_threads()
        n1 = int(max(8, min(len(tgt), len(tgt) * 0.4 / max(threads, 1))))
        oracle.set_num_threads(1)
        try:
            tc = time.perf_counter()
            oracle.ewald_sum(x_np, f_np, wl.box, targets=tgt[:n1])
            one_s = time.perf_counter() - tc
        finally:
            oracle.set_num_threads(threads)
        cpu["value_1core"] = n1 / one_s
        cpu["sample_1core"] = "%d of the same targets on 1 thread, %.1f s" % (n1, one_s)
        log("oracle on 1 core: %.2f particles/s" % cpu["value_1core"])

    # roofline of the dominant kernel (P2P): algorithmic flops per launch / its mean time,
    # on the exact number of ordered pairs inside r_c (the library's count-only pass)
    pairs = plan.count_pairs(x, f, workspace=ws)
    log("ordered pairs in r_c: %d (uniform expectation %.4g)" % (pairs, p2p_pairs_uniform(wl.n, wl.box, info["r_c"])))
    p2p_s = stages["p2p"] * 1e-3
    peak = FP64_VECTOR_TFLOPS if precision == "fp64" else FP32_VECTOR_TFLOPS
    achieved = (pairs * P2P_FLOPS_PER_PAIR / p2p_s / 1e12) if pairs else None
    # the symmetric kernel's instance: FP64 at the pair formula's accuracy level for this tol
    # (2: tol >= 1e-8, 1: tol >= 1e-10, 0: full), or the FP32 formula
    level = 2 if wl.tol >= 1e-8 else 1 if wl.tol >= 1e-10 else 0
    kernel = ("k_p2p_sym<double, %d, false>" % level) if precision == "fp64" else "k_p2p_sym<float, 0, false>"
    roofline = {
        "kernel": kernel,
        "bound": "alu",
        "achieved": achieved,
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": (achieved / peak) if achieved else None,
        "traffic": measured_traffic(kernel) if (wl.name == "c2" and precision == "fp64") else None,
        "per_unit": "%g flop per (target, source) pair inside r_c; %.4g ordered pairs per launch"
                    % (P2P_FLOPS_PER_PAIR, pairs or 0),
    }
    # the same N and tolerance with the plan the cost model picks from the tolerance alone,
    # and with the Kaiser-Bessel window on the configured grid
    legs = {}
    if not args.no_extra_plans:
        auto = E.Plan(wl.box, wl.tol, precision=precision, n_max=wl.n, timers=True)
        ms_auto, _ = timed_evals(auto, x, f, 5, 2)
        legs["model_plan"] = {"grid": list(auto.info["grid"]), "P": auto.info["P"], "r_c": auto.info["r_c"],
                              "predicted_ms": auto.info["predicted_ms"], "measured_ms": ms_auto,
                              "particles_per_s": wl.n / (ms_auto * 1e-3)}
        del auto
        kbp = E.Plan(wl.box, wl.tol, grid=wl.grid, precision=precision, n_max=wl.n, timers=True, window="kb")
        ms_kb, u_kb = timed_evals(kbp, x, f, 5, 2)
        legs["kb_window"] = {"grid": list(kbp.info["grid"]), "P": kbp.info["P"], "measured_ms": ms_kb,
                             "stage_ms": kbp.stage_ms(),
                             "particles_per_s": wl.n / (ms_kb * 1e-3),
                             "rel_err_vs_gaussian_window_result": float(
                                 (torch.linalg.norm(u_kb - u) / torch.linalg.norm(u)).item())}
        del kbp, u_kb
        # combined single and double layer sources (the paper's benchmark workload): the same
        # particles with stresslet vectors q, n ~ N(0, 1) per component
        rng = np.random.default_rng(wl.seed + 500)
        qd = torch.from_numpy(rng.standard_normal((3, wl.n))).to(dev)
        nd = torch.from_numpy(rng.standard_normal((3, wl.n))).to(dev)
        stp = E.Plan(wl.box, wl.tol, grid=wl.grid, precision=precision, n_max=wl.n, timers=True, stresslet=True)
        ws_st = stp.workspace(wl.n, dev)
        u_st = torch.empty_like(x)
        for _ in range(2):
            stp.eval_combined(x, f, qd, nd, out=u_st, workspace=ws_st)
        torch.cuda.synchronize()
        st_ms = {k: 0.0 for k in E.STAGES}
        for _ in range(5):
            stp.eval_combined(x, f, qd, nd, out=u_st, workspace=ws_st)
            torch.cuda.synchronize()
            for k, v in stp.stage_ms().items():
                st_ms[k] += v / 5
        legs["combined_stresslet"] = {"grid": list(stp.info["grid"]), "P": stp.info["P"], "stage_ms": st_ms,
                                      "particles_per_s": wl.n / (st_ms["total"] * 1e-3)}
        del stp, ws_st, u_st, qd, nd
        # the 1e-6 headline: FP32 bulk against the plain FP64 path at equal accuracy, on the H
        # particles (1e6 uniform, 128^3), errors against an FP64 evaluation at tol 1e-8
        hw = W.WORKLOADS["H"]
        hx, hf = hw.make()
        hX, hF = torch.from_numpy(hx).to(dev), torch.from_numpy(hf).to(dev)
        ref = E.Plan(hw.box, 1e-8, n_max=hw.n, precision="fp64").eval(hX, hF)
        head = {}
        for prec in ("fp32", "fp64"):
            hp = E.Plan(hw.box, hw.tol, grid=hw.grid, precision=prec, n_max=hw.n, timers=True)
            ms_h, u_h = timed_evals(hp, hX, hF, 5, 2)
            head[prec] = {"grid": list(hp.info["grid"]), "P": hp.info["P"], "measured_ms": ms_h,
                          "particles_per_s": hw.n / (ms_h * 1e-3),
                          "rel_err_vs_fp64_1e-8": float((torch.linalg.norm(u_h - ref) / torch.linalg.norm(ref)).item())}
            del hp, u_h
        legs["H_1e-6_fp32_vs_fp64"] = head
        del hX, hF, ref
        log("extra plans:", json.dumps(legs))
    # P2G GB/s: algorithmic bytes = particle reads (6 reals) + one write of the 3-component grid
    real = 8 if precision == "fp64" else 4
    ncell = info["grid"][0] * info["grid"][1] * info["grid"][2]
    p2g_bytes = wl.n * 6 * real + 3 * ncell * real
    p2g_gbs = p2g_bytes / (stages["p2g"] * 1e-3) / 1e9 if stages["p2g"] > 0 else None
    per_stage = stage_roofline(stages, wl.n, ncell, info["P"], real, pairs, peak)
    configs = {}
    for name in [c for c in args.configs.split(",") if c and c != wl.name]:
        cw = W.WORKLOADS[name]
        n_t = cw.n if cw.n <= 1000 else (64 if cw.n <= 4_000_000 else 48)
        configs[name] = config_leg(E, name, 20 if cw.n <= 1000 else 10, 3 if cw.n <= 1000 else 2, n_t, dev)
        log("config %s:" % name, json.dumps(configs[name]))
    serving = None
    if args.serve_requests > 0:
        serving = serving_leg(args.serve_requests)
        log("serving:", json.dumps(serving))
    s_ms = sorted(step_ms)
    p50 = s_ms[len(s_ms) // 2]
    p99 = s_ms[min(len(s_ms) - 1, int(math.ceil(0.99 * len(s_ms))) - 1)]

    out = {
        "metric": METRIC,
        "value": wl.n / (ms_per_step * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": "%s: N=%d %s in box %s, forces N(0,1) mean-removed, tol %g, grid %s, window P=%d "
                        "(Gaussian), %s" % (wl.name, wl.n, wl.dist, "x".join("%g" % b for b in wl.box), wl.tol,
                                             "x".join(str(m) for m in info["grid"]), info["P"], precision),
            "n": wl.n, "tol": wl.tol, "grid": list(info["grid"]), "P": info["P"], "xi": info["xi"],
            "r_c": info["r_c"], "rel_err_sampled": rel_err, "stage_ms": stages,
            "p2g_GBs": p2g_gbs, "p50_ms": p50, "p99_ms": p99, "stage_roofline": per_stage,
            "entry_point": "ewald_eval_overlap" if args.entry == "overlap" else "ewald_eval",
            "other_entry_point_ms_per_step": ({("ewald_eval_overlap" if other == "overlap" else "ewald_eval"): other_ms}
                                              if other_ms is not None else None),
        },
        "serving": serving,
        "configs": configs,
        "other_plans": legs,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
