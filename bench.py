#!/usr/bin/env python3
"""Throughput of the L-tsNET gradient iteration on one MI355X.

One step = one full evaluation of the gradient (grid plan, binning, spread,
FFT convolution, gather, Z, attraction + assembly) followed by the vertex
move, on a Barabasi-Albert graph with n = 1,000,000 and m0 = 4 (seed 3),
perplexity 40 (k = 120), layout initialised N(0, 1e-4) (seed 0). P is built
once on the GPU before timing. The timed region holds exactly --steps steps
between two device synchronisations, inputs resident in HBM.

Prints one JSON line on stdout; progress goes to stderr.
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

METRIC = "tsNET gradient iters/sec and ns/vertex-iter at n=1M, FP32-interp vs FP64 direct"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# --------------------------------------------------------------------------- CPU baseline
_CPU_X = None


def _cpu_worker(rows):
    from oracle import gradient
    t0 = time.perf_counter()
    gradient.pair_sums(_CPU_X, 0.05, rows=np.asarray(rows))
    return time.perf_counter() - t0


def cpu_baseline(X: np.ndarray, budget_s: float = 12.0):
    """The FP64 oracle's exact O(n^2) pair sums on a bounded row sample, all worker
    processes in parallel; extrapolated to one full iteration (n(n-1) pairs)."""
    import multiprocessing as mp
    from oracle import gradient
    global _CPU_X
    _CPU_X = X.astype(np.float64)
    n = X.shape[0]
    cores = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    gradient.pair_sums(_CPU_X, 0.05, rows=np.arange(4))
    per_row = (time.perf_counter() - t0) / 4
    rows_per_worker = max(4, int(budget_s / max(per_row, 1e-6)))
    rng = np.random.default_rng(3)
    sample = rng.choice(n, size=min(n, rows_per_worker * cores), replace=False)
    chunks = np.array_split(sample, cores)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        pool.map(_cpu_worker, chunks)
    wall = time.perf_counter() - t0
    pairs = sample.shape[0] * (n - 1)
    pairs_per_s = pairs / wall
    iter_s = n * (n - 1) / pairs_per_s
    return {
        "value": 1.0 / iter_s,
        "unit": "iters/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"exact FP64 pair sums (Z_i, F_rep, F_ent) of {sample.shape[0]} random rows of "
                   f"the n={n} layout in {cores} processes, {wall:.1f} s wall; one iteration "
                   f"extrapolated as n(n-1) pairs at the measured {pairs_per_s:.3e} pairs/s"),
    }


# --------------------------------------------------------------------------- GPU
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--direct-iters", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--max-intervals", type=int, default=512)
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="iterations per captured HIP graph in the timed region (0: plain launches; "
                         "graph replays measured slower than plain launches on ROCm 7, and event "
                         "times read from graph nodes are not usable)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run 5 device copies of 1 GiB (reference for the HBM traffic counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied 5 x 1 GiB")
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    from synth import graphs
    t0 = time.perf_counter()
    g = graphs.workload_ba1m(args.n)
    X0 = graphs.initial_layout(g.n, 0)
    log(f"graph: BA n={g.n} m={g.m} max deg {int(g.degrees().max())} ({time.perf_counter() - t0:.1f} s)")

    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        cpu = cpu_baseline(X0)
        log(f"cpu baseline: {cpu['value']:.3e} iters/s on {cpu['cores']} cores "
            f"({time.perf_counter() - t0:.1f} s)")

    import torch
    from paper_2509_19785_amd import api
    dev = torch.device("cuda", 0)
    ctx = api.Context(0)
    prm = api.Params(max_intervals=args.max_intervals)
    sp = api.StepParams()
    ip = torch.as_tensor(g.indptr).to(dev)
    ix = torch.as_tensor(g.indices).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob = api.Problem.build(ctx, ip, ix, 40.0, seed=3)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    log(f"build_P: nnz={prob.nnz} in {build_ms:.1f} ms")
    del ip, ix

    X = torch.tensor(X0, device=dev)
    upd = torch.zeros_like(X)
    gains = torch.ones_like(X)
    G = torch.empty_like(X)
    Z = torch.empty(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def one(it):
        prob.grad(X, prm, G=G, Z=Z, stream=stream)
        prob.step(X, upd, gains, G, it, sp, stream=stream)

    for it in range(args.warmup):
        one(it)
    torch.cuda.synchronize()
    log(f"warmup done, status {ctx.status():#x}")

    # timed region: events only around the dominant kernel
    K = args.graph_steps
    graphs_used = K > 0
    if graphs_used:
        # events for the graphs come from the context's pool: fill it with
        # gradient evaluations on a scratch copy (the trajectory is untouched)
        Xs, Gs, Zs = X.clone(), torch.empty_like(X), torch.empty_like(Z)
        ctx.set_timing(["attract_assemble"])
        for _ in range(2 * K + 2):
            prob.grad(Xs, prm, G=Gs, Z=Zs)
        torch.cuda.synchronize()
        ctx.stage_times()
        del Xs, Gs, Zs
        sw = sp.momentum_switch_iter
        g_early = api.StepGraph(prob, X, upd, gains, G, Z, prm, sp, 0, K)
        g_late = api.StepGraph(prob, X, upd, gains, G, Z, prm, sp, sw, K)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it = args.warmup
        end = args.warmup + args.steps
        while it < end:
            if it + K <= end and (it + K <= sw or it >= sw):
                (g_early if it < sw else g_late).replay()
                it += K
            else:  # a block that straddles the momentum switch or the end
                one(it)
                it += 1
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = ctx.stage_times()  # the events in the graphs hold their last replay
        ctx.set_timing(None)
        del g_early, g_late
    else:
        ctx.set_timing(["attract_assemble"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(args.warmup, args.warmup + args.steps):
            one(it)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = ctx.stage_times()
        ctx.set_timing(None)
    ms_per_step = wall / args.steps * 1e3
    iters_per_s = args.steps / wall
    attr_ms, attr_calls = st["attract_assemble"]
    attr_avg_s = attr_ms / max(attr_calls, 1) * 1e-3
    n, nnz = prob.n, prob.nnz
    attr_bytes = 8 * nnz + 8 * (n + 1) + 8 * n + 16 * n + 8 * n
    achieved = attr_bytes / attr_avg_s / 1e9
    log(f"timed ({'graphs of ' + str(K) if graphs_used else 'plain launches'}): {ms_per_step:.4f} ms/step, "
        f"{iters_per_s:.1f} iters/s; attract {attr_avg_s * 1e6:.1f} us over {attr_calls} launches "
        f"-> {achieved:.0f} GB/s")

    # stage breakdown (separate short run, every stage bracketed)
    ctx.set_timing("all")
    it0 = args.warmup + args.steps
    for it in range(it0, it0 + 20):
        one(it)
    torch.cuda.synchronize()
    stages = {k: v[0] / v[1] for k, v in ctx.stage_times().items() if v[1]}
    ctx.set_timing(None)
    gi = prob.grid_info()
    Xh = X.cpu().numpy()
    span = float((Xh.max(0) - Xh.min(0)).max())
    log("stages (ms/call): " + ", ".join(f"{k} {v:.4f}" for k, v in stages.items()))

    # FP64 direct all-pairs baseline on the same problem and layout
    direct = None
    if args.direct_iters > 0:
        X64 = X.double()
        prob.grad_direct_f64(X64, prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.direct_iters):
            Gd, Zd = prob.grad_direct_f64(X64, prm)
        torch.cuda.synchronize()
        dwall = (time.perf_counter() - t0) / args.direct_iters
        # accuracy of the FP32 interpolation gradient against it at this layout
        prob.grad(X, prm, G=G, Z=Z)
        torch.cuda.synchronize()
        err = float(torch.linalg.norm(G.double() - Gd) / torch.linalg.norm(Gd))
        pairs = float(n) * (n - 1)
        direct = {
            "iters_per_s": 1.0 / dwall,
            "ms_per_iter": dwall * 1e3,
            "pairs_per_s": pairs / dwall,
            "speedup_of_interp": iters_per_s * dwall,
            "rel_l2_interp_vs_direct": err,
            "Z_direct": float(Zd.item()),
            "Z_interp": float(Z.item()),
        }
        log(f"direct f64: {dwall * 1e3:.1f} ms/iter; interp speedup {iters_per_s * dwall:.1f}x; "
            f"rel L2 {err:.2e}")

    out = {
        "metric": METRIC,
        "value": iters_per_s,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ns_per_vertex_iter": ms_per_step * 1e6 / n,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "barabasi_albert_n1e6_m4_seed3",
            "n": n, "edges": int(g.m), "perplexity": 40.0, "k": prob.k, "nnz_P": nnz,
            "init": "N(0,1e-4) seed 0", "interval_width": prm.interval_width,
            "min_intervals": prm.min_intervals, "max_intervals": prm.max_intervals,
            "n_intervals_end": int(gi["n_intervals"][0]), "span_end": span,
            "launch": f"HIP graphs of {K} iterations" if graphs_used else "plain launches",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_attract (attract_assemble)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "algorithmic_bytes": attr_bytes,
            "avg_launch_us": attr_avg_s * 1e6,
            "launches_timed": attr_calls,
        },
        "cpu_baseline": cpu,
        "build_P_ms": build_ms,
        "stages_ms": stages,
        "direct_f64": direct,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
