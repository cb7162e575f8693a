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

# HBM bytes of one k_attract_tiled launch seen by the rocprofv3 counters
# (FETCH_SIZE x 2 + WRITE_SIZE x 1, KiB x 1024; the factors from a 1 GiB device
# copy), summarised under profiles/. They hold for the kernel source with the
# hash below only: for any other source the traffic is reported as null.
ATTRACT_TRAFFIC_BYTES = 1_824_396_638
ATTRACT_TRAFFIC_SOURCE_SHA256 = "35f8a3af941ac3538812a2266335c839df048d2bb97f11072ef6373272e006ba"


def attract_traffic():
    import hashlib
    src = os.path.join(ROOT, "paper_2509_19785_amd", "csrc", "tile.hip")
    try:
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    return ATTRACT_TRAFFIC_BYTES if sha == ATTRACT_TRAFFIC_SOURCE_SHA256 else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# --------------------------------------------------------------------------- CPU baseline
_CPU_X = None


def _cpu_worker(rows):
    from oracle import gradient
    t0 = time.perf_counter()
    gradient.pair_sums(_CPU_X, 0.05, rows=np.asarray(rows))
    return time.perf_counter() - t0


def host_cpu():
    """Model name and core counts of the host CPU (lscpu, else /proc/cpuinfo)."""
    import subprocess
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    if model is None:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": model, "cpus_visible": os.cpu_count(), "cpus_usable": usable}


# worker processes of the oracle timings: every usable core, at most the host's
# share per GPU of the machines this runs on (16)
HOST_SHARE = 16


def cpu_baseline(X: np.ndarray, budget_s: float = 12.0):
    """The FP64 oracle's exact O(n^2) pair sums on a bounded row sample, all worker
    processes in parallel; extrapolated to one full iteration (n(n-1) pairs)."""
    import multiprocessing as mp
    from oracle import gradient
    global _CPU_X
    _CPU_X = X.astype(np.float64)
    n = X.shape[0]
    host = host_cpu()
    cores = max(1, min(HOST_SHARE, host["cpus_usable"]))
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
        "cpu": host,
        "kind": "oracle",
        "sample": (f"exact FP64 pair sums (Z_i, F_rep, F_ent) of {sample.shape[0]} random rows of "
                   f"the n={n} layout in {cores} processes, {wall:.1f} s wall; one iteration "
                   f"extrapolated as n(n-1) pairs at the measured {pairs_per_s:.3e} pairs/s"),
    }


def pmds_cpu_baseline(g, pivots: int, sample: int = 3):
    """The oracle's Pivot MDS on the host: the max-min search over `sample` pivots
    timed and extrapolated to `pivots` (the BFS dominates its cost)."""
    from oracle import pmds as opmds
    A = opmds._csr(g.indptr, g.indices)
    t0 = time.perf_counter()
    opmds.select_pivots(A, 0, g.n, sample, opmds.first_pivot(0, 0, g.n, 3))
    per = (time.perf_counter() - t0) / sample
    return {"ms": per * pivots * 1e3, "cores": 1, "kind": "oracle",
            "sample": f"{sample} of the {pivots} max-min BFS searches (scipy, one core), "
                      f"extrapolated; the eigen-solve and projection are not counted"}


def small_n_oracle(g, iters: int = 20):
    """The oracle's exact FP64 gradient + step on the 32 x 32 grid (P from k = 120),
    timed over `iters` iterations on one host core."""
    from oracle import affinities, gradient, step as ostep
    from synth import graphs
    P = affinities.build_P(g.indptr, g.indices, 40.0, seed=0)
    X = graphs.initial_layout(g.n, 0).astype(np.float64)
    U, Ga = np.zeros_like(X), np.ones_like(X)
    t0 = time.perf_counter()
    for it in range(iters):
        G = gradient.grad_terms(X, P).G
        X, U, Ga = ostep.step(X, U, Ga, G, it)
    dt = time.perf_counter() - t0
    return {"iters_per_s": iters / dt, "cores": 1, "kind": "oracle",
            "sample": f"{iters} iterations of the exact FP64 gradient and step (n = {g.n}, k = 120)"}


def small_n_leg(api, ctx, iters: int, cpu: bool = True):
    """The 32 x 32 grid (n = 1024): L-tsNET (P from k = 120) against the original
    tsNET's full P (k = n - 1), both from the same Pivot MDS start with the
    two-stage schedule, then the quality of each final layout (NP of every
    vertex, stress over every source) and the FP64 direct gradient's rate."""
    import torch
    from synth import graphs
    g = graphs.workload_grid32()
    start = api.pmds(ctx, g.indptr, g.indices, pivots=50, seed=0)["X"]
    sched = api.staged_schedule(iters)
    res = {"workload": "grid 32 x 32, perplexity 40, Pivot MDS start, "
                       f"{iters} iterations ({sched[0][0]} + {sched[1][0]})"}
    for name, k in (("L-tsNET k=120", 120), ("tsNET full P k=1023", g.n - 1)):
        prob = api.Problem.build(ctx, g.indptr, g.indices, 40.0, k=k, seed=0)
        X = start.clone()
        U, Ga, G = torch.zeros_like(X), torch.ones_like(X), torch.empty_like(X)
        prob.run(X, U, Ga, G, [(1, sched[0][1])])          # first evaluation sizes the workspace
        X.copy_(start)
        U.zero_()
        Ga.fill_(1.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob.run(X, U, Ga, G, sched)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        q = api.neighbourhood_preservation(ctx, g.indptr, g.indices, X)
        st = api.stress(ctx, g.indptr, g.indices, X, np.arange(g.n, dtype=np.int32))
        entry = {"nnz_P": prob.nnz, "iters_per_s": iters / wall, "np": float(q["np"][0]),
                 "stress": float(st["stress"][0]), "stress_best_scale": float(st["stress_best_scale"][0])}
        # the same schedule replayed from HIP graphs, one per stage (gk iterations
        # recorded once, at the stage's iteration numbers): launch overhead removed,
        # the layout equal to the eager run's bit for bit
        gk = 10
        if all(n_it % gk == 0 for n_it, _ in sched):
            X_eager = X.clone()
            Zb = torch.empty(1, dtype=torch.float64, device=X.device)
            sp, first, graphs_ = api.StepParams(), 0, []
            for n_it, prm in sched:
                graphs_.append(api.StepGraph(prob, X, U, Ga, G, Zb, prm, sp, first, gk))
                first += n_it
            X.copy_(start)
            U.zero_()
            Ga.fill_(1.0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for (n_it, _), gr in zip(sched, graphs_):
                for _ in range(n_it // gk):
                    gr.replay()
            torch.cuda.synchronize()
            entry["graph_replay"] = {"iters_per_s": iters / (time.perf_counter() - t0),
                                     "iters_per_graph": gk,
                                     "equals_eager": bool(torch.equal(X, X_eager))}
            del graphs_
        if k == g.n - 1:
            X64 = X.double()
            prob.grad_direct_f64(X64)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(20):
                prob.grad_direct_f64(X64)
            torch.cuda.synchronize()
            entry["direct_f64_grads_per_s"] = 20 / (time.perf_counter() - t0)
        res[name] = entry
        if cpu and k == 120:
            entry["cpu_oracle"] = small_n_oracle(g)
        gr = entry.get("graph_replay")
        log(f"small n, {name}: {entry['iters_per_s']:.0f} iters/s" +
            (f" ({gr['iters_per_s']:.0f} by graph replay, equal: {gr['equals_eager']})" if gr else "") +
            f", NP {entry['np']:.4f}, stress {entry['stress']:.4f} "
            f"(best scale {entry['stress_best_scale']:.4f})")
        prob.free()
    return res


def c1_leg(api, ctx, iters: int):
    """The 32 x 32 grid from N(0, 1e-4) (seed 0), perplexity 40 (k = 120),
    lambda_c 1.2, lambda_r 0.01, eps 0.05: `iters` iterations with the exact
    FP64 all-pairs gradient (cast to FP32 for the vertex move), and the same
    run with the FP32 interpolation gradient; rates and the quality of both
    final layouts (NP of every vertex, stress over every source)."""
    import torch
    from synth import graphs
    g = graphs.workload_grid32()
    prob = api.Problem.build(ctx, g.indptr, g.indices, 40.0, seed=0)
    prm, sp = api.Params(), api.StepParams()
    X0 = torch.tensor(graphs.initial_layout(g.n, 0), device="cuda")
    out = {"workload": f"grid 32 x 32, N(0, 1e-4) seed 0, perplexity 40, {iters} iterations, "
                       "lambda_c 1.2, lambda_r 0.01, eps 0.05"}
    for name in ("exact FP64 gradient", "FP32 interpolation gradient"):
        X = X0.clone()
        U, Ga, G = torch.zeros_like(X), torch.ones_like(X), torch.empty_like(X)
        exact = name.startswith("exact")

        def one(it):
            if exact:
                Gd, _ = prob.grad_direct_f64(X.double(), prm)
                G.copy_(Gd)
            else:
                prob.grad(X, prm, G=G)
            prob.step(X, U, Ga, G, it, sp)
        one(0)  # the first evaluation sizes the workspace
        X.copy_(X0)
        U.zero_()
        Ga.fill_(1.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(iters):
            one(it)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        q = api.neighbourhood_preservation(ctx, g.indptr, g.indices, X)
        st = api.stress(ctx, g.indptr, g.indices, X, np.arange(g.n, dtype=np.int32))
        out[name] = {"iters_per_s": iters / wall, "np": float(q["np"][0]),
                     "stress": float(st["stress"][0]),
                     "stress_best_scale": float(st["stress_best_scale"][0]),
                     "span": float((X.max(0).values - X.min(0).values).max())}
        log(f"C1 {name}: {iters / wall:.0f} iters/s, NP {out[name]['np']:.4f}, stress "
            f"{out[name]['stress']:.4f} (best scale {out[name]['stress_best_scale']:.4f})")
    prob.free()
    return out


def metrics_cpu_baseline(g, X, np_sample: int = 16, stress_sample: int = 2, sources: int = 64):
    """The oracle's metrics on the host: neighbourhood preservation of `np_sample`
    vertices extrapolated to all n, stress of `stress_sample` sources extrapolated
    to `sources`."""
    from oracle import metrics as om
    rng = np.random.default_rng(5)
    verts = np.sort(rng.choice(g.n, np_sample, replace=False))
    t0 = time.perf_counter()
    om.neighbourhood_preservation(g.indptr, g.indices, X, vertices=verts)
    np_per = (time.perf_counter() - t0) / np_sample
    t0 = time.perf_counter()
    om.stress_sums(g.indptr, g.indices, X, rng.choice(g.n, stress_sample, replace=False))
    st_per = (time.perf_counter() - t0) / stress_sample
    return {"np_ms": np_per * g.n * 1e3, "stress_ms": st_per * sources * 1e3, "cores": 1,
            "kind": "oracle",
            "sample": f"NP of {np_sample} vertices extrapolated to all {g.n}; stress of "
                      f"{stress_sample} sources (scipy BFS, one core) extrapolated to {sources}"}


# --------------------------------------------------------------------------- descent legs
def descent_leg(api, ctx, prob, X0d, iters, prm, sp, block=100, direct_rows=4096, seed=0):
    """`iters` steps of (gradient + step) from X0d between two device
    synchronisations, HIP events every `block` steps; then the status word of
    the timed steps, the grid of every step (an untimed replay: reading it
    synchronises), and the FP32 gradient at the final layout against the FP64
    direct kernel on sampled rows (per graph for a batch)."""
    import torch
    n, Gn = prob.n, prob.num_graphs
    X = X0d.clone()
    upd, gains = torch.zeros_like(X), torch.ones_like(X)
    G = torch.empty_like(X)
    Z = torch.empty(Gn, dtype=torch.float64, device=X.device)
    stream = torch.cuda.current_stream()
    prob.grad(X, prm, G=G, Z=Z, stream=stream)   # the first evaluation sizes the workspace
    torch.cuda.synchronize()
    ctx.status()
    nb = iters // block
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(nb + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for it in range(iters):
        prob.grad(X, prm, G=G, Z=Z, stream=stream)
        prob.step(X, upd, gains, G, it, sp, stream=stream)
        if (it + 1) % block == 0:
            evs[(it + 1) // block].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    status = ctx.status()
    rates = [block / (evs[k].elapsed_time(evs[k + 1]) * 1e-3) for k in range(nb)]
    # accuracy at the final layout, against the FP64 direct kernel on sampled rows;
    # per graph the relative L2 error of G and, since G of a converged layout is
    # a small difference of large terms, the error against the size of its terms
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(n, min(direct_rows, n), replace=False)).astype(np.int32)
    prob.grad(X, prm, G=G, Z=Z)
    Gd, Zd, Td = prob.grad_direct_f64(X.double(), prm, rows=rows, with_terms=True)
    torch.cuda.synchronize()
    rt = torch.as_tensor(rows, device=X.device).long()
    Gs, Xs = G[rt].double(), X[rt].double()
    goff = np.asarray(prob_offsets(prob))
    gid = np.searchsorted(goff, rows, side="right") - 1
    rel, rel_terms, conv = [], [], []
    for g in np.unique(gid):
        m = torch.as_tensor(gid == g, device=X.device)
        ng = float(goff[g + 1] - goff[g])
        size = (float(torch.linalg.norm(4 * prm.lambda_kl * Td[m, 0:2])) +
                float(torch.linalg.norm(4 * prm.lambda_kl * Td[m, 2:4] / Zd[g])) +
                float(torch.linalg.norm(prm.lambda_c / ng * Xs[m])) +
                float(torch.linalg.norm(prm.lambda_r / ng ** 2 * Td[m, 4:6])))
        den = float(torch.linalg.norm(Gd[m]))
        dif = float(torch.linalg.norm(Gs[m] - Gd[m]))
        if size > 0:
            rel_terms.append(dif / size)
            conv.append(den / size)
        if den > 0 and den >= 1e-3 * size:
            rel.append(dif / den)
    acc = {"rows": int(rows.size), "graphs": len(rel_terms),
           "rel_l2_max": max(rel) if rel else None,
           "rel_l2_median": float(np.median(rel)) if rel else None,
           "graphs_not_converged": len(rel),
           "term_normalised_max": max(rel_terms),
           "G_over_terms_min": min(conv),
           "note": "rel_l2 over graphs with |G| >= 1e-3 of the sum of its terms' norms; "
                   "term_normalised = |dG| / sum of the terms' norms, every graph"}
    z_err = float(torch.max(torch.abs(Z - Zd) / Zd).item()) if Gn else 0.0
    # the grid along the run (untimed replay from the same start)
    Xr = X0d.clone()
    upd.zero_()
    gains.fill_(1.0)
    ni_max, far_tot, ni_hist = [], [], {}
    for it in range(iters):
        prob.grad(Xr, prm, G=G, Z=Z, stream=stream)
        prob.step(Xr, upd, gains, G, it, sp, stream=stream)
        gi = prob.grid_info()
        ni_max.append(int(gi["n_intervals"].max()))
        far_tot.append(int(gi["far_points"].sum()))
        for v in gi["n_intervals"].tolist():
            ni_hist[v] = ni_hist.get(v, 0) + 1
    return {
        "iters": iters, "iters_per_s": iters / wall, "ms_per_step": wall / iters * 1e3,
        "ns_per_vertex_iter": wall / iters / n * 1e9,
        f"iters_per_s_per_{block}": rates,
        "status_after_timed_steps": status,
        "grid_capped_in_timed_steps": bool(status & 0x2),
        "n_intervals_max": max(ni_max), "n_intervals_end": ni_max[-1],
        "n_intervals_graph_steps": {str(k): v for k, v in sorted(ni_hist.items())},
        "far_points_range": [min(far_tot), max(far_tot)],
        "accuracy_vs_direct_f64": acc,
        "Z_rel_vs_direct_max": z_err,
    }


def prob_offsets(prob):
    return prob.graph_offsets if getattr(prob, "graph_offsets", None) is not None else [0, prob.n]


def workload_legs(api, ctx, which, iters):
    """Rates of the other configurations: SBM n = 2e4 and RGG n = 1e5 (one graph
    each), the mixed batch of 256 graphs (one launch per stage for all of
    them), each from N(0, 1e-4) with P built on the GPU."""
    import torch
    from synth import graphs
    dev = torch.device("cuda", 0)
    prm, sp = api.Params(), api.StepParams()
    out = {}
    specs = {
        "sbm20k": ("SBM 20 blocks of 1000, p_in 0.01, p_out 5e-5, seed 1; perplexity 40", graphs.workload_sbm20k, 1),
        "rgg100k": ("RGG n = 1e5, mean degree 8, seed 2; perplexity 40", graphs.workload_rgg100k, 2),
        "mixed256": ("256 SBM / grid / tree graphs, n ~ U{500..50000}, seed 4; perplexity 40",
                     graphs.workload_mixed256, 4),
    }
    for key in which:
        desc, make, seed = specs[key]
        t0 = time.perf_counter()
        g = make()
        goff = getattr(g, "graph_offsets", None)
        n = g.indptr.shape[0] - 1
        log(f"{key}: n={n} graph made in {time.perf_counter() - t0:.1f} s")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob = api.Problem.build(ctx, g.indptr, g.indices, 40.0, seed=seed,
                                 graph_offsets=None if goff is None else goff.astype(np.int64))
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - t0) * 1e3
        prob.graph_offsets = None if goff is None else goff.astype(np.int64)
        X0d = torch.tensor(graphs.initial_layout(n, seed), device=dev)
        r = descent_leg(api, ctx, prob, X0d, iters, prm, sp, seed=seed)
        r.update({"workload": desc, "n": n, "graphs": prob.num_graphs, "nnz_P": prob.nnz,
                  "build_P_ms": build_ms, "grid_workspace_bytes": prob.workspace_bytes()})
        log(f"{key}: {r['iters_per_s']:.1f} iters/s over {iters} steps, status {r['status_after_timed_steps']:#x}, "
            f"n_int max {r['n_intervals_max']}, far points {r['far_points_range']}, "
            f"G vs direct: {r['accuracy_vs_direct_f64']}")
        out[key] = r
        prob.free()
        del prob, X0d
        torch.cuda.empty_cache()
    return out


# --------------------------------------------------------------------------- per-kernel table
# layouts N(0, std^2) and the interval cap: 256, 512 and 1024 intervals at n = 1e6
FIXED_GRID_PHASES = ((6.0, 512), (12.0, 512), (25.0, 1024))
FIXED_GRID_EVALS = 20


def fixed_grids(info_path: str):
    """Gradient evaluations (each followed by a step on a copy, so the layout and
    its grid stay fixed) at two fixed layouts of the benchmark problem, for a
    kernel trace; writes the sizes the per-kernel table needs to info_path."""
    import torch
    from synth import graphs
    from paper_2509_19785_amd import api
    g = graphs.workload_ba1m()
    ctx = api.Context(0)
    dev = torch.device("cuda", 0)
    prob = api.Problem.build(ctx, torch.as_tensor(g.indptr).to(dev), torch.as_tensor(g.indices).to(dev),
                             40.0, seed=3)
    sp = api.StepParams()
    info = {"n": prob.n, "nnz": prob.nnz, "phases": []}
    for std, max_int in FIXED_GRID_PHASES:
        prm = api.Params(max_intervals=max_int)
        X = torch.tensor(graphs.initial_layout(g.n, 1, std=std), device=dev)
        upd, gains = torch.zeros_like(X), torch.ones_like(X)
        G, Z = torch.empty_like(X), torch.empty(1, dtype=torch.float64, device=dev)
        for _ in range(FIXED_GRID_EVALS):
            prob.grad(X, prm, G=G, Z=Z)
            prob.step(X.clone(), upd, gains, G, 300, sp)
        torch.cuda.synchronize()
        ni = int(prob.grid_info()["n_intervals"][0])
        info["phases"].append({"std": std, "n_int": ni, "evals": FIXED_GRID_EVALS})
        log(f"fixed layout std={std}: {ni} intervals")
    with open(info_path, "w") as f:
        json.dump(info, f)


def kernel_algorithmic_bytes(kernel: str, n: int, nnz: int, ni: int):
    """Compulsory HBM bytes of one launch of each per-iteration kernel at n
    vertices, nnz nonzeros and ni intervals per axis (N_g = 3 ni nodes, M = 6 ni)."""
    ng, Mh = 3 * ni, 3 * ni + 1
    return {
        "k_attract_tiled": 8 * nnz + 40 * n + 8,
        "k_bbox_part": 8 * n,
        "k_bin_keys": 12 * n,
        "k_box_bounds": 12 * ng * ng,                         # clears the 3 charge grids
        "k_spread_ranges": 12 * n + 12 * ng * ng,
        "k_gather": 32 * n + 32 * ng * ng,
        "k_fft_rows_fwd": 12 * ng * ng + 3 * ng * Mh * 8 + 4 * Mh * Mh * 4,
        "k_fft_cols": 3 * ng * Mh * 8 + 4 * Mh * Mh * 4 + 7 * Mh * ng * 8,
        "k_fft_rows_inv": 7 * Mh * ng * 8 + 32 * ng * ng,
        "k_step": 56 * n,
        "k_step_pairs": 56 * n,
    }.get(kernel)


def kernel_table(trace_csv: str, info_path: str):
    """Markdown table of the per-iteration kernels from a rocprofv3 kernel trace
    of --fixed-grids: mean duration per layout, algorithmic bytes, GB/s and the
    fraction of the 8 TB/s HBM peak. Launches are assigned to the layouts by
    time (the step kernel runs once per evaluation in every layout); a
    transform kernel of the large class (FFT length 6144) is listed as such
    and only where it ran."""
    import collections
    import csv
    import re
    info = json.load(open(info_path))
    n, nnz, phases = info["n"], info["nnz"], info["phases"]
    seq = collections.defaultdict(list)
    for r in csv.DictReader(open(trace_csv)):
        name = r["Kernel_Name"]
        name = name[:name.index("(")] if "(" in name else name
        name = name.replace("void ", "").replace("tsnet::", "")
        m = re.match(r"(\w+)<FftCfg<(\d+), \d+> >", name)
        if m:
            name = m.group(1) + (" (M <= 3072)" if int(m.group(2)) <= 3072 else " (M 6144)")
        seq[name].append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    # the step runs as k_step_pairs where its arrays are 16-byte aligned, else as k_step
    steps = sorted(seq["k_step"] + seq["k_step_pairs"])
    per = FIXED_GRID_EVALS
    # phase p spans its per-evaluation steps (the last step of the previous phase to its own last)
    ends = [steps[(p + 1) * per - 1][0] for p in range(len(phases))]
    starts = [0] + [steps[p * per - 1][0] for p in range(1, len(phases))]
    print("| kernel | intervals | launches | mean us | algorithmic bytes | GB/s | of 8 TB/s |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for k in sorted(seq, key=lambda x: -sum(d for _, d in seq[x])):
        for p, ph in enumerate(phases):
            d = [dur for t, dur in seq[k] if starts[p] < t <= ends[p]]
            if len(d) < per or len(d) % per:
                continue  # not a once-per-evaluation kernel of this layout
            if k.endswith("(M <= 3072)") and ph["n_int"] > 512:
                continue  # launched, but its blocks leave the grid to the large class
            avg_us = sum(d) / len(d) / 1e3
            b = kernel_algorithmic_bytes(k.split(" ")[0], n, nnz, ph["n_int"])
            if b:
                gbs = b / (avg_us * 1e-6) / 1e9
                print(f"| {k} | {ph['n_int']} | {len(d)} | {avg_us:.1f} | {b:,} | {gbs:.0f} | "
                      f"{gbs / HBM_PEAK_GBS:.2f} |")
            else:
                print(f"| {k} | {ph['n_int']} | {len(d)} | {avg_us:.1f} | | | |")


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
    ap.add_argument("--pmds-pivots", type=int, default=50,
                    help="pivots of the Pivot MDS leg (0: skip it)")
    ap.add_argument("--metric-sources", type=int, default=64,
                    help="stress sources for the quality-metric leg on the final layout (0: skip the leg)")
    ap.add_argument("--small-iters", type=int, default=500,
                    help="iterations of the 32 x 32 grid comparison of L-tsNET and full-P tsNET (0: skip)")
    ap.add_argument("--variant-steps", type=int, default=100,
                    help="timed steps of the FIt-tsNET and BH-tsNET variants (0: skip them)")
    ap.add_argument("--runs", type=int, default=5,
                    help="timed runs from the initial layout (plain launches); value is their mean")
    ap.add_argument("--last", type=int, default=100,
                    help="the rate of the last LAST steps of every run is reported beside the whole-run rate")
    ap.add_argument("--c1-iters", type=int, default=500,
                    help="iterations of the 32 x 32 grid run from N(0, 1e-4), exact FP64 gradient "
                         "and FP32 interpolation (0: skip)")
    ap.add_argument("--long-steps", type=int, default=1000,
                    help="steps of the long run of the benchmark problem from the initial layout (0: skip)")
    ap.add_argument("--legs", default="sbm20k,rgg100k,mixed256",
                    help="comma-separated rate legs of the other configurations ('' to skip)")
    ap.add_argument("--leg-iters", type=int, default=0,
                    help="steps of every rate leg (0: 1000 for sbm20k and mixed256, 500 for rgg100k)")
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="iterations per captured HIP graph in the timed region (0: plain launches; "
                         "graph replays measured slower than plain launches on ROCm 7, and event "
                         "times read from graph nodes are not usable)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run 5 device copies of 1 GiB (reference for the HBM traffic counters)")
    ap.add_argument("--fixed-grids", metavar="INFO_JSON",
                    help="only run gradient evaluations at two fixed layouts (for a kernel trace)")
    ap.add_argument("--kernel-table", nargs=2, metavar=("TRACE_CSV", "INFO_JSON"),
                    help="only print the per-kernel roofline table of a --fixed-grids trace")
    args = ap.parse_args()
    if args.kernel_table:
        kernel_table(*args.kernel_table)
        return
    if args.fixed_grids:
        fixed_grids(args.fixed_grids)
        return
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
        print("bench.py measures one GPU only: the library has no multi-GPU path "
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

    # Pivot MDS starting layout of the same graph (not part of the timed steps)
    pm = None
    if args.pmds_pivots > 0:
        for rep in range(2):  # the second call is timed (the first allocates)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = api.pmds(ctx, ip, ix, pivots=args.pmds_pivots, seed=3)
            torch.cuda.synchronize()
            pm_s = time.perf_counter() - t0
        pm = {
            "ms": pm_s * 1e3,
            "pivots": args.pmds_pivots,
            "bfs_levels": r["levels"],
            "arcs_per_s": args.pmds_pivots * int(ix.numel()) / pm_s,
            "eig": [float(v) for v in r["eig"][0]],
        }
        if not args.no_cpu_baseline:
            pm["cpu_oracle"] = pmds_cpu_baseline(g, args.pmds_pivots)
        log(f"pmds: {args.pmds_pivots} pivots in {pm_s * 1e3:.1f} ms ({r['levels']} BFS levels)")
        del r
    del ip, ix

    X0d = torch.tensor(X0, device=dev)
    X = X0d.clone()
    upd = torch.zeros_like(X)
    gains = torch.ones_like(X)
    G = torch.empty_like(X)
    Z = torch.empty(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def one(it):
        prob.grad(X, prm, G=G, Z=Z, stream=stream)
        prob.step(X, upd, gains, G, it, sp, stream=stream)

    def restart():
        X.copy_(X0d)
        upd.zero_()
        gains.fill_(1.0)

    for it in range(args.warmup):
        one(it)
    torch.cuda.synchronize()
    log(f"warmup done, status {ctx.status():#x}")
    last = max(1, min(args.last, args.steps))

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
        status_timed = ctx.status()
        del g_early, g_late
        run_rates, last_rates = [args.steps / wall], []
    else:
        # every run starts from the initial layout: warmup steps untimed, then
        # exactly --steps steps between two device synchronisations
        run_rates, last_rates, attr_ms, attr_calls = [], [], 0.0, 0
        status_timed = 0
        for r in range(max(1, args.runs)):
            if r > 0:
                restart()
                for it in range(args.warmup):
                    one(it)
            ev_last = torch.cuda.Event(enable_timing=True)
            ev_end = torch.cuda.Event(enable_timing=True)
            ctx.set_timing(["attract_assemble"])
            ctx.stage_times()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for it in range(args.warmup, args.warmup + args.steps):
                if it == args.warmup + args.steps - last:
                    ev_last.record(stream)
                one(it)
            ev_end.record(stream)
            torch.cuda.synchronize()
            w = time.perf_counter() - t0
            status_timed |= ctx.status()  # raised during the warm-up and timed steps of this run
            a_ms, a_calls = ctx.stage_times()["attract_assemble"]
            ctx.set_timing(None)
            attr_ms += a_ms
            attr_calls += a_calls
            run_rates.append(args.steps / w)
            last_rates.append(last / (ev_last.elapsed_time(ev_end) * 1e-3))
            log(f"run {r}: {run_rates[-1]:.1f} iters/s, last {last} steps {last_rates[-1]:.1f} iters/s")
        st = {"attract_assemble": (attr_ms, attr_calls)}
        wall = args.steps / (sum(run_rates) / len(run_rates))
    ms_per_step = wall / args.steps * 1e3
    iters_per_s = args.steps / wall
    attr_ms, attr_calls = st["attract_assemble"]
    attr_avg_s = attr_ms / max(attr_calls, 1) * 1e-3
    n, nnz, prob_k = prob.n, prob.nnz, prob.k
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

    # grid of every iteration of one run (replayed untimed: reading it synchronises)
    restart()
    grid_ni, grid_span, grid_far = [], [], []
    for it in range(args.warmup + args.steps):
        one(it)
        g_i = prob.grid_info()
        grid_ni.append(int(g_i["n_intervals"][0]))
        grid_span.append(float(g_i["n_intervals"][0]) * float(g_i["box_side"][0]))
        grid_far.append(int(g_i["far_points"][0]))
    log("grid per iteration (it span n_int M far): " + "; ".join(
        f"{i} {grid_span[i]:.2f} {grid_ni[i]} {6 * grid_ni[i]} {grid_far[i]}" for i in range(len(grid_ni))))
    # quality metrics of the layout the run ended with (not part of the timed steps):
    # neighbourhood preservation of every vertex, stress over sampled sources
    met = None
    if args.metric_sources > 0:
        ipm = torch.as_tensor(g.indptr).to(dev)
        ixm = torch.as_tensor(g.indices).to(dev)
        Xf = X.clone()
        src = np.random.default_rng(3).choice(g.n, min(args.metric_sources, g.n),
                                              replace=False).astype(np.int32)
        for rep in range(2):  # the second calls are timed (the first allocate)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r_np = api.neighbourhood_preservation(ctx, ipm, ixm, Xf)
            torch.cuda.synchronize()
            np_s = time.perf_counter() - t0
            t0 = time.perf_counter()
            r_st = api.stress(ctx, ipm, ixm, Xf, src)
            torch.cuda.synchronize()
            st_s = time.perf_counter() - t0
        ball = r_np["ball"].to(torch.int64)
        met = {
            "layout": f"after {args.warmup + args.steps} steps",
            "np": {"value": float(r_np["np"][0]), "ms": np_s * 1e3, "vertices_per_s": g.n / np_s,
                   "sum_ball": int(ball.sum()), "max_ball": int(ball.max())},
            "stress": {"value": float(r_st["stress"][0]),
                       "best_scale": float(r_st["stress_best_scale"][0]),
                       "ms": st_s * 1e3, "sources": int(len(src)), "levels": r_st["levels"],
                       "pairs": float(r_st["sums"][0, 0]),
                       "pairs_per_s": float(r_st["sums"][0, 0]) / st_s},
        }
        if not args.no_cpu_baseline:
            met["cpu_oracle"] = metrics_cpu_baseline(g, Xf.cpu().numpy(), sources=len(src))
        log(f"metrics: NP {met['np']['value']:.6f} in {np_s * 1e3:.1f} ms; stress "
            f"{met['stress']['value']:.4f} ({len(src)} sources) in {st_s * 1e3:.1f} ms")
        del ipm, ixm, Xf, r_np, ball
    timed_ni = grid_ni[args.warmup:]
    ni_runs = []
    for v in timed_ni:
        if ni_runs and ni_runs[-1][0] == v:
            ni_runs[-1][1] += 1
        else:
            ni_runs.append([v, 1])

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
            # per pair: 2 differences, r2 (an fma and a product), 1 + r2 and eps + r2,
            # their product, a reciprocal with Newton steps (5), w, ke, w^2, the z sum
            # and four fmas: 25 FP64 operations, an fma counted as 2
            "flop_per_pair": 25,
            "fp64_tflops": pairs / dwall * 25 / 1e12,
            "frac_of_fp64_peak": pairs / dwall * 25 / 78.6e12,
            "rel_l2_interp_vs_direct": err,
            "Z_direct": float(Zd.item()),
            "Z_interp": float(Z.item()),
        }
        log(f"direct f64: {dwall * 1e3:.1f} ms/iter; interp speedup {iters_per_s * dwall:.1f}x; "
            f"rel L2 {err:.2e}")

    # the paper's other two algorithms on the same problem: FIt-tsNET (quadtree
    # entropy) and BH-tsNET (quadtree repulsion and entropy), each from the initial
    # layout with the same warm-up, then --variant-steps timed steps
    variants = None
    if args.variant_steps > 0:
        variants = {}
        if direct is not None:
            # exact FP64 terms at the same layout: errors of the repulsion F_rep / Z and of
            # F_ent per method (the gradient error grows where attraction and repulsion cancel)
            _, Zd_t, Td = prob.grad_direct_f64(X64, prm, with_terms=True)
            rep_d = Td[:, 2:4] / Zd_t[0]
            ent_d = Td[:, 4:6]

            def term_errors(pv):
                t = prob.grad_terms(X, pv)
                torch.cuda.synchronize()
                rep = t["F_rep"].double() / t["Z"][0]
                return {"rel_l2_vs_direct": float(torch.linalg.norm(t["G"].double() - Gd) / torch.linalg.norm(Gd)),
                        "rep_over_Z_rel_l2": float(torch.linalg.norm(rep - rep_d) / torch.linalg.norm(rep_d)),
                        "F_ent_rel_l2": float(torch.linalg.norm(t["F_ent"].double() - ent_d) / torch.linalg.norm(ent_d))}
            direct["terms_L-tsNET"] = term_errors(prm)
            direct["BH-tsNET_theta_0.25"] = term_errors(api.Params.variant("BH-tsNET", theta=0.25,
                                                                             max_intervals=args.max_intervals))
        names = ("FIt-tsNET", "BH-tsNET")
        for name in names:  # accuracy first, all at the layout the direct kernel saw
            pv = api.Params.variant(name, max_intervals=args.max_intervals)
            variants[name] = {"theta": pv.theta}
            if direct is not None:
                variants[name].update(term_errors(pv))
        for name in names:
            pv = api.Params.variant(name, max_intervals=args.max_intervals)
            entry = variants[name]
            restart()
            for it in range(args.warmup):
                prob.grad(X, pv, G=G, Z=Z, stream=stream)
                prob.step(X, upd, gains, G, it, sp, stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for it in range(args.warmup, args.warmup + args.variant_steps):
                prob.grad(X, pv, G=G, Z=Z, stream=stream)
                prob.step(X, upd, gains, G, it, sp, stream=stream)
            torch.cuda.synchronize()
            vw = time.perf_counter() - t0
            ctx.set_timing("all")
            for it in range(args.warmup + args.variant_steps, args.warmup + args.variant_steps + 10):
                prob.grad(X, pv, G=G, Z=Z, stream=stream)
                prob.step(X, upd, gains, G, it, sp, stream=stream)
            torch.cuda.synchronize()
            vst = {k: v[0] / v[1] for k, v in ctx.stage_times().items() if v[1]}
            ctx.set_timing(None)
            entry.update({"iters_per_s": args.variant_steps / vw, "steps": args.variant_steps,
                          "ms_per_step": vw / args.variant_steps * 1e3, "stages_ms": vst})
            log(f"{name}: {entry['iters_per_s']:.1f} iters/s, quadtree stage "
                f"{vst.get('quadtree', 0.0):.3f} ms" +
                (f", rel L2 vs direct: G {entry['rel_l2_vs_direct']:.2e}, F_rep/Z "
                 f"{entry['rep_over_Z_rel_l2']:.2e}, F_ent {entry['F_ent_rel_l2']:.2e}"
                 if "rel_l2_vs_direct" in entry else ""))
        if direct is not None:
            log(f"L-tsNET terms vs direct: {direct['terms_L-tsNET']}; BH theta 0.25: {direct['BH-tsNET_theta_0.25']}")
        # the paper's whole-run speed-ups (CPU implementations, hardware not named),
        # beside the ratios of the iteration rates measured here
        variants["paper_speedups"] = {
            "source": "Sec. 4.2, averages over its benchmark graphs, 500 iterations, CPU (hardware not named)",
            "L-tsNET / tsNET runtime": "98.6 % less (about 71x)", "FIt-tsNET / tsNET runtime": "96 % less (about 25x)",
            "BH-tsNET / tsNET runtime": "93.5 % less (about 15x)",
            "L-tsNET vs BH-tsNET": 4.7, "L-tsNET vs FIt-tsNET": 3.0, "FIt-tsNET vs BH-tsNET": 1.58}
        variants["measured_ratios"] = {
            "L-tsNET vs BH-tsNET": iters_per_s / variants["BH-tsNET"]["iters_per_s"],
            "L-tsNET vs FIt-tsNET": iters_per_s / variants["FIt-tsNET"]["iters_per_s"],
            "FIt-tsNET vs BH-tsNET": variants["FIt-tsNET"]["iters_per_s"] / variants["BH-tsNET"]["iters_per_s"]}

    long_run = None
    if args.long_steps > 0:
        long_run = descent_leg(api, ctx, prob, X0d, args.long_steps, prm, sp, seed=3)
        long_run["workload"] = "the benchmark problem, one run of --long-steps steps from the initial layout"
        log(f"long run: {long_run['iters_per_s']:.1f} iters/s over {args.long_steps} steps "
            f"(per 100: {', '.join(f'{v:.0f}' for v in long_run['iters_per_s_per_100'])}), status "
            f"{long_run['status_after_timed_steps']:#x}, n_int max {long_run['n_intervals_max']}, far points "
            f"{long_run['far_points_range']}, G vs direct {long_run['accuracy_vs_direct_f64']}")

    small = small_n_leg(api, ctx, args.small_iters, cpu=not args.no_cpu_baseline) \
        if args.small_iters > 0 else None
    c1 = c1_leg(api, ctx, args.c1_iters) if args.c1_iters > 0 else None

    legs = None
    which = [w for w in args.legs.split(",") if w]
    if which:
        prob.free()
        del prob
        torch.cuda.empty_cache()
        legs = {}
        for w in which:
            iters = args.leg_iters or (500 if w == "rgg100k" else 1000)
            legs.update(workload_legs(api, ctx, [w], iters))

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
            "n": n, "edges": int(g.m), "perplexity": 40.0, "k": prob_k, "nnz_P": nnz,
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
            "traffic": attract_traffic(),
            "algorithmic_bytes": attr_bytes,
            "avg_launch_us": attr_avg_s * 1e6,
            "launches_timed": attr_calls,
        },
        "cpu_baseline": cpu,
        "runs": {
            "count": len(run_rates),
            "iters_per_s": run_rates,
            "mean": float(np.mean(run_rates)),
            "sd": float(np.std(run_rates, ddof=1)) if len(run_rates) > 1 else 0.0,
            "last_steps": last,
            "last_iters_per_s": last_rates,
            "last_mean": float(np.mean(last_rates)) if last_rates else None,
        },
        "grid_timed_steps": {
            "n_intervals_runs": ni_runs,
            "fft_length_M": "6 * n_intervals",
            "span_min": float(min(grid_span[args.warmup:])),
            "span_max": float(max(grid_span[args.warmup:])),
            "span_is": "side of the region the grid covers (the core when far points are set apart)",
            "far_points_min": int(min(grid_far[args.warmup:])),
            "far_points_max": int(max(grid_far[args.warmup:])),
            "status_after_timed_steps": status_timed,
            "grid_capped_in_timed_steps": bool(status_timed & 0x2),
        },
        "build_P_ms": build_ms,
        "pmds": pm,
        "metrics": met,
        "stages_ms": stages,
        "direct_f64": direct,
        "variants": variants,
        "long_run": long_run,
        "small_n": small,
        "c1_grid32": c1,
        "workloads": legs,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
