"""Torch-facing wrappers over the C ABI (device memory and streams come from torch).

Nothing here computes: each method checks tensor shapes/dtypes/devices and
calls the matching ``tsnet_*`` entry point of libtsnet.so on the current (or
given) torch stream.
"""
from __future__ import annotations

import ctypes
import weakref
from dataclasses import dataclass, fields

import numpy as np
import torch

from . import _lib
from ._lib import check, lib


@dataclass
class Params:
    lambda_kl: float = 1.0
    lambda_c: float = 1.2
    lambda_r: float = 0.01
    eps_r: float = 0.05
    interval_width: float = 0.25
    min_intervals: int = 50
    max_intervals: int = 512
    nodes_per_interval: int = 3
    attract_layout: int = 0   # 0 automatic, 1 CSR rows, 2 tiled (row tiles x column windows)
    repulsion: int = 0        # 0 interpolation, 1 quadtree (Barnes-Hut)
    entropy: int = 0          # 0 interpolation, 1 quadtree (Eq. 7)
    theta: float = 0.5        # quadtree opening threshold, (0, 0.7]
    far_trim: int = 64        # t of the far-point rule of the grid (0: the grid covers the bounding box)

    @classmethod
    def variant(cls, name: str, **kw) -> "Params":
        """The settings of one of the paper's three algorithms: "L-tsNET"
        (interpolation), "FIt-tsNET" (quadtree entropy), "BH-tsNET" (quadtree
        repulsion and entropy)."""
        rep, ent = {"L-tsNET": (0, 0), "FIt-tsNET": (0, 1), "BH-tsNET": (1, 1)}[name]
        return cls(repulsion=rep, entropy=ent, **kw)

    def to_c(self) -> _lib.tsnet_params:
        p = _lib.tsnet_params()
        for f in fields(self):
            setattr(p, f.name, getattr(self, f.name))
        p.reserved = 0
        return p


@dataclass
class StepParams:
    eta: float = 0.0
    momentum_early: float = 0.5
    momentum_late: float = 0.8
    min_gain: float = 0.01
    gain_up: float = 0.2
    gain_down: float = 0.8
    momentum_switch_iter: int = 250

    def to_c(self) -> _lib.tsnet_step_params:
        p = _lib.tsnet_step_params()
        for f in fields(self):
            setattr(p, f.name, getattr(self, f.name))
        return p


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev(t: torch.Tensor, dtype, shape=None, name="tensor") -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


def _opt(t, dtype, shape, name):
    return None if t is None else _dev(t, dtype, shape, name)


class Context:
    def __init__(self, device: int = 0):
        self.device = device
        h = ctypes.c_void_p()
        check(lib.tsnet_ctx_create(ctypes.byref(h), device))
        self.handle = h
        self._problems = weakref.WeakSet()

    def close(self):
        """Free the problems still alive in this context, then the context."""
        if self.handle:
            for p in list(self._problems):
                p.free()
            check(lib.tsnet_ctx_destroy(self.handle))
            self.handle = None

    def status(self) -> int:
        v = ctypes.c_uint32()
        check(lib.tsnet_status(self.handle, ctypes.byref(v)))
        return v.value

    def set_timing(self, stages=None):
        """Time the named stages with HIP events (None or [] = off, "all" = every stage)."""
        k = lib.tsnet_stage_count()
        names = [lib.tsnet_stage_name(i).decode() for i in range(k)]
        if stages == "all":
            mask = (1 << k) - 1
        else:
            mask = 0
            for s in stages or []:
                mask |= 1 << names.index(s)
        check(lib.tsnet_set_timing(self.handle, mask))

    def stage_times(self):
        k = lib.tsnet_stage_count()
        ms = (ctypes.c_double * k)()
        calls = (ctypes.c_int64 * k)()
        check(lib.tsnet_stage_times(self.handle, ms, calls))
        return {lib.tsnet_stage_name(i).decode(): (ms[i], calls[i]) for i in range(k)}

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


def _offsets(graph_offsets, n):
    if graph_offsets is None:
        return None, 1
    go = np.ascontiguousarray(np.asarray(graph_offsets, dtype=np.int32))
    return go, go.shape[0] - 1


class Problem:
    """One graph batch with its affinities P and evaluation workspace."""

    def __init__(self, ctx: Context, handle: ctypes.c_void_p):
        self.ctx = ctx
        self.handle = handle
        ctx._problems.add(self)
        n, nnz, G, k = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        check(lib.tsnet_P_info(handle, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(G),
                               ctypes.byref(k)))
        self.n, self.nnz, self.num_graphs, self.k = n.value, nnz.value, G.value, k.value

    @classmethod
    def build(cls, ctx: Context, indptr, indices, perplexity: float, k: int = 0, seed: int = 0,
              tie_mode: str = "hash", graph_offsets=None, stream=None) -> "Problem":
        dev = torch.device("cuda", ctx.device)
        ip = torch.as_tensor(np.asarray(indptr, dtype=np.int64)).to(dev) \
            if not isinstance(indptr, torch.Tensor) else indptr
        ix = torch.as_tensor(np.asarray(indices, dtype=np.int32)).to(dev) \
            if not isinstance(indices, torch.Tensor) else indices
        n = ip.shape[0] - 1
        go, G = _offsets(graph_offsets, n)
        mode = {"hash": _lib.TSNET_TIE_HASH, "id": _lib.TSNET_TIE_ID}[tie_mode]
        h = ctypes.c_void_p()
        check(lib.tsnet_build_P(ctx.handle, _dev(ip, torch.int64, None, "indptr"),
                                ix.data_ptr() if ix.numel() else None, n, ix.numel(),
                                None if go is None else go.ctypes.data, G, float(perplexity), k,
                                seed & ((1 << 64) - 1), mode, ctypes.byref(h), _stream(stream)))
        return cls(ctx, h)

    @classmethod
    def from_host(cls, ctx: Context, rowptr, col, val, graph_offsets=None) -> "Problem":
        rp = np.ascontiguousarray(np.asarray(rowptr, dtype=np.int64))
        cl = np.ascontiguousarray(np.asarray(col, dtype=np.int32))
        vl = np.ascontiguousarray(np.asarray(val, dtype=np.float32))
        n = rp.shape[0] - 1
        go, G = _offsets(graph_offsets, n)
        h = ctypes.c_void_p()
        check(lib.tsnet_P_from_host(ctx.handle, n, rp.ctypes.data, cl.ctypes.data if cl.size else None,
                                    vl.ctypes.data if vl.size else None,
                                    None if go is None else go.ctypes.data, G, ctypes.byref(h)))
        return cls(ctx, h)

    def free(self):
        if self.handle:
            check(lib.tsnet_P_free(self.handle))
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.free()
        except Exception:
            pass

    # ------------------------------------------------------------ exports
    def export(self, conditional: bool = False) -> dict:
        rowptr = np.zeros(self.n + 1, np.int64)
        col = np.zeros(max(self.nnz, 1), np.int32)
        val = np.zeros(max(self.nnz, 1), np.float32)
        out = {"rowptr": rowptr, "col": col[: self.nnz], "val": val[: self.nnz]}
        args = [rowptr.ctypes.data, col.ctypes.data, val.ctypes.data, None, None, None, None, None]
        if conditional:
            nk = max(self.n * self.k, 1)
            beta = np.zeros(self.n, np.float64)
            status = np.zeros(self.n, np.int8)
            clen = np.zeros(self.n, np.int32)
            cnbr = np.zeros(nk, np.int32)
            cdist = np.zeros(nk, np.uint16)
            args[3:] = [beta.ctypes.data, status.ctypes.data, clen.ctypes.data, cnbr.ctypes.data,
                        cdist.ctypes.data]
            out.update(beta=beta, status=status, cond_len=clen,
                       cond_nbr=cnbr[: self.n * self.k].reshape(self.n, self.k),
                       cond_dist=cdist[: self.n * self.k].reshape(self.n, self.k))
        check(lib.tsnet_P_export(self.handle, *args))
        return out

    def grid_info(self) -> dict:
        G = self.num_graphs
        ni = np.zeros(G, np.int32)
        h = np.zeros(G, np.float32)
        x0 = np.zeros(G, np.float32)
        y0 = np.zeros(G, np.float32)
        far = np.zeros(G, np.int32)
        check(lib.tsnet_grid_info(self.handle, ni.ctypes.data, h.ctypes.data, x0.ctypes.data,
                                  y0.ctypes.data, far.ctypes.data))
        return {"n_intervals": ni, "box_side": h, "x0": x0, "y0": y0, "far_points": far}

    def workspace_bytes(self) -> int:
        v = ctypes.c_size_t()
        check(lib.tsnet_workspace_bytes(self.handle, ctypes.byref(v)))
        return v.value

    # ------------------------------------------------------------ evaluation
    def grad(self, X: torch.Tensor, params: Params = Params(), G=None, Z=None, stream=None):
        n = self.n
        xp = _dev(X, torch.float32, (n, 2), "X")
        if G is None:
            G = torch.empty((n, 2), dtype=torch.float32, device=X.device)
        if Z is None:
            Z = torch.empty(self.num_graphs, dtype=torch.float64, device=X.device)
        prm = params.to_c()
        check(lib.tsnet_grad(self.ctx.handle, self.handle, xp, ctypes.byref(prm),
                             _dev(G, torch.float32, (n, 2), "G"),
                             _dev(Z, torch.float64, (self.num_graphs,), "Z"), _stream(stream)))
        return G, Z

    def grad_terms(self, X: torch.Tensor, params: Params = Params(), stream=None) -> dict:
        n = self.n
        dev = X.device
        out = {
            "G": torch.empty((n, 2), dtype=torch.float32, device=dev),
            "Z": torch.empty(self.num_graphs, dtype=torch.float64, device=dev),
            "F_attr": torch.empty((n, 2), dtype=torch.float32, device=dev),
            "F_rep": torch.empty((n, 2), dtype=torch.float32, device=dev),
            "F_ent": torch.empty((n, 2), dtype=torch.float32, device=dev),
            "Z_i": torch.empty(n, dtype=torch.float32, device=dev),
        }
        prm = params.to_c()
        check(lib.tsnet_grad_terms(self.ctx.handle, self.handle,
                                   _dev(X, torch.float32, (n, 2), "X"), ctypes.byref(prm),
                                   out["G"].data_ptr(), out["Z"].data_ptr(),
                                   out["F_attr"].data_ptr(), out["F_rep"].data_ptr(),
                                   out["F_ent"].data_ptr(), out["Z_i"].data_ptr(), _stream(stream)))
        return out

    def step(self, X, update, gains, G, it: int, sp: StepParams = StepParams(), stream=None):
        n = self.n
        spc = sp.to_c()
        check(lib.tsnet_step(self.ctx.handle, self.handle, _dev(X, torch.float32, (n, 2), "X"),
                             _dev(update, torch.float32, (n, 2), "update"),
                             _dev(gains, torch.float32, (n, 2), "gains"),
                             _dev(G, torch.float32, (n, 2), "G"), ctypes.byref(spc), int(it),
                             _stream(stream)))

    def run(self, X, update, gains, G, stages, first_iter: int = 0, sp: StepParams = StepParams(),
            Z=None, stream=None):
        """tsnet_run: the descent over a table of stages, each (iterations, Params);
        X, update and gains are updated in place, G and Z hold the last gradient."""
        n = self.n
        arr = (_lib.tsnet_stage * len(stages))()
        for k, (iters, prm) in enumerate(stages):
            arr[k].iterations = int(iters)
            arr[k].reserved = 0
            arr[k].params = prm.to_c()
        spc = sp.to_c()
        check(lib.tsnet_run(self.ctx.handle, self.handle, _dev(X, torch.float32, (n, 2), "X"),
                            _dev(update, torch.float32, (n, 2), "update"),
                            _dev(gains, torch.float32, (n, 2), "gains"),
                            _dev(G, torch.float32, (n, 2), "G"),
                            _opt(Z, torch.float64, (self.num_graphs,), "Z"), arr, len(stages),
                            int(first_iter), ctypes.byref(spc), _stream(stream)))

    def cost(self, X: torch.Tensor, params: Params = Params(), out=None, stream=None):
        if out is None:
            out = torch.empty((self.num_graphs, 4), dtype=torch.float64, device=X.device)
        prm = params.to_c()
        check(lib.tsnet_cost(self.ctx.handle, self.handle, _dev(X, torch.float32, (self.n, 2), "X"),
                             ctypes.byref(prm), _dev(out, torch.float64, (self.num_graphs, 4), "cost"),
                             _stream(stream)))
        return out

    def grad_direct_f64(self, X: torch.Tensor, params: Params = Params(), rows=None,
                        with_terms: bool = False, stream=None):
        n = self.n
        xp = _dev(X, torch.float64, (n, 2), "X")
        dev = X.device
        if rows is not None:
            rows = torch.as_tensor(rows, dtype=torch.int32, device=dev).contiguous()
            nr = rows.numel()
        else:
            nr = n
        G = torch.empty((nr, 2), dtype=torch.float64, device=dev)
        Z = torch.empty(self.num_graphs, dtype=torch.float64, device=dev)
        T = torch.empty((nr, 7), dtype=torch.float64, device=dev) if with_terms else None
        prm = params.to_c()
        check(lib.tsnet_grad_direct_f64(self.ctx.handle, self.handle, xp, ctypes.byref(prm),
                                        G.data_ptr(), Z.data_ptr(),
                                        None if rows is None else rows.data_ptr(), nr,
                                        None if T is None else T.data_ptr(), _stream(stream)))
        return (G, Z, T) if with_terms else (G, Z)


def pmds(ctx: Context, indptr, indices, pivots: int = 50, seed: int = 0, scale: float = 1e-2,
         graph_offsets=None, stream=None) -> dict:
    """Pivot MDS starting layout of a graph batch (tsnet_pmds): returns the layout
    X (float32 [n, 2] on the device), the pivots (int32 [graphs, pivots], -1 past
    a graph's count), the two leading eigenvalues per graph and the BFS levels run."""
    dev = torch.device("cuda", ctx.device)
    ip = torch.as_tensor(np.asarray(indptr, dtype=np.int64)).to(dev) \
        if not isinstance(indptr, torch.Tensor) else indptr
    ix = torch.as_tensor(np.asarray(indices, dtype=np.int32)).to(dev) \
        if not isinstance(indices, torch.Tensor) else indices
    n = ip.shape[0] - 1
    go, G = _offsets(graph_offsets, n)
    prm = _lib.tsnet_pmds_params()
    lib.tsnet_default_pmds_params(ctypes.byref(prm))
    prm.pivots, prm.seed, prm.scale = int(pivots), seed & ((1 << 64) - 1), float(scale)
    X = torch.empty((n, 2), dtype=torch.float32, device=dev)
    piv = torch.empty((G, int(pivots)), dtype=torch.int32, device=dev)
    eig = np.zeros((G, 2), dtype=np.float64)
    levels = ctypes.c_int32()
    check(lib.tsnet_pmds(ctx.handle, _dev(ip, torch.int64, None, "indptr"),
                         ix.data_ptr() if ix.numel() else None, n, ix.numel(),
                         None if go is None else go.ctypes.data, G, ctypes.byref(prm),
                         X.data_ptr(), piv.data_ptr(), eig.ctypes.data, ctypes.byref(levels),
                         _stream(stream)))
    return {"X": X, "pivots": piv, "eig": eig, "levels": levels.value}


def staged_schedule(total: int = 500, switch: int = 250, variant: str = "L-tsNET", **kw) -> list:
    """A two-stage table for Problem.run: compression without entropy up to
    `switch` (lambda_c 1.2, lambda_r 0), then light compression with entropy
    (lambda_c 0.01, lambda_r 0.01). The paper changes the multipliers between
    stages of the descent without giving values; these are this project's."""
    first = Params.variant(variant, lambda_c=1.2, lambda_r=0.0, **kw)
    second = Params.variant(variant, lambda_c=0.01, lambda_r=0.01, **kw)
    return [(min(switch, total), first), (max(0, total - switch), second)]


def _graph_dev(ctx: Context, indptr, indices):
    dev = torch.device("cuda", ctx.device)
    ip = torch.as_tensor(np.asarray(indptr, dtype=np.int64)).to(dev) \
        if not isinstance(indptr, torch.Tensor) else indptr
    ix = torch.as_tensor(np.asarray(indices, dtype=np.int32)).to(dev) \
        if not isinstance(indices, torch.Tensor) else indices
    return dev, ip, ix


def _ids_dev(ids, dev, name):
    t = torch.as_tensor(np.asarray(ids, dtype=np.int32)).to(dev) \
        if not isinstance(ids, torch.Tensor) else ids
    _dev(t, torch.int32, None, name)
    return t


def neighbourhood_preservation(ctx: Context, indptr, indices, X, vertices=None,
                               graph_offsets=None, stream=None) -> dict:
    """Neighbourhood preservation with r = 2 (tsnet_np): per evaluated vertex the
    2-hop ball size k and the hits (int32 on the device), and NP per graph."""
    dev, ip, ix = _graph_dev(ctx, indptr, indices)
    n = ip.shape[0] - 1
    go, G = _offsets(graph_offsets, n)
    _dev(X, torch.float32, (n, 2), "X")
    vt = None if vertices is None else _ids_dev(vertices, dev, "vertices")
    nv = n if vt is None else vt.numel()
    ball = torch.empty(nv, dtype=torch.int32, device=dev)
    hits = torch.empty(nv, dtype=torch.int32, device=dev)
    npg = np.zeros(G, dtype=np.float64)
    check(lib.tsnet_np(ctx.handle, _dev(ip, torch.int64, None, "indptr"),
                       ix.data_ptr() if ix.numel() else None, n, ix.numel(),
                       None if go is None else go.ctypes.data, G, X.data_ptr(),
                       None if vt is None else vt.data_ptr(), nv, ball.data_ptr(), hits.data_ptr(),
                       npg.ctypes.data, _stream(stream)))
    return {"ball": ball, "hits": hits, "np": npg}


def stress(ctx: Context, indptr, indices, X, sources, graph_offsets=None, stream=None) -> dict:
    """Stress over the pairs of the given sources (tsnet_stress): per graph the
    sums [pairs, sum (1 - e/d)^2, sum e/d, sum (e/d)^2], the stress, the stress
    at the best uniform scale, and the BFS levels run."""
    dev, ip, ix = _graph_dev(ctx, indptr, indices)
    n = ip.shape[0] - 1
    go, G = _offsets(graph_offsets, n)
    _dev(X, torch.float32, (n, 2), "X")
    st = _ids_dev(sources, dev, "sources")
    out = np.zeros((G, 6), dtype=np.float64)
    levels = ctypes.c_int32()
    check(lib.tsnet_stress(ctx.handle, _dev(ip, torch.int64, None, "indptr"),
                           ix.data_ptr() if ix.numel() else None, n, ix.numel(),
                           None if go is None else go.ctypes.data, G, X.data_ptr(), st.data_ptr(),
                           st.numel(), out.ctypes.data, ctypes.byref(levels), _stream(stream)))
    return {"sums": out[:, :4].copy(), "stress": out[:, 4].copy(),
            "stress_best_scale": out[:, 5].copy(), "levels": levels.value}


class StepGraph:
    """k iterations of (gradient, step) recorded once as a HIP graph and replayed.

    The library's calls only enqueue kernels on the given stream, so a stream
    capture records them as they are (torch.cuda.CUDAGraph is HIP's graph on
    ROCm). Everything is fixed at capture: the buffers, the parameters and the
    iteration numbers first_iter .. first_iter + k - 1 (they select the
    momentum of the step). Run every call once before capturing (the first
    gradient sizes the evaluation workspace). Stage timing that is on during
    the capture is recorded into the graph: each replay re-records the same
    events, so the stage times read afterwards are those of the last replay.
    """

    def __init__(self, problem: Problem, X, update, gains, G, Z, params: Params,
                 step_params: StepParams, first_iter: int, k: int):
        self.k = k
        self.first_iter = first_iter
        s = torch.cuda.Stream(device=X.device)
        s.wait_stream(torch.cuda.current_stream(X.device))
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(self.graph, stream=s):
                for t in range(k):
                    problem.grad(X, params, G=G, Z=Z, stream=s)
                    problem.step(X, update, gains, G, first_iter + t, step_params, stream=s)
        torch.cuda.current_stream(X.device).wait_stream(s)

    def replay(self):
        self.graph.replay()
