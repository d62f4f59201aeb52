"""MI355X (gfx950) Generalized Euclidean node-vector distances.

d(a, b) = sqrt((a - b)^T L^+ (a - b)) on an undirected weighted graph
(Coscia & Devriendt, section 3.1), computed with a Jacobi-preconditioned CG
Laplacian solve on the GPU instead of the pseudoinverse (section 3.2).

This module is a thin ctypes binding over libnvd.so (include/nvd.h): it
checks shapes, takes device pointers from torch tensors and passes the
current HIP stream.  Every numerical step runs in the library's HIP kernels;
if the library is missing, calls fail loudly.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _abi
from ._abi import (NvdOpts, PairInfo, Stats, NvdError, check, load,
                   NVD_FP64, NVD_MIXED, NVD_DT_F64, NVD_DT_F32, NVD_WARM_START)

__all__ = ["Graph", "Batch", "distance", "opts", "load", "NvdError", "PairInfo",
           "NVD_FP64", "NVD_MIXED"]


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _as_dev64(M, name):
    torch = _torch()
    if not isinstance(M, torch.Tensor):
        M = torch.as_tensor(np.asarray(M, dtype=np.float64))
    if M.dim() == 1:
        M = M.reshape(-1, 1)
    if M.dtype != torch.float64 or not M.is_cuda or M.stride(1) != 1:
        M = M.to(device="cuda", dtype=torch.float64).contiguous()
    return M


def opts(precision="fp64", rtol=1e-10, inner_rtol=1e-5, max_iter=20000, max_refine=30,
         tile_k=0, warm_start=False, precond="jacobi") -> NvdOpts:
    o = NvdOpts()
    check(load().nvd_opts_default(C.byref(o)))
    o.precision = {"fp64": NVD_FP64, "mixed": NVD_MIXED}[precision]
    o.rtol = rtol
    o.inner_rtol = inner_rtol
    o.max_iter = max_iter
    o.max_refine = max_refine
    o.tile_k = tile_k
    o.flags = NVD_WARM_START if warm_start else 0
    if precond == "tree":
        o.flags |= _abi.NVD_PRECOND_TREE
    elif precond == "auto":
        o.flags |= _abi.NVD_PRECOND_AUTO
    elif precond != "jacobi":
        raise ValueError("precond must be 'jacobi', 'tree' or 'auto'")
    return o


class Graph:
    """Device-resident graph handle built from a host CSR (symmetric, both
    directions stored; weights None for unit weights)."""

    def __init__(self, row_ptr, col_idx, weights=None, n=None):
        lib = load()
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
        self.n = int(rp.size - 1 if n is None else n)
        self.nnz_in = int(ci.size)
        h = C.c_void_p()
        st = lib.nvd_graph_create(self.n, self.nnz_in, rp.ctypes.data_as(C.c_void_p),
                                  ci.ctypes.data_as(C.c_void_p),
                                  None if w is None else w.ctypes.data_as(C.c_void_p),
                                  _stream(), C.byref(h))
        check(st, "nvd_graph_create")
        self._h = h
        self.weighted = w is not None

    @classmethod
    def from_csr(cls, row_ptr, col_idx, weights=None):
        return cls(row_ptr, col_idx, weights)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            load().nvd_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self) -> dict:
        s = Stats()
        check(load().nvd_graph_stats(self._h, C.byref(s)), "nvd_graph_stats")
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def query(self):
        lab = np.empty(self.n, dtype=np.int32)
        deg = np.empty(self.n, dtype=np.float64)
        check(load().nvd_graph_query(self._h, lab.ctypes.data_as(C.c_void_p),
                                     deg.ctypes.data_as(C.c_void_p)), "nvd_graph_query")
        return lab, deg

    # -- operator -----------------------------------------------------------
    def laplacian_apply(self, X, out=None):
        torch = _torch()
        if X.dim() == 1:
            X = X.reshape(-1, 1)
        assert X.is_cuda and X.shape[0] == self.n and X.stride(1) == 1
        dt = {torch.float64: NVD_DT_F64, torch.float32: NVD_DT_F32}[X.dtype]
        Y = torch.empty_like(X) if out is None else out
        check(load().nvd_laplacian_apply(self._h, dt, X.shape[1], _ptr(X), X.stride(0),
                                         _ptr(Y), Y.stride(0), _stream()),
              "nvd_laplacian_apply")
        return Y

    def project(self, P, Q):
        torch = _torch()
        P = _as_dev64(P, "P")
        Q = _as_dev64(Q, "Q")
        k = P.shape[1]
        D = torch.empty_like(P)
        norms = torch.empty(k, dtype=torch.float64, device=P.device)
        check(load().nvd_project(self._h, k, _ptr(P), _ptr(Q), P.stride(0), _ptr(D),
                                 D.stride(0), _ptr(norms), _stream()), "nvd_project")
        return D, norms

    # -- distances ----------------------------------------------------------
    def distances(self, P, Q, precision="fp64", rtol=1e-10, inner_rtol=1e-5, max_iter=20000,
                  max_refine=30, tile_k=0, return_x=False, X0=None, raise_on_noconv=False,
                  precond="jacobi"):
        """Returns (d, X or None, info list).  P, Q: (n, k) or (n,) float64.
        precond: "jacobi" (the diagonal), "tree" (a spanning forest, solved
        exactly) or "auto" (the forest when at most n/100 edges lie off it,
        else the diagonal)."""
        torch = _torch()
        P = _as_dev64(P, "P")
        Q = _as_dev64(Q, "Q")
        if P.shape != Q.shape or P.shape[0] != self.n:
            raise ValueError(f"P, Q must both be ({self.n}, k)")
        k = P.shape[1]
        o = opts(precision, rtol, inner_rtol, max_iter, max_refine, tile_k, X0 is not None, precond)
        d = torch.empty(k, dtype=torch.float64, device=P.device)
        X = None
        if return_x or X0 is not None:
            X = X0.clone().contiguous() if X0 is not None else \
                torch.empty_like(P)
        info = (PairInfo * k)()
        st = load().nvd_distances(self._h, k, _ptr(P), _ptr(Q), P.stride(0), C.byref(o),
                                  _ptr(d), _ptr(X), X.stride(0) if X is not None else 0,
                                  info, _stream())
        if st not in (_abi.NVD_OK, _abi.NVD_E_NOCONV, _abi.NVD_E_BREAKDOWN) or \
                (raise_on_noconv and st != _abi.NVD_OK):
            check(st, "nvd_distances")
        infos = [{f: getattr(i, f) for f, _ in PairInfo._fields_} for i in info]
        return d, X, infos


    def pairwise(self, V, precision="fp64", rtol=1e-10, inner_rtol=1e-5, max_iter=20000,
                 max_refine=30, tile_k=0, return_gram=False, precond="jacobi"):
        """All pairwise distances among the m columns of V (n x m): returns
        (D m x m, G m x m or None, info list of the m column solves)."""
        torch = _torch()
        V = _as_dev64(V, "V")
        if V.dim() != 2 or V.shape[0] != self.n:
            raise ValueError(f"V must be ({self.n}, m)")
        m = V.shape[1]
        o = opts(precision, rtol, inner_rtol, max_iter, max_refine, tile_k, precond=precond)
        D = torch.empty(m, m, dtype=torch.float64, device=V.device)
        G = torch.empty_like(D) if return_gram else None
        info = (PairInfo * m)()
        st = load().nvd_pairwise(self._h, m, _ptr(V), V.stride(0), C.byref(o), _ptr(D),
                                 D.stride(0), _ptr(G), G.stride(0) if G is not None else 0,
                                 info, _stream())
        if st not in (_abi.NVD_OK, _abi.NVD_E_NOCONV, _abi.NVD_E_BREAKDOWN):
            check(st, "nvd_pairwise")
        infos = [{f: getattr(i, f) for f, _ in PairInfo._fields_} for i in info]
        return D, G, infos
    def tuning(self, k, precision="mixed"):
        """(tile, neighbour lanes) the autotuner picks for k pairs."""
        t = C.c_int32()
        nl = C.c_int32()
        check(load().nvd_tune_query(self._h, k, {"fp64": NVD_FP64, "mixed": NVD_MIXED}[precision],
                                    C.byref(t), C.byref(nl), _stream()), "nvd_tune_query")
        return t.value, nl.value

    def set_weights(self, w):
        """Replace the edge weights (device float64, input CSR order)."""
        torch = _torch()
        w = w.detach().to(device="cuda", dtype=torch.float64).contiguous()
        assert w.numel() == self.nnz_in
        check(load().nvd_graph_set_weights(self._h, _ptr(w), _stream()), "nvd_graph_set_weights")
        self.weighted = True

    def grad_weights(self, X, gscale):
        """-1/2 sum_j g_j (x_i - x_c)^2 for every input CSR entry (i, c)."""
        torch = _torch()
        X = _as_dev64(X, "X")
        g = gscale.to(device=X.device, dtype=torch.float64).contiguous()
        out = torch.empty(self.nnz_in, dtype=torch.float64, device=X.device)
        check(load().nvd_grad_weights(self._h, X.shape[1], _ptr(X), X.stride(0), _ptr(g),
                                      _ptr(out), _stream()), "nvd_grad_weights")
        return out


class Batch:
    """Many graphs solved together in one persistent launch."""

    def __init__(self, graphs: Sequence[Graph]):
        lib = load()
        self.graphs = list(graphs)
        arr = (C.c_void_p * len(self.graphs))(*[g.handle for g in self.graphs])
        h = C.c_void_p()
        check(lib.nvd_batch_create(len(self.graphs), arr, _stream(), C.byref(h)),
              "nvd_batch_create")
        self._h = h
        self.ns = [g.n for g in self.graphs]

    def close(self):
        if getattr(self, "_h", None):
            load().nvd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self) -> dict:
        c, r, e = C.c_int64(), C.c_int64(), C.c_int64()
        check(load().nvd_batch_query(self._h, C.byref(c), C.byref(r), C.byref(e)), "nvd_batch_query")
        return {"captures": c.value, "replays": r.value, "eager": e.value}

    def trace(self):
        """(start_end ticks (G, 2), team sizes (G,)) of the last traced call."""
        G = len(self.graphs)
        se = np.zeros((G, 2), dtype=np.int64)
        ts = np.zeros(G, dtype=np.int32)
        check(load().nvd_batch_trace(self._h, G, se.ctypes.data_as(C.c_void_p),
                                     ts.ctypes.data_as(C.c_void_p)), "nvd_batch_trace")
        return se, ts

    @staticmethod
    def pack(P_list, Q_list):
        """Graph-major packed device copies of per-graph (n_g, k_g) blocks."""
        torch = _torch()
        ks = np.array([p.shape[1] if p.ndim == 2 else 1 for p in P_list], dtype=np.int32)
        Pf = torch.cat([_as_dev64(p, "P").reshape(-1) for p in P_list])
        Qf = torch.cat([_as_dev64(q, "Q").reshape(-1) for q in Q_list])
        return ks, Pf, Qf

    def distances(self, P_list, Q_list, precision="mixed", rtol=1e-8, inner_rtol=1e-5,
                  max_iter=20000, max_refine=30, return_x=False, packed=None, out=None,
                  persistent=False):
        """packed = (ks, Pf, Qf) from Batch.pack reuses device buffers (and so
        the persistent solver's captured launch); out = preallocated d tensor;
        persistent = the single persistent launch instead of the sweep
        solver."""
        torch = _torch()
        if packed is None:
            ks, Pf, Qf = self.pack(P_list, Q_list)
        else:
            ks, Pf, Qf = packed
        K = int(ks.sum())
        d = out if out is not None else torch.empty(K, dtype=torch.float64, device="cuda")
        X = torch.empty_like(Pf) if return_x else None
        info = (PairInfo * K)()
        o = opts(precision, rtol, inner_rtol, max_iter, max_refine)
        if persistent:
            o.flags |= _abi.NVD_BATCH_PERSISTENT
        st = load().nvd_batch_distances(self._h, ks.ctypes.data_as(C.c_void_p), _ptr(Pf),
                                        _ptr(Qf), C.byref(o), _ptr(d), _ptr(X), info,
                                        _stream())
        if st not in (_abi.NVD_OK, _abi.NVD_E_NOCONV, _abi.NVD_E_BREAKDOWN):
            check(st, "nvd_batch_distances")
        infos = [{f: getattr(i, f) for f, _ in PairInfo._fields_} for i in info]
        return d, X, infos


def prof_enable(on=True):
    """Bracket the solver's kernel launches with HIP events (see nvd.h)."""
    check(load().nvd_prof_enable(1 if on else 0), "nvd_prof_enable")


def prof_read() -> dict:
    """Per kernel kind: {'ms', 'launches', 'bytes'} summed since the last read."""
    k = _abi.NVD_PROF_KINDS
    ms = np.zeros(k)
    la = np.zeros(k, dtype=np.int64)
    by = np.zeros(k)
    check(load().nvd_prof_read(ms.ctypes.data_as(C.c_void_p), la.ctypes.data_as(C.c_void_p),
                               by.ctypes.data_as(C.c_void_p)), "nvd_prof_read")
    return {name: {"ms": float(ms[i]), "launches": int(la[i]), "bytes": float(by[i])}
            for i, name in enumerate(_abi.PROF_KIND_NAMES)}


def distance(g: Graph, p, q, **kw):
    """d(p, q) for vectors or column blocks; returns (d, info)."""
    d, _, info = g.distances(p, q, **kw)
    return d, info


from .autograd import DistanceSq, distance_sq, distance_t  # noqa: E402,F401
