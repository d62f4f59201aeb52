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

import atexit
import ctypes as C
import weakref
from typing import Optional, Sequence

import numpy as np

from . import _abi
from ._abi import (NvdOpts, PairInfo, Stats, NvdError, check, load,
                   NVD_FP64, NVD_MIXED, NVD_DT_F64, NVD_DT_F32, NVD_WARM_START)

__all__ = ["Graph", "Batch", "distance", "opts", "load", "NvdError", "PairInfo",
           "NVD_FP64", "NVD_MIXED", "grad_scale_from_d"]


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
    if M.dim() != 2:
        raise ValueError(f"{name} must be a vector or a 2-D block, got shape {tuple(M.shape)}")
    if M.dtype != torch.float64 or not M.is_cuda or M.stride(1) != 1 or M.stride(0) < M.shape[1]:
        M = M.to(device="cuda", dtype=torch.float64).contiguous()
    return M


def _check_out(t, name, shape, dtype):
    """A caller-supplied output buffer: a CUDA tensor of the given shape and
    dtype whose rows are contiguous (the library writes through its data
    pointer with row stride t.stride(0))."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if t.dim() == 2 and (t.stride(1) != 1 or t.stride(0) < t.shape[1]):
        raise ValueError(f"{name} must have unit column stride and rows that do not overlap")
    if t.dim() == 1 and t.stride(0) != 1:
        raise ValueError(f"{name} must be contiguous")
    return t


# Live handles, closed at interpreter exit (batches first, then graphs)
# while the HIP runtime is still up, so that no device memory, captured
# graph or stream is released from a finaliser during runtime teardown.
_live_graphs = weakref.WeakSet()
_live_batches = weakref.WeakSet()


@atexit.register
def _close_live_handles():
    for b in list(_live_batches):
        try:
            b.close()
        except Exception:
            pass
    for g in list(_live_graphs):
        try:
            g.close()
        except Exception:
            pass


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
    elif precond == "achol":
        o.flags |= _abi.NVD_PRECOND_ACHOL
    elif precond != "jacobi":
        raise ValueError("precond must be 'jacobi', 'tree', 'auto' or 'achol'")
    return o


class Graph:
    """Device-resident graph handle built from a symmetric CSR (both
    directions stored; weights None for unit weights).  The arrays may be
    host arrays (NumPy or anything array-like) or CUDA tensors (int64
    row_ptr, int32 col_idx, float64 weights), which the library reads in
    place."""

    def __init__(self, row_ptr, col_idx, weights=None, n=None):
        lib = load()
        torch = _torch()
        on_dev = isinstance(row_ptr, torch.Tensor) and row_ptr.is_cuda
        if on_dev:
            rp = row_ptr.to(dtype=torch.int64).contiguous()
            ci = torch.as_tensor(col_idx, device=rp.device).to(dtype=torch.int32).contiguous()
            w = None if weights is None else \
                torch.as_tensor(weights, device=rp.device).to(dtype=torch.float64).contiguous()
            nrp, nnz = rp.numel(), ci.numel()
            ptrs = (_ptr(rp), _ptr(ci), None if w is None else _ptr(w))
            flags = _abi.NVD_PTR_DEVICE
        else:
            rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
            ci = np.ascontiguousarray(col_idx, dtype=np.int32)
            w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
            nrp, nnz = rp.size, ci.size
            ptrs = (rp.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p),
                    None if w is None else w.ctypes.data_as(C.c_void_p))
            flags = _abi.NVD_PTR_HOST
        if w is not None and (w.numel() if on_dev else w.size) != nnz:
            raise ValueError("weights must have one entry per col_idx entry")
        self.n = int(nrp - 1 if n is None else n)
        if self.n != nrp - 1:
            raise ValueError("row_ptr must have n + 1 entries")
        self.nnz_in = int(nnz)
        h = C.c_void_p()
        st = lib.nvd_graph_create_ex(self.n, self.nnz_in, *ptrs, flags, _stream(), C.byref(h))
        check(st, "nvd_graph_create")
        self._h = h
        self.weighted = w is not None
        _live_graphs.add(self)

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
        """Y = L X for a CUDA tensor X (n,) or (n, k), float64 or float32;
        out: optional preallocated Y of the same shape and dtype."""
        torch = _torch()
        if not isinstance(X, torch.Tensor) or not X.is_cuda:
            raise ValueError("X must be a CUDA tensor")
        if X.dim() == 1:
            X = X.reshape(-1, 1)
            if out is not None:
                out = out.reshape(-1, 1)
        if X.dim() != 2 or X.shape[0] != self.n:
            raise ValueError(f"X must be ({self.n},) or ({self.n}, k)")
        if X.dtype not in (torch.float64, torch.float32):
            raise ValueError("X must be float64 or float32")
        if X.stride(1) != 1 or X.stride(0) < X.shape[1]:
            X = X.contiguous()
        dt = {torch.float64: NVD_DT_F64, torch.float32: NVD_DT_F32}[X.dtype]
        Y = torch.empty_like(X) if out is None else _check_out(out, "out", X.shape, X.dtype)
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
                  precond="jacobi", out="d", noalloc=False):
        """Returns (d, X or None, info list).  P, Q: (n, k) or (n,) float64.
        precond: "jacobi" (the diagonal), "tree" (a spanning forest, solved
        exactly), "auto" (the forest when at most n/100 edges lie off it,
        else the diagonal) or "achol" (an approximate Cholesky factor).  X0: starting guess, (n, k) like P.
        out: "d" for distances, "dsq" for their squares.
        noalloc: solve through nvd_distances_noalloc (no device allocation by
        the library; Jacobi only, n * tile up to about 1e6)."""
        torch = _torch()
        P = _as_dev64(P, "P")
        Q = _as_dev64(Q, "Q")
        if P.shape != Q.shape or P.shape[0] != self.n:
            raise ValueError(f"P, Q must both be ({self.n}, k)")
        if out not in ("d", "dsq"):
            raise ValueError("out must be 'd' or 'dsq'")
        k = P.shape[1]
        o = opts(precision, rtol, inner_rtol, max_iter, max_refine, tile_k, X0 is not None, precond)
        if out == "dsq":
            o.flags |= _abi.NVD_OUT_DSQ
        d = torch.empty(k, dtype=torch.float64, device=P.device)
        X = None
        if X0 is not None:
            X0 = _as_dev64(X0, "X0")
            if X0.shape != P.shape:
                raise ValueError(f"X0 must have the shape of P, {tuple(P.shape)}")
            X = X0.clone()
        elif return_x:
            X = torch.empty_like(P)
        info = (PairInfo * k)()
        fn = load().nvd_distances_noalloc if noalloc else load().nvd_distances
        st = fn(self._h, k, _ptr(P), _ptr(Q), P.stride(0), C.byref(o), _ptr(d), _ptr(X),
                X.stride(0) if X is not None else 0, info, _stream())
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
        """Replace the edge weights (float64, input CSR order)."""
        torch = _torch()
        w = torch.as_tensor(w).detach().to(device="cuda", dtype=torch.float64).reshape(-1).contiguous()
        if w.numel() != self.nnz_in:
            raise ValueError(f"w must have {self.nnz_in} entries (one per input CSR entry)")
        check(load().nvd_graph_set_weights(self._h, _ptr(w), _stream()), "nvd_graph_set_weights")
        self.weighted = True

    def _gscale(self, gscale, k, device):
        torch = _torch()
        g = torch.as_tensor(gscale).to(device=device, dtype=torch.float64).reshape(-1).contiguous()
        if g.numel() != k:
            raise ValueError(f"gscale must have one entry per column ({k})")
        return g

    def grad_weights(self, X, gscale):
        """-1/2 sum_j g_j (x_i - x_c)^2 for every input CSR entry (i, c)."""
        torch = _torch()
        X = _as_dev64(X, "X")
        if X.shape[0] != self.n:
            raise ValueError(f"X must be ({self.n}, k)")
        g = self._gscale(gscale, X.shape[1], X.device)
        out = torch.empty(self.nnz_in, dtype=torch.float64, device=X.device)
        check(load().nvd_grad_weights(self._h, X.shape[1], _ptr(X), X.stride(0), _ptr(g),
                                      _ptr(out), _stream()), "nvd_grad_weights")
        return out

    def grad_vectors(self, X, gscale, want_p=True, want_q=True):
        """(2 X diag(g), -2 X diag(g)): the gradients of sum_j g_j d_j^2 with
        respect to P and Q (None where not wanted)."""
        torch = _torch()
        X = _as_dev64(X, "X")
        if X.shape[0] != self.n:
            raise ValueError(f"X must be ({self.n}, k)")
        k = X.shape[1]
        g = self._gscale(gscale, k, X.device)
        GP = torch.empty_like(X) if want_p else None
        GQ = torch.empty_like(X) if want_q else None
        if GP is None and GQ is None:
            return None, None
        check(load().nvd_grad_vectors(self._h, k, _ptr(X), X.stride(0), _ptr(g), _ptr(GP),
                                      GP.stride(0) if GP is not None else 0, _ptr(GQ),
                                      GQ.stride(0) if GQ is not None else 0, _stream()),
              "nvd_grad_vectors")
        return GP, GQ


def grad_scale_from_d(g_d, d):
    """g_d / (2 d) where d > 0, else 0: an upstream gradient on distances
    turned into the scale on their squares (computed by the library)."""
    torch = _torch()
    d = torch.as_tensor(d).to(device="cuda", dtype=torch.float64).reshape(-1).contiguous()
    g = torch.as_tensor(g_d).to(device=d.device, dtype=torch.float64).reshape(-1).contiguous()
    if g.numel() != d.numel():
        raise ValueError("g_d and d must have the same length")
    out = torch.empty_like(d)
    check(load().nvd_grad_scale_from_d(d.numel(), _ptr(g), _ptr(d), _ptr(out), _stream()),
          "nvd_grad_scale_from_d")
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
        _live_batches.add(self)

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
        if len(ks) != len(self.graphs) or Pf.numel() != Qf.numel() or \
                Pf.numel() != int(sum(n * k for n, k in zip(self.ns, ks))):
            raise ValueError("packed P, Q must hold an (n_g, k_g) block for every graph of the batch")
        d = torch.empty(K, dtype=torch.float64, device="cuda") if out is None else \
            _check_out(out, "out", (K,), torch.float64)
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


from .autograd import DistanceSq, Distance, distance_sq, distance_t  # noqa: E402,F401
