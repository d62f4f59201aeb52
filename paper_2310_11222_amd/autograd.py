"""Differentiable GE distances (torch.autograd), backed by the library's
forward solve and hand-written adjoint kernels.

For d_j^2 = delta_j^T L^+ delta_j with delta_j = p_j - q_j and x_j = L^+ delta_j
(the mean-zero solution the forward solve returns):
    d(d_j^2)/dp_j = 2 x_j,   d(d_j^2)/dq_j = -2 x_j,
    d(d_j^2)/dw_e = -(x_ij - x_kj)^2  for an undirected edge e = {i, k}.
The backward reuses the saved x (no second solve: L^+ is symmetric).  Every
number is computed by the library: the forward returns d or d^2
(NVD_OUT_DSQ), nvd_grad_vectors forms 2 X diag(g) and its negative,
nvd_grad_weights reports -1/2 (x_i - x_k)^2 per CSR entry (when the CSR
weights are gathered from a per-edge tensor, w_csr = w_edge[csr_edge],
autograd adds the two stored directions and the edge receives the full
derivative), and nvd_grad_scale_from_d turns an upstream gradient on d into
the scale on d^2, g / (2 d), zero where d = 0.  This module only marshals
tensors between autograd and the library.
"""
from __future__ import annotations

import torch


def _forward(ctx, P, Q, w_csr, graph, opts, out):
    opts = dict(opts or {})
    opts.setdefault("precision", "fp64")
    if w_csr is not None:
        graph.set_weights(w_csr)
    val, X, info = graph.distances(P.detach(), Q.detach(), return_x=True, out=out, **opts)
    ctx.graph = graph
    ctx.has_w = w_csr is not None
    ctx.info = info
    return val, X


def _backward(ctx, X, gscale):
    gP, gQ = ctx.graph.grad_vectors(X, gscale, want_p=ctx.needs_input_grad[0],
                                    want_q=ctx.needs_input_grad[1])
    gw = None
    if ctx.has_w and ctx.needs_input_grad[2]:
        gw = ctx.graph.grad_weights(X, gscale)
    return gP, gQ, gw, None, None


class DistanceSq(torch.autograd.Function):
    """dsq = DistanceSq.apply(P, Q, w_csr, graph, opts) -> (k,) squared distances.

    P, Q: (n, k) float64 CUDA tensors; w_csr: (nnz,) float64 CUDA tensor of
    edge weights in the graph's input CSR order, or None to keep the graph's
    weights; opts: dict of Graph.distances keyword arguments.
    """

    @staticmethod
    def forward(ctx, P, Q, w_csr, graph, opts=None):
        dsq, X = _forward(ctx, P, Q, w_csr, graph, opts, "dsq")
        ctx.save_for_backward(X)
        return dsq

    @staticmethod
    def backward(ctx, g):
        (X,) = ctx.saved_tensors
        return _backward(ctx, X, g)


class Distance(torch.autograd.Function):
    """d = Distance.apply(P, Q, w_csr, graph, opts) -> (k,) distances, with
    the gradient of d defined as zero where d = 0 (arguments as DistanceSq)."""

    @staticmethod
    def forward(ctx, P, Q, w_csr, graph, opts=None):
        d, X = _forward(ctx, P, Q, w_csr, graph, opts, "d")
        ctx.save_for_backward(X, d)
        return d

    @staticmethod
    def backward(ctx, g):
        from . import grad_scale_from_d
        X, d = ctx.saved_tensors
        return _backward(ctx, X, grad_scale_from_d(g, d))


def distance_sq(P, Q, graph, w_csr=None, **opts):
    """Squared distances with gradients to P, Q and (optionally) w_csr."""
    return DistanceSq.apply(P, Q, w_csr, graph, opts)


def distance_t(P, Q, graph, w_csr=None, **opts):
    """Distances d with gradients (zero gradient where d = 0)."""
    return Distance.apply(P, Q, w_csr, graph, opts)
