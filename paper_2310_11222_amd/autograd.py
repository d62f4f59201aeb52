"""Differentiable GE distances (torch.autograd), backed by the library's
forward solve and hand-written adjoint.

For d_j^2 = delta_j^T L^+ delta_j with delta_j = p_j - q_j and x_j = L^+ delta_j
(the mean-zero solution the forward solve returns):
    d(d_j^2)/dp_j = 2 x_j,   d(d_j^2)/dq_j = -2 x_j,
    d(d_j^2)/dw_e = -(x_ij - x_kj)^2  for an undirected edge e = {i, k}.
The backward reuses the saved x (no second solve: L^+ is symmetric) and the
library's nvd_grad_weights kernel, which reports -1/2 (x_i - x_k)^2 per CSR
entry; when the CSR weights are gathered from a per-edge tensor
(w_csr = w_edge[csr_edge]), autograd adds the two stored directions and the
edge receives the full derivative.
"""
from __future__ import annotations

import torch


class DistanceSq(torch.autograd.Function):
    """dsq = DistanceSq.apply(P, Q, w_csr, graph, opts) -> (k,) squared distances.

    P, Q: (n, k) float64 CUDA tensors; w_csr: (nnz,) float64 CUDA tensor of
    edge weights in the graph's input CSR order, or None to keep the graph's
    weights; opts: dict of Graph.distances keyword arguments.
    """

    @staticmethod
    def forward(ctx, P, Q, w_csr, graph, opts=None):
        opts = dict(opts or {})
        opts.setdefault("precision", "fp64")
        if w_csr is not None:
            graph.set_weights(w_csr)
        d, X, info = graph.distances(P.detach(), Q.detach(), return_x=True, **opts)
        ctx.save_for_backward(X)
        ctx.graph = graph
        ctx.has_w = w_csr is not None
        ctx.info = info
        return d * d

    @staticmethod
    def backward(ctx, g):
        (X,) = ctx.saved_tensors
        g = g.to(dtype=torch.float64).contiguous()
        gp = 2.0 * X * g[None, :]
        gw = None
        if ctx.has_w and ctx.needs_input_grad[2]:
            gw = ctx.graph.grad_weights(X, g)
        return gp, -gp, gw, None, None


def distance_sq(P, Q, graph, w_csr=None, **opts):
    """Squared distances with gradients to P, Q and (optionally) w_csr."""
    return DistanceSq.apply(P, Q, w_csr, graph, opts)


class _SafeSqrt(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        y = torch.sqrt(torch.clamp(x, min=0.0))
        ctx.save_for_backward(y)
        return y

    @staticmethod
    def backward(ctx, g):
        (y,) = ctx.saved_tensors
        # d sqrt(s)/ds = 1 / (2 sqrt(s)); defined as 0 where the distance is 0
        safe = torch.where(y > 0, 0.5 / torch.where(y > 0, y, torch.ones_like(y)),
                           torch.zeros_like(y))
        return g * safe


def distance_t(P, Q, graph, w_csr=None, **opts):
    """Distances d = sqrt(d^2) with gradients (zero gradient where d = 0)."""
    return _SafeSqrt.apply(distance_sq(P, Q, graph, w_csr, **opts))
