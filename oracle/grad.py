"""Gradients of d^2 = delta^T L^+ delta (paper, section 3.1), delta = a - b.

TEST INFRASTRUCTURE ONLY (see the package docstring).

With x = L^+ delta (per-component mean-zero):
* d(d^2)/da = 2 x and d(d^2)/db = -2 x, since L^+ is symmetric;
* for an undirected edge e = {i, j} with weight w_e, L = sum_e w_e
  (e_i - e_j)(e_i - e_j)^T and d(L^+)/dw_e = -L^+ (e_i - e_j)(e_i - e_j)^T L^+
  on the fixed range of L, so d(d^2)/dw_e = -(x_i - x_j)^2.
Per CSR entry (each edge is stored twice) the value reported is half of that,
-(x_i - x_j)^2 / 2, so that summing both stored directions gives the edge's
derivative.
"""
from __future__ import annotations

import numpy as np

from .dense import ge_dense

__all__ = ["grad_dense", "grad_from_x"]


def grad_from_x(n, row_ptr, col_idx, x, gscale=None):
    """Gradients from a solution x (n x k) and upstream weights gscale (k,)
    = dLoss/d(d_k^2).  Returns (grad_p (n x k), grad_w_csr (nnz,))."""
    x = np.asarray(x, dtype=np.float64).reshape(n, -1)
    k = x.shape[1]
    g = np.ones(k) if gscale is None else np.asarray(gscale, dtype=np.float64)
    row = np.repeat(np.arange(n), np.diff(np.asarray(row_ptr, dtype=np.int64)))
    col = np.asarray(col_idx, dtype=np.int64)
    diff = x[row] - x[col]
    gw = -0.5 * np.sum(g[None, :] * diff * diff, axis=1)
    gw[row == col] = 0.0
    return 2.0 * x * g[None, :], gw


def grad_dense(n, row_ptr, col_idx, w, P, Q, gscale=None):
    r = ge_dense(n, row_ptr, col_idx, w, P, Q)
    gp, gw = grad_from_x(n, row_ptr, col_idx, r["x"], gscale)
    return {"dsq": r["dsq"], "grad_p": gp, "grad_q": -gp, "grad_w_csr": gw,
            "x": r["x"]}
