"""Route O2: grounded (Dirichlet) solve -- an exact route independent of O1.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For each connected component C, remove the mean of delta = a - b on C
(the part of delta outside the range of L, which L^+ maps to zero), pick the
lowest-numbered node g of C, delete row and column g from L_CC (the result is
symmetric positive definite for a connected C), solve for the other entries
with x_g = 0, and use delta_bar^T x = delta^T L^+ delta (x differs from
L^+ delta only by a constant on C, which delta_bar is orthogonal to).
Dense Cholesky for small components, sparse LU otherwise.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import cho_factor, cho_solve
from scipy.sparse.linalg import splu

from .laplacian import laplacian_dense, laplacian_sparse, components, project

__all__ = ["ge_grounded"]


def ge_grounded(n, row_ptr, col_idx, w, P, Q, sparse=None):
    P = np.asarray(P, dtype=np.float64).reshape(n, -1)
    Q = np.asarray(Q, dtype=np.float64).reshape(n, -1)
    lab = components(n, row_ptr, col_idx)
    dbar = project(P - Q, lab)
    if sparse is None:
        sparse = n > 4000
    L = laplacian_sparse(n, row_ptr, col_idx, w) if sparse else \
        laplacian_dense(n, row_ptr, col_idx, w)
    x = np.zeros_like(dbar)
    for c in range(int(lab.max()) + 1 if n else 0):
        nodes = np.nonzero(lab == c)[0]
        if nodes.size == 1:
            continue
        rest = nodes[1:]                      # ground the lowest node id
        if sparse:
            Lg = L[rest][:, rest].tocsc()
            lu = splu(Lg, permc_spec="COLAMD")
            x[rest] = lu.solve(dbar[rest])
        else:
            Lg = L[np.ix_(rest, rest)]
            x[rest] = cho_solve(cho_factor(Lg), dbar[rest])
    # canonical output: per-component mean-zero x (= L^+ delta)
    x = project(x, lab)
    dsq = np.maximum(np.sum(dbar * x, axis=0), 0.0)
    return {"d": np.sqrt(dsq), "dsq": dsq, "x": x, "labels": lab}
