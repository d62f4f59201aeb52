"""Route O1: the GE distance straight from its definition (paper, section 3.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

d(a, b)^2 = (a-b)^T L^+ (a-b), with L^+ the Moore-Penrose pseudoinverse.  The
paper's exact baseline obtains L^+ by SVD; L is symmetric positive
semidefinite, so its SVD is its eigendecomposition L = U diag(lam) U^T and
L^+ = U diag(lam^+) U^T, where lam^+ inverts the nonzero eigenvalues and keeps
the zero ones at zero.

Reading (the paper gives no threshold for "zero"): the number of zero
eigenvalues of a graph Laplacian equals the number c of connected components,
so exactly the c smallest eigenpairs are dropped (c from breadth-first
search), never an rcond cut-off.
"""
from __future__ import annotations

import numpy as np

from .laplacian import laplacian_dense, components

__all__ = ["ge_dense"]


def ge_dense(n, row_ptr, col_idx, w, P, Q):
    """Distances for every column pair of P, Q (n x k) on one graph.

    Returns dict with d (k,), dsq (k,), x = L^+ (P - Q) (n x k) and the
    eigenvalues used.
    """
    P = np.asarray(P, dtype=np.float64).reshape(n, -1)
    Q = np.asarray(Q, dtype=np.float64).reshape(n, -1)
    delta = P - Q
    L = laplacian_dense(n, row_ptr, col_idx, w)
    lab = components(n, row_ptr, col_idx)
    c = int(lab.max()) + 1 if n else 0
    lam, U = np.linalg.eigh(L)
    coef = U[:, c:].T @ delta                      # eigen-coordinates of delta
    dsq = np.sum(coef * coef / lam[c:, None], axis=0)
    x = U[:, c:] @ (coef / lam[c:, None])
    dsq = np.maximum(dsq, 0.0)
    return {"d": np.sqrt(dsq), "dsq": dsq, "x": x, "lam": lam, "ncomp": c,
            "labels": lab}
