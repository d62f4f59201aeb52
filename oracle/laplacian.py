"""Graph Laplacian L = D - A and connected components (paper, section 3.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions taken where the paper is silent (section 3.1 defines L only for
unit weights and says weights are positive reals):
* weights are conductances: A_uv = w_uv, D_uu = sum_v w_uv, L_uv = -w_uv;
* self-loops are dropped -- they would add w to D_uu and subtract it again
  through A_uu, so L is unchanged;
* an isolated node has an all-zero row and column and is its own component.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse import csr_matrix, diags

__all__ = ["laplacian_dense", "laplacian_sparse", "components", "project"]


def _entries(n, row_ptr, col_idx, w):
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col_idx, dtype=np.int64)
    row = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    val = np.ones(col.size) if w is None else np.asarray(w, dtype=np.float64)
    off = row != col
    return row[off], col[off], val[off]


def laplacian_dense(n, row_ptr, col_idx, w=None):
    """Dense FP64 L = D - A from a symmetric CSR adjacency."""
    row, col, val = _entries(n, row_ptr, col_idx, w)
    A = np.zeros((n, n))
    np.add.at(A, (row, col), val)
    D = np.diag(A.sum(axis=1))
    return D - A


def laplacian_sparse(n, row_ptr, col_idx, w=None):
    """SciPy CSR FP64 L = D - A."""
    row, col, val = _entries(n, row_ptr, col_idx, w)
    A = csr_matrix((val, (row, col)), shape=(n, n))
    deg = np.asarray(A.sum(axis=1)).ravel()
    return (diags(deg) - A).tocsr()


def components(n, row_ptr, col_idx):
    """Connected components by breadth-first search.

    Returns labels (int64 [n]) numbered 0, 1, ... in order of each
    component's smallest node id.
    """
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col_idx, dtype=np.int64)
    lab = np.full(n, -1, dtype=np.int64)
    cur = 0
    for s in range(n):
        if lab[s] >= 0:
            continue
        lab[s] = cur
        frontier = np.array([s], dtype=np.int64)
        while frontier.size:
            starts = row_ptr[frontier]
            ends = row_ptr[frontier + 1]
            cnt = ends - starts
            if cnt.sum() == 0:
                break
            idx = np.repeat(starts - np.cumsum(np.concatenate([[0], cnt[:-1]])), cnt) \
                + np.arange(cnt.sum())
            nb = np.unique(col[idx])
            nb = nb[lab[nb] < 0]
            lab[nb] = cur
            frontier = nb
        cur += 1
    return lab


def project(delta, labels):
    """Remove the per-component mean from each column of delta (n x k):
    delta_bar = delta - sum_C (1_C^T delta / |C|) 1_C."""
    delta = np.asarray(delta, dtype=np.float64)
    nc = int(labels.max()) + 1 if labels.size else 0
    out = delta.copy()
    size = np.bincount(labels, minlength=nc).astype(np.float64)
    for j in range(delta.shape[1]):
        s = np.bincount(labels, weights=delta[:, j], minlength=nc)
        out[:, j] -= (s / size)[labels]
    return out
