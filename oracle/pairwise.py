"""All pairwise distances among m node vectors (test infrastructure only).

Many phenomena, or one phenomenon observed at many times, are compared on the
same network (introduction; section 5.2 compares regions, airlines,
countries, community pairs and categories).  For node vectors v_1 .. v_m the
oracle writes out the section 3.1 definition for every pair:

    D[i, j] = sqrt((v_i - v_j)^T L^+ (v_i - v_j)),   D[i, i] = 0.

Two routes, sharing nothing but the Laplacian helpers:

* ``pairwise_dense`` -- L^+ from the full eigendecomposition of L (the c null
  eigenpairs dropped, c = number of components): with U the remaining
  eigenvectors and lam their eigenvalues, (v_i - v_j)^T L^+ (v_i - v_j) =
  sum_k (u_k^T v_i - u_k^T v_j)^2 / lam_k, evaluated pair by pair.
* ``pairwise_pcg``   -- the FP64 PCG route applied to the m(m-1)/2 pair
  differences as separate right-hand sides (for graphs the dense route
  cannot hold).
"""
import numpy as np

from .laplacian import laplacian_dense, components
from .pcg import ge_pcg


def _pairs(m):
    iu, ju = np.triu_indices(m, k=1)
    return iu, ju


def pairwise_dense(n, row_ptr, col_idx, w, V):
    """D (m x m) through L^+ = U diag(1/lam) U^T on the non-null eigenpairs."""
    V = np.asarray(V, dtype=np.float64).reshape(n, -1)
    m = V.shape[1]
    L = laplacian_dense(n, row_ptr, col_idx, w)
    c = int(components(n, row_ptr, col_idx).max()) + 1
    lam, U = np.linalg.eigh(L)
    coef = U[:, c:].T @ V                      # eigen-coordinates of every v_i
    D = np.zeros((m, m))
    for i in range(m):
        for j in range(i + 1, m):
            diff = coef[:, i] - coef[:, j]
            dsq = max(float(np.sum(diff * diff / lam[c:])), 0.0)
            D[i, j] = D[j, i] = np.sqrt(dsq)
    return D


def pairwise_pcg(n, row_ptr, col_idx, w, V, rtol=1e-13):
    """D (m x m) from one FP64 PCG solve per pair difference."""
    V = np.asarray(V, dtype=np.float64).reshape(n, -1)
    m = V.shape[1]
    iu, ju = _pairs(m)
    r = ge_pcg(n, row_ptr, col_idx, w, V[:, iu], V[:, ju], rtol=rtol)
    D = np.zeros((m, m))
    D[iu, ju] = r["d"]
    D[ju, iu] = r["d"]
    return D
