"""Route O3: textbook Jacobi-preconditioned CG in FP64 (paper, section 3.2:
the distance through a Laplacian solve of L x = a - b instead of L^+).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Used where the exact routes cannot go (n beyond ~1e4).  Each column of the
right-hand side is an independent CG run (Hestenes-Stiefel form, preconditioner
M = D, i.e. z = r / deg, zero on isolated nodes), from x0 = 0, on the
per-component projected right-hand side delta_bar (the system L x = delta is
consistent only after that projection).  Stops when the TRUE relative
residual ||delta_bar - L x|| / ||delta_bar|| is <= rtol (checked every
``check_every`` steps and at the end) or after max_iter steps.

Returned value (reading; the paper only says "solve, then take the quadratic
form"): J(x) = delta_bar^T x + x^T r with r = delta_bar - L x.  For any x,
d^2 - J(x) = (x* - x)^T L (x* - x) >= 0, so J is a lower bound whose error is
quadratic in the residual; for plain CG from zero it equals delta_bar^T x up to
rounding.  SciPy's sparse product is the only library step.
"""
from __future__ import annotations

import numpy as np

from .laplacian import laplacian_sparse, components, project

__all__ = ["ge_pcg", "pcg_solve"]


def pcg_solve(L, deg, b, rtol=1e-13, max_iter=100000, check_every=10,
              stall_checks=50):
    """Independent Jacobi-PCG per column of b (n x k).  Returns x, the
    iteration count per column, the final true relative residual and the
    true residual itself.

    A column also stops when its true residual has not reached a new minimum
    for ``stall_checks`` consecutive checks (the attainable accuracy of CG in
    floating point is about eps * cond(L), which can sit above rtol); it then
    keeps the iterate with the smallest true residual seen."""
    n, k = b.shape
    inv = np.zeros(n)
    nz = deg > 0
    inv[nz] = 1.0 / deg[nz]
    bnorm = np.linalg.norm(b, axis=0)
    x = np.zeros_like(b)
    r = b.copy()
    z = r * inv[:, None]
    p = z.copy()
    rho = np.sum(r * z, axis=0)
    active = bnorm > 0
    iters = np.zeros(k, dtype=np.int64)
    relres = np.zeros(k)
    best = np.full(k, np.inf)
    best_x = x.copy()
    stall = np.zeros(k, dtype=np.int64)
    it = 0
    while active.any() and it < max_iter:
        cols = np.nonzero(active)[0]
        q = L @ p[:, cols]
        pq = np.sum(p[:, cols] * q, axis=0)
        # exact convergence (rho = 0) or loss of positivity: stop that column
        stop = ~(pq > 0) | ~(rho[cols] > 0)
        if stop.any():
            active[cols[stop]] = False
            keep = ~stop
            cols, q, pq = cols[keep], q[:, keep], pq[keep]
            if cols.size == 0:
                break
        alpha = rho[cols] / pq
        x[:, cols] += alpha * p[:, cols]
        r[:, cols] -= alpha * q
        z_c = r[:, cols] * inv[:, None]
        rho_new = np.sum(r[:, cols] * z_c, axis=0)
        beta = rho_new / rho[cols]
        p[:, cols] = z_c + beta * p[:, cols]
        rho[cols] = rho_new
        iters[cols] += 1
        it += 1
        if it % check_every == 0 or it == max_iter:
            tr = b[:, cols] - L @ x[:, cols]
            rr = np.linalg.norm(tr, axis=0) / bnorm[cols]
            relres[cols] = rr
            better = rr < best[cols]
            bc = cols[better]
            best[bc] = rr[better]
            best_x[:, bc] = x[:, bc]
            stall[bc] = 0
            stall[cols[~better]] += 1
            done = (rr <= rtol) | (stall[cols] >= stall_checks)
            active[cols[done]] = False
            x[:, cols[done]] = best_x[:, cols[done]]
    # final true residual for every column
    tr = b - L @ x
    relres = np.where(bnorm > 0, np.linalg.norm(tr, axis=0) / np.where(bnorm > 0, bnorm, 1), 0.0)
    return x, iters, relres, tr


def ge_pcg(n, row_ptr, col_idx, w, P, Q, rtol=1e-13, max_iter=100000):
    P = np.asarray(P, dtype=np.float64).reshape(n, -1)
    Q = np.asarray(Q, dtype=np.float64).reshape(n, -1)
    lab = components(n, row_ptr, col_idx)
    dbar = project(P - Q, lab)
    L = laplacian_sparse(n, row_ptr, col_idx, w)
    deg = L.diagonal()
    x, iters, relres, r = pcg_solve(L, deg, dbar, rtol=rtol, max_iter=max_iter)
    # x is defined up to a constant per component; fix it to mean zero before
    # forming J so that the rounding-level component of r along the constant
    # vector is not multiplied by an arbitrary offset
    x = project(x, lab)
    r = dbar - L @ x
    J = np.sum(dbar * x, axis=0) + np.sum(x * r, axis=0)
    dsq = np.maximum(J, 0.0)
    return {"d": np.sqrt(dsq), "dsq": dsq, "x": x,
            "iters": iters, "relres": relres, "labels": lab}
