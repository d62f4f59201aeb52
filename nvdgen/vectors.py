"""Seeded node-vector pairs and edge weights (host side, NumPy).

Node vectors are the paper's a, b in R^|V| (section 3.1).  Each pair (p, q)
gets values on independent random supports and zeros elsewhere.  The output
is stored row-major n x k (one column per pair), the layout the library reads.
"""
from __future__ import annotations

import numpy as np

__all__ = ["sparse_support_pairs", "uniform_weights", "lognormal_weights"]


def _support(n, count, rng):
    if count >= n:
        return np.arange(n)
    return np.sort(rng.permutation(n)[:count])


def sparse_support_pairs(n, k, frac, rng, dist="uniform"):
    """k pairs of node vectors.  For every pair, p and q each take
    floor(frac*n) nodes drawn without replacement (independently) and put
    uniform[0,1) values (dist="uniform") or standard normal values
    (dist="normal") there; all other entries are zero.

    Returns P, Q as float64 arrays of shape (n, k), C-contiguous.
    """
    n = int(n)
    cnt = max(1, int(np.floor(frac * n)))
    P = np.zeros((n, k), dtype=np.float64)
    Q = np.zeros((n, k), dtype=np.float64)
    for j in range(k):
        for M in (P, Q):
            s = _support(n, cnt, rng)
            if dist == "uniform":
                vals = rng.random(s.size)
            elif dist == "normal":
                vals = rng.standard_normal(s.size)
            else:
                raise ValueError(dist)
            M[s, j] = vals
    return P, Q


def uniform_weights(m, lo, hi, rng):
    """m iid edge weights uniform on [lo, hi)."""
    return lo + (hi - lo) * rng.random(int(m))


def lognormal_weights(m, rng, mu=0.0, sigma=1.0):
    """m iid edge weights lognormal(mu, sigma)."""
    return rng.lognormal(mu, sigma, size=int(m))
