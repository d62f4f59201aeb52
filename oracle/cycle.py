"""Route O5: exact GE distance on a cycle with one common edge weight w.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The cycle Laplacian is circulant, so the Fourier modes diagonalise it with
eigenvalues lam_k = w (2 - 2 cos(2 pi k / n)) = 4 w sin^2(pi k / n),
k = 0..n-1 (lam_0 = 0 is the constant mode).  With delta_hat = unnormalised
DFT of delta = a - b, d^2 = (1/n) sum_{k=1}^{n-1} |delta_hat_k|^2 / lam_k.
The eigenvalues are evaluated in the sine form: 2 - 2 cos cancels for the
smallest k, whose 1/lam_k dominate the sum (at n = 2e5 the cosine form
loses about seven digits of lam_1).
NumPy's FFT is the only library step.  Node i of the cycle is adjacent to
i-1 and i+1 (mod n).
"""
from __future__ import annotations

import numpy as np

__all__ = ["ge_cycle"]


def ge_cycle(n, P, Q, w=1.0):
    P = np.asarray(P, dtype=np.float64).reshape(n, -1)
    Q = np.asarray(Q, dtype=np.float64).reshape(n, -1)
    dh = np.fft.fft(P - Q, axis=0)
    kk = np.arange(1, n)
    lam = 4.0 * w * np.sin(np.pi * kk / n) ** 2
    dsq = np.sum(np.abs(dh[1:]) ** 2 / lam[:, None], axis=0) / n
    return {"d": np.sqrt(dsq), "dsq": dsq}
