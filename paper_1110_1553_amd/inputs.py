"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws random matrices; it holds none of the factorization's
arithmetic.  All matrices are float64 in column-major (Fortran) order.

* :func:`gaussian` -- iid N(0,1) entries, ``numpy.random.default_rng(seed)``.
* :func:`graded` -- U diag(sigma) V^T with sigma logspaced from 1 down to
  ``smin`` and Haar-distributed orthogonal U, V (QR of a Gaussian with the
  usual sign fix, by numpy's LAPACK binding); used for the ill-conditioned
  square workload.
"""
import numpy as np


def gaussian(M: int, N: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    # draw column by column so the first columns do not depend on N
    return np.asfortranarray(rng.standard_normal((N, M)).T)


def haar(n: int, rng) -> np.ndarray:
    Z = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    return Q * np.where(np.diagonal(R) < 0, -1.0, 1.0)


def graded(n: int, seed: int, smin: float = 1e-8, m: int = 0) -> np.ndarray:
    """m x n (m defaults to n) matrix U diag(sigma) V^T, sigma_i = smin^(i/(n-1))."""
    rng = np.random.default_rng(seed)
    m = m or n
    sigma = np.logspace(0.0, np.log10(smin), n)
    if m == n:
        U = haar(n, rng)
    else:
        U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V = haar(n, rng)
    return np.asfortranarray((U * sigma) @ V.T)
