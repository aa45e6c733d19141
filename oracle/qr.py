"""Householder QR oracle (test infrastructure only).

Wraps ``qr_oracle.c`` (an unblocked double-precision Householder QR, one
reflector per column, LAPACK geqr2 conventions) and adds helpers that are
plain definitions on top of it:

* ``factor(A)``        -> (QR-in-place array, tau)
* ``r_factor(A)``      -> upper-triangular R (min(M,N) x N)
* ``sign_normalize(R)``-> D R with D = diag(sign(R_ii)), sign(0) = +1; R is
                          unique up to these signs for a full-rank A, so
                          every elimination list must agree with the oracle
                          after this normalisation (Section II: any list
                          performs the same algebra in another order).
* ``apply_qt / apply_q / thin_q`` -- the implicit Q from the reflectors.
* ``lstsq(A, b)``      -> x = R^{-1} (Q^T b)[:N] (triangular solve by scipy).

Everything is float64.  Arrays cross the ctypes boundary in Fortran
(column-major) order.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        i64, dp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        lib.oracle_geqr2.argtypes = [i64, i64, dp, i64, dp, ctypes.c_int]
        lib.oracle_geqr2.restype = ctypes.c_int
        for name in ("oracle_apply_qt", "oracle_apply_q"):
            f = getattr(lib, name)
            f.argtypes = [i64, i64, dp, i64, dp, dp, i64, i64]
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def factor(A, nthreads: int = 0):
    """Householder QR of A (M x N).  Returns (F, tau): F holds R in its upper
    triangle and the reflector tails below the diagonal (column-major)."""
    F = np.array(A, dtype=np.float64, order="F", copy=True)
    m, n = F.shape
    tau = np.zeros(min(m, n), dtype=np.float64)
    rc = _load().oracle_geqr2(m, n, _dp(F), max(m, 1), _dp(tau), nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_geqr2 rejected its arguments")
    return F, tau


def r_of(F):
    m, n = F.shape
    return np.triu(F[: min(m, n), :])


def r_factor(A, nthreads: int = 0):
    F, _ = factor(A, nthreads)
    return r_of(F)


def sign_normalize(R):
    """D R with D = diag(sign(R_ii)), sign(0) = +1."""
    R = np.asarray(R, dtype=np.float64)
    d = np.where(np.diagonal(R) < 0, -1.0, 1.0)
    return R * d[:, None]


def apply_qt(F, tau, B):
    B2 = np.array(B, dtype=np.float64, order="F", copy=True)
    if B2.ndim == 1:
        B2 = B2.reshape(-1, 1, order="F")
    m, n = F.shape
    rc = _load().oracle_apply_qt(m, n, _dp(F), max(m, 1), _dp(tau), _dp(B2), max(m, 1), B2.shape[1])
    if rc != 0:
        raise ValueError("oracle_apply_qt rejected its arguments")
    return B2


def apply_q(F, tau, B):
    B2 = np.array(B, dtype=np.float64, order="F", copy=True)
    if B2.ndim == 1:
        B2 = B2.reshape(-1, 1, order="F")
    m, n = F.shape
    rc = _load().oracle_apply_q(m, n, _dp(F), max(m, 1), _dp(tau), _dp(B2), max(m, 1), B2.shape[1])
    if rc != 0:
        raise ValueError("oracle_apply_q rejected its arguments")
    return B2


def thin_q(F, tau):
    """The first min(M,N) columns of Q = H_0 ... H_{k-1}."""
    m, n = F.shape
    k = min(m, n)
    E = np.zeros((m, k), dtype=np.float64, order="F")
    E[np.arange(k), np.arange(k)] = 1.0
    return apply_q(F, tau, E)


def lstsq(A, b, nthreads: int = 0):
    """Least-squares solution of min ||A x - b|| for full-rank A (M >= N)."""
    import scipy.linalg

    F, tau = factor(A, nthreads)
    n = F.shape[1]
    c = apply_qt(F, tau, b)
    x = scipy.linalg.solve_triangular(np.triu(F[:n, :n]), c[:n], lower=False)
    return x
