"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws random matrices; it holds none of the factorization's
arithmetic.  All matrices are float64 and column-major: numpy arrays in
Fortran order, torch tensors of shape (M, N) with strides (1, M).

* :func:`gaussian` / :func:`gaussian_device` -- iid N(0,1) entries
  (numpy ``default_rng(seed)`` on the host; torch's seeded Philox generator
  on the device for the large benchmark matrices).
* :func:`graded` / :func:`graded_device` -- U diag(sigma) V^T with sigma
  logspaced from 1 down to ``smin`` and random orthogonal U, V.  U and V are
  exponentials of random skew-symmetric matrices (exp(K) with K = -K^T is
  orthogonal), so no QR is involved in making the input.
"""
import numpy as np


def gaussian(M: int, N: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    # drawn column by column, so the leading columns do not depend on N
    return np.asfortranarray(rng.standard_normal((N, M)).T)


def gaussian_device(M: int, N: int, seed: int, device="cuda"):
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return torch.randn((N, M), generator=g, device=device, dtype=torch.float64).t()


def _skew(n: int, rng) -> np.ndarray:
    S = rng.standard_normal((n, n)) * (1.5 / np.sqrt(2.0 * n))
    return S - S.T


def orthogonal(n: int, rng) -> np.ndarray:
    import scipy.linalg

    return scipy.linalg.expm(_skew(n, rng))


def graded(n: int, seed: int, smin: float = 1e-8) -> np.ndarray:
    """n x n matrix U diag(sigma) V^T, sigma_i = smin^(i/(n-1))."""
    rng = np.random.default_rng(seed)
    sigma = np.logspace(0.0, np.log10(smin), n)
    U = orthogonal(n, rng)
    V = orthogonal(n, rng)
    return np.asfortranarray((U * sigma) @ V.T)


def graded_device(n: int, seed: int, smin: float = 1e-8, device="cuda"):
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)

    def orth():
        S = torch.randn((n, n), generator=g, device=device, dtype=torch.float64) * (1.5 / (2.0 * n) ** 0.5)
        return torch.linalg.matrix_exp(S - S.t())

    sigma = torch.logspace(0.0, float(np.log10(smin)), n, device=device, dtype=torch.float64)
    U = orth()
    V = orth()
    # row-major V (U diag(sigma))^T is the column-major storage of U diag(sigma) V^T
    At = V @ (U * sigma).t()
    return At.t()


def request_shapes(count: int, seed: int, mlo: int = 256, mhi: int = 16384, nlo: int = 32, nhi: int = 512):
    """(m, n) int64 arrays of `count` request shapes, m >= n."""
    rng = np.random.default_rng(seed)
    m = np.zeros(count, dtype=np.int64)
    n = np.zeros(count, dtype=np.int64)
    for q in range(count):
        while True:
            mq = int(rng.integers(mlo, mhi + 1))
            nq = int(rng.integers(nlo, nhi + 1))
            if mq >= nq:
                break
        m[q], n[q] = mq, nq
    return m, n


def arrival_gaps(count: int, rate: float, seed: int) -> np.ndarray:
    """Exponential inter-arrival times (seconds) of a Poisson stream."""
    return np.random.default_rng(seed).exponential(1.0 / rate, count)


def graded_tall_device(M: int, N: int, seed: int, smin: float = 1e-6, device="cuda"):
    """M x N (M >= N) column-major U diag(sigma) V^T, condition number 1/smin."""
    import math

    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    cols = torch.randperm(M, generator=g, device=device)[:N].to(torch.float64)
    signs = torch.randint(0, 2, (M,), generator=g, device=device).to(torch.float64) * 2.0 - 1.0
    i = torch.arange(M, device=device, dtype=torch.float64) + 0.5
    # orthonormal DCT-II basis vectors: c_j(i) = s_j cos(pi (i + 1/2) j / M), s_0 = sqrt(1/M), s_j = sqrt(2/M)
    scale = torch.where(cols == 0, torch.full_like(cols, math.sqrt(1.0 / M)), torch.full_like(cols, math.sqrt(2.0 / M)))
    U = torch.cos(math.pi * i[:, None] * cols[None, :] / M) * scale[None, :] * signs[:, None]
    S = torch.randn((N, N), generator=g, device=device, dtype=torch.float64) * (1.5 / (2.0 * N) ** 0.5)
    V = torch.linalg.matrix_exp(S - S.t())
    sigma = torch.logspace(0.0, float(np.log10(smin)), N, device=device, dtype=torch.float64)
    At = V @ (U * sigma).t()  # row-major N x M = column-major M x N
    return At.t()
