"""Parity of the benchmarked factorizations at their full sizes.

* 131072 x 2048 iid N(0,1) (seed 2), nb = 256, with the benchmark's
  hierarchical tree (TS domains of 4, Greedy low level, domino coupling,
  Fibonacci high level, 8 virtual clusters): the sign-normalised R against
  the oracle's unblocked Householder QR of the same bytes, relative Frobenius
  error <= 1e-12.  The same tree on the 16384 x 2048 leading block.
* 16384 x 16384 U diag(sigma) V^T with sigma logspaced 1 .. 1e-8 (seed 3),
  nb = 256, FlatTree with TS kernels and Greedy with TT kernels.  The oracle
  would take minutes on the host, so R is checked where it can be computed
  one block at a time and through properties that hold at any size:
  - the leading 768 columns of R (three tile columns, all 64 tile rows) are
    the R of the leading 768 columns of A: oracle, <= 1e-12;
  - R^T R = A^T A and Q R = A (Q applied by hqr_apply_q to [R; 0]), relative
    to ||A||_F^2 and ||A||_F: <= 1e-12 (Householder QR is backward stable);
  - the two trees give the same R: <= 1e-12.
"""
import os
import sys

import numpy as np
import pytest

from oracle import qr as oq
from paper_1110_1553_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12
SPIN = 20000000
HQR_TALL = dict(nb=256, p=8, a=4, low="greedy", high="fibonacci", coupling="chain", domino=1)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def threads():
    return max(1, min(16, os.cpu_count() or 1))


def rel_err(R_gpu, R_ref):
    a, b = oq.sign_normalize(R_gpu), oq.sign_normalize(R_ref)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def gpu_r(dA, N):
    return np.triu(dA[:N, :N].cpu().numpy())


@pytest.mark.timeout(600)
@pytest.mark.parametrize("M", [16384, 131072])
def test_tall_hierarchical_full_size(cuda, M):
    import torch

    import paper_1110_1553_amd as h

    N = 2048
    say("case tall hierarchical %dx%d nb 256 %s" % (M, N, HQR_TALL))
    A0 = inputs.gaussian_device(131072, N, 2, cuda)[:M]
    dA = h.colmajor(A0)
    A_host = np.asfortranarray(dA.cpu().numpy())
    del A0
    h.factor(dA, h.make_params(**HQR_TALL), h.make_exec(spin_limit=SPIN), timeout_s=120.0)
    torch.cuda.synchronize()
    R = gpu_r(dA, N)
    del dA
    torch.cuda.empty_cache()
    say("  oracle on %d threads" % threads())
    Rref = oq.r_factor(A_host, nthreads=threads())
    err = rel_err(R, Rref)
    say("  rel err %.3e" % err)
    assert err <= TOL


@pytest.fixture(scope="module")
def graded16k(cuda):
    import paper_1110_1553_amd as h

    say("input 16384^2 graded, sigma 1..1e-8, seed 3")
    A = h.colmajor(inputs.graded_device(16384, 3, 1e-8, cuda))
    return A


@pytest.fixture(scope="module")
def square_results(cuda, graded16k):
    """R of the square matrix under both trees (and the flat-TS workspace)."""
    import torch

    import paper_1110_1553_amd as h

    out = {}
    for tag, prm in (("flatTS", dict(nb=256, p=1, a=64, low="flat")),
                     ("greedyTT", dict(nb=256, p=1, a=1, low="greedy"))):
        say("factor 16384^2 %s" % tag)
        dA = graded16k.clone()
        params = h.make_params(**prm)
        work = h.factor(dA, params, h.make_exec(spin_limit=SPIN), timeout_s=120.0)
        torch.cuda.synchronize()
        out[tag] = (dA, params, work)
    return out


@pytest.mark.timeout(600)
def test_square_leading_columns_match_oracle(cuda, graded16k, square_results):
    import numpy as np

    k = 768
    A_lead = np.asfortranarray(graded16k[:, :k].cpu().numpy())
    Rref = oq.r_factor(A_lead, nthreads=threads())
    for tag, (dA, _, _) in square_results.items():
        R = np.triu(dA[:k, :k].cpu().numpy())
        err = rel_err(R, Rref)
        say("  %s: leading %d columns rel err %.3e" % (tag, k, err))
        assert err <= TOL


@pytest.mark.timeout(600)
def test_square_gram_and_backward_error(cuda, graded16k, square_results):
    import torch

    import paper_1110_1553_amd as h

    N = 16384
    A = graded16k
    nA = torch.linalg.norm(A).item()
    AtA = A.t() @ A
    Rs = {}
    for tag, (dA, params, work) in square_results.items():
        R = torch.triu(dA[:N, :N])
        e_gram = torch.linalg.norm(R.t() @ R - AtA).item() / nA ** 2
        # Q R with the factorization's own Q: hqr_apply_q on [R; 0] (square: R itself)
        QR = h.colmajor(R)
        h.apply_q(QR, N, N, params, work, h.make_exec(spin_limit=SPIN))
        torch.cuda.synchronize()
        e_qr = torch.linalg.norm(QR - A).item() / nA
        say("  %s: ||R^T R - A^T A|| / ||A||^2 = %.3e, ||QR - A|| / ||A|| = %.3e" % (tag, e_gram, e_qr))
        assert e_gram <= TOL and e_qr <= TOL
        d = torch.sign(torch.diagonal(R))
        d[d == 0] = 1.0
        Rs[tag] = R * d[:, None]
        del QR
    e_trees = (torch.linalg.norm(Rs["flatTS"] - Rs["greedyTT"]) / torch.linalg.norm(Rs["greedyTT"])).item()
    say("  flat TS vs Greedy TT: %.3e" % e_trees)
    assert e_trees <= TOL
