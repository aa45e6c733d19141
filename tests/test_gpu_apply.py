"""GPU parity of hqr_apply_qt / hqr_apply_q / hqr_lstsq against the CPU oracle.

Q^T B replays the update kernels of the factorization on B (Section I,
Algorithm 2).  Q itself is not unique, but its first N columns are, up to the
signs that also flip the rows of R: with D = diag(sign(R_ii)) the first N rows
of D Q^T B match the oracle's (D_ref Q_ref^T B), relative error <= 1e-12, and
the column norms of the remaining M - N rows (the least-squares residual
norms) match.  Q (Q^T B) = B, the first N columns of Q are orthonormal and
reproduce A = Q R, and the least-squares solutions match the oracle's
R^{-1} (Q^T b)(0:N) solved with LAPACK's triangular solve.
"""
import sys

import numpy as np
import pytest

from oracle import qr as oq
from paper_1110_1553_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12
SPIN = 4000000


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(X):
    import torch

    import paper_1110_1553_amd as h

    return h.colmajor(torch.from_numpy(np.ascontiguousarray(X)).cuda())


def signs(R):
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return d


CASES = [
    ("flatTS-nb64", 512, 256, 1, dict(nb=64, p=1, a=8, low="flat")),
    ("greedyTT-nb64-ragged", 1000, 300, 5, dict(nb=64, low="greedy")),
    ("hqr-nb128-2blocks", 1536, 448, 70, dict(nb=128, p=3, a=2, low="greedy", high="fibonacci", domino=1)),
    ("hqr-nb256", 2100, 513, 3, dict(nb=256, p=2, a=2, low="greedy", high="binary", domino=1)),
    ("narrow-nb256", 900, 37, 2, dict(nb=256, p=1, a=2, low="greedy", high="greedy")),
    ("square-binary-nb64", 320, 320, 2, dict(nb=64, low="binary")),
]


@pytest.mark.parametrize("tag,M,N,nrhs,prm", CASES, ids=[c[0] for c in CASES])
def test_apply_qt_q_lstsq(cuda, tag, M, N, nrhs, prm):
    import torch

    import paper_1110_1553_amd as h

    say("case %s: %dx%d nrhs %d %s" % (tag, M, N, nrhs, prm))
    A = inputs.gaussian(M, N, 11)
    B = inputs.gaussian(M, nrhs, 12)
    params = h.make_params(**prm)
    ex = h.make_exec(spin_limit=SPIN)
    dA = dev(A)
    work = h.factor(dA, params, ex, timeout_s=60.0)
    R = np.triu(dA[:N, :N].cpu().numpy())
    F, tau = oq.factor(A)
    Rref = oq.r_of(F)

    dB = dev(B)
    bwork = h.apply_qt(dB, M, N, params, work, ex)
    QtB = dB.cpu().numpy()
    QtBref = oq.apply_qt(F, tau, B)
    top = signs(R)[:, None] * QtB[:N]
    top_ref = signs(Rref)[:, None] * QtBref[:N]
    e_top = np.linalg.norm(top - top_ref) / np.linalg.norm(top_ref)
    e_res = np.abs(np.linalg.norm(QtB[N:], axis=0) - np.linalg.norm(QtBref[N:], axis=0)).max() / np.linalg.norm(B)
    say("  Q^T B: top %.3e residual norms %.3e" % (e_top, e_res))
    assert e_top <= TOL and e_res <= TOL

    h.apply_q(dB, M, N, params, work, ex, bwork=bwork)
    e_rt = np.linalg.norm(dB.cpu().numpy() - B) / np.linalg.norm(B)
    say("  Q Q^T B - B: %.3e" % e_rt)
    assert e_rt <= TOL

    # the first N columns of Q: orthonormal, and Q1 R = A
    E = np.zeros((M, N))
    E[np.arange(N), np.arange(N)] = 1.0
    dE = dev(E)
    h.apply_q(dE, M, N, params, work, ex)
    Q1 = dE.cpu().numpy()
    e_orth = np.linalg.norm(Q1.T @ Q1 - np.eye(N)) / np.sqrt(N)
    e_qr = np.linalg.norm(Q1 @ R - A) / np.linalg.norm(A)
    say("  Q1: orthogonality %.3e  ||Q1 R - A||/||A|| %.3e" % (e_orth, e_qr))
    assert e_orth <= TOL and e_qr <= TOL

    dA2, dB2 = dev(A), dev(B)
    h.lstsq(dA2, dB2, params, ex)
    # the factorization inside hqr_lstsq is the same launch with B appended
    assert np.array_equal(np.triu(dA2[:N, :N].cpu().numpy()), R)
    X = dB2.cpu().numpy()[:N]
    Xref = oq.lstsq(A, B)
    e_x = np.linalg.norm(X - Xref) / np.linalg.norm(Xref)
    # residual components below the solution: their norms are the residual norms
    rn = np.linalg.norm(dB2.cpu().numpy()[N:], axis=0)
    rn_ref = np.linalg.norm(A @ Xref - B, axis=0)
    e_rn = np.abs(rn - rn_ref).max() / np.linalg.norm(B)
    say("  lstsq: x %.3e residual norms %.3e" % (e_x, e_rn))
    assert e_x <= 1e-11 and e_rn <= 1e-12
    torch.cuda.synchronize()


def test_apply_ragged_columns_and_leading_dimension(cuda):
    """B with ldb > M and a column count that is not a multiple of 64."""
    import torch

    import paper_1110_1553_amd as h

    M, N, nrhs = 700, 200, 67
    say("case ldb: %dx%d nrhs %d" % (M, N, nrhs))
    A = inputs.gaussian(M, N, 21)
    B = inputs.gaussian(M, nrhs, 22)
    params = h.make_params(nb=64, p=2, a=2, low="greedy", high="flat", domino=0)
    ex = h.make_exec(spin_limit=SPIN)
    work = h.factor(dev(A), params, ex, timeout_s=60.0)
    big = torch.zeros((nrhs, M + 13), dtype=torch.float64, device="cuda")
    big[:, :M] = torch.from_numpy(B.T.copy()).cuda()
    dB = big.t()[:M]  # column-major view, ldb = M + 13
    assert dB.stride() == (1, M + 13)
    h.apply_qt(dB, M, N, params, work, ex)
    F, tau = oq.factor(A)
    QtB = dB.cpu().numpy()
    ref = oq.apply_qt(F, tau, B)
    # per-column norms of the first N rows do not depend on the signs of Q
    e = np.abs(np.linalg.norm(QtB[:N], axis=0) - np.linalg.norm(ref[:N], axis=0)).max() / np.linalg.norm(B)
    say("  column norms of the first N rows: %.3e" % e)
    assert e <= TOL
    assert big[:, M:].abs().max().item() == 0.0  # the padding rows beyond M were not written


def test_lstsq_reports_zero_diagonal(cuda):
    """A zero column makes R_jj = 0: the launch finishes and hqr_status
    reports HQR_ERR_SINGULAR with the column index."""
    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import _lib

    M, N = 400, 150
    A = inputs.gaussian(M, N, 31)
    A[:, 77] = 0.0
    B = inputs.gaussian(M, 1, 32)
    params = h.make_params(nb=64, low="greedy")
    ex = h.make_exec(spin_limit=SPIN)
    dA, dB = dev(A), dev(B)
    with pytest.raises(h.HQRError) as e:
        h.lstsq(dA, dB, params, ex)
    assert e.value.code == _lib.ERR_SINGULAR
    assert e.value.detail[0] == 77
