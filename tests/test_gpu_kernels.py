"""Each tile kernel against the identity that defines it (Section II: the
kernels of a tiled Householder QR and what they compute).

Every case is a tile matrix small enough that its task list holds only the
kernel under test next to the panel factorizations it needs (checked on the
plan), with inputs built so that the kernel's own identity can be read off
the result:

* GEQRT on one tile A: R^T R = A^T A, and R is the oracle's R.
* TSQRT on [R0; A1] (R0 upper triangular, A1 square): the new triangle R'
  satisfies R'^T R' = R0^T R0 + A1^T A1, and Q^T [R0; A1] = [R'; 0].
* TTQRT on [R1; R2] (both upper triangular): R'^T R' = R1^T R1 + R2^T R2, and
  Q^T [R1; R2] = [R'; 0].
* UNMQR: one tile factored by GEQRT, then Q^T B through hqr_apply_qt:
  R^T (Q^T B)(0:N) = A^T B, Q^T keeps the norm of every column of B, and
  Q (Q^T B) = B.
* TSMQR, TTMQR: a 2 x 2 tile matrix whose first tile column is factored
  with GEQRT + TSQRT or GEQRT + TTQRT, so that its second tile column goes
  through UNMQR and one kind of two-tile update kernel.  The whole R
  satisfies R^T R = A^T A and matches the oracle's R, and the same factors
  applied to A through hqr_apply_qt give [R; 0] (the apply path replays the
  update kernels on B).

Bars: the identities hold to a few units of roundoff times the norms
involved (backward stability of Householder QR); 1e-13 relative is used.
R against the oracle: 1e-12 relative after sign normalisation.
"""
import sys

import numpy as np
import pytest

from oracle import qr as oq
from paper_1110_1553_amd import inputs

pytestmark = pytest.mark.gpu

SPIN = 4000000
TOL_ID = 1e-13
TOL_R = 1e-12
OPS = {0: "GEQRT", 1: "UNMQR", 2: "TSQRT", 3: "TSMQR", 4: "TTQRT", 5: "TTMQR"}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def ops_of(M, N, nb, params):
    from paper_1110_1553_amd import _lib

    tasks = _lib.plan_tasks(-(-M // nb), -(-N // nb), params)
    return sorted({OPS[int(o)] for o in tasks["op"]})


def run(A, params):
    """Factors A (numpy, float64) on the GPU; returns (factored A, R, workspace)."""
    import torch

    import paper_1110_1553_amd as h

    dA = h.colmajor(torch.from_numpy(np.ascontiguousarray(A)).cuda())
    work = h.factor(dA, params, h.make_exec(spin_limit=SPIN))
    F = dA.cpu().numpy()
    N = A.shape[1]
    return F, np.triu(F[:N, :N]), work


def rel(X, Y):
    return np.linalg.norm(X - Y) / np.linalg.norm(Y)


def gram_err(R, G):
    """|| R^T R - G || / || G ||."""
    return rel(R.T @ R, G)


def apply_qt_of(A, params, work):
    """Q^T A through hqr_apply_qt with the factors in `work`."""
    import torch

    import paper_1110_1553_amd as h

    M, N = A.shape
    dB = h.colmajor(torch.from_numpy(np.ascontiguousarray(A)).cuda())
    h.apply_qt(dB, M, N, params, work, h.make_exec(spin_limit=SPIN))
    return dB.cpu().numpy()


def flat_ts(nb):
    import paper_1110_1553_amd as h

    return h.make_params(nb=nb, p=1, a=1 << 20, low="flat")


def flat_tt(nb):
    import paper_1110_1553_amd as h

    return h.make_params(nb=nb, p=1, a=1, low="flat")


@pytest.mark.parametrize("nb,ncols", [(64, 64), (128, 91), (256, 256)])
def test_geqrt(cuda, nb, ncols):
    A = inputs.gaussian(nb, ncols, 31)
    params = flat_ts(nb)
    assert ops_of(nb, ncols, nb, params) == ["GEQRT"]
    _, R, _ = run(A, params)
    e1, e2 = gram_err(R, A.T @ A), rel(oq.sign_normalize(R), oq.sign_normalize(oq.r_factor(A)))
    say("GEQRT nb %d, %d columns: R^T R - A^T A %.2e, R vs oracle %.2e" % (nb, ncols, e1, e2))
    assert e1 <= TOL_ID and e2 <= TOL_R


def triangle(n, seed, scale=1.0):
    """Upper-triangular n x n with a positive diagonal (an R as GEQRT leaves it)."""
    rng = np.random.default_rng(seed)
    T = np.triu(rng.standard_normal((n, n)))
    T[np.diag_indices(n)] = np.abs(T[np.diag_indices(n)]) + 1.0
    return scale * T


@pytest.mark.parametrize("nb", [64, 128, 256])
def test_tsqrt(cuda, nb):
    R0 = triangle(nb, 41)
    A1 = inputs.gaussian(nb, nb, 42)
    A = np.vstack([R0, A1])
    params = flat_ts(nb)
    assert ops_of(2 * nb, nb, nb, params) == ["GEQRT", "TSQRT"]
    _, R, work = run(A, params)
    e1 = gram_err(R, R0.T @ R0 + A1.T @ A1)
    QtA = apply_qt_of(A, params, work)
    e2 = np.linalg.norm(QtA[nb:]) / np.linalg.norm(A)
    e3 = rel(QtA[:nb], R)
    say("TSQRT nb %d: R'^T R' - (R0^T R0 + A1^T A1) %.2e, |Q^T [R0; A1] below| %.2e, top vs R' %.2e" % (nb, e1, e2,
                                                                                                        e3))
    assert e1 <= TOL_ID and e2 <= TOL_ID and e3 <= TOL_ID


@pytest.mark.parametrize("nb", [64, 128, 256])
def test_ttqrt(cuda, nb):
    R1 = triangle(nb, 51)
    R2 = triangle(nb, 52, scale=0.7)
    A = np.vstack([R1, R2])
    params = flat_tt(nb)
    assert ops_of(2 * nb, nb, nb, params) == ["GEQRT", "TTQRT"]
    _, R, work = run(A, params)
    e1 = gram_err(R, R1.T @ R1 + R2.T @ R2)
    QtA = apply_qt_of(A, params, work)
    e2 = np.linalg.norm(QtA[nb:]) / np.linalg.norm(A)
    e3 = rel(QtA[:nb], R)
    say("TTQRT nb %d: R'^T R' - (R1^T R1 + R2^T R2) %.2e, |Q^T [R1; R2] below| %.2e, top vs R' %.2e" % (nb, e1, e2,
                                                                                                         e3))
    assert e1 <= TOL_ID and e2 <= TOL_ID and e3 <= TOL_ID


@pytest.mark.parametrize("nb,ncols,nrhs", [(64, 64, 100), (256, 227, 70)])
def test_unmqr(cuda, nb, ncols, nrhs):
    """UNMQR on its own: one tile factored by GEQRT, then Q^T B through
    hqr_apply_qt (the apply path runs UNMQR on B's blocks).  With A = Q1 R,
    R^T (Q^T B)(0:N) = A^T B; Q^T keeps every column's norm; Q (Q^T B) = B.
    (None of the three needs a solve, whose error would grow with the
    condition of A.)"""
    import torch

    import paper_1110_1553_amd as h

    A = inputs.gaussian(nb, ncols, 71)
    B = inputs.gaussian(nb, nrhs, 72)
    params = flat_ts(nb)
    assert ops_of(nb, ncols, nb, params) == ["GEQRT"]
    _, R, work = run(A, params)
    dB = h.colmajor(torch.from_numpy(np.ascontiguousarray(B)).cuda())
    h.apply_qt(dB, nb, ncols, params, work, h.make_exec(spin_limit=SPIN))
    QtB = dB.cpu().numpy()
    e1 = np.linalg.norm(R.T @ QtB[:ncols] - A.T @ B) / (np.linalg.norm(A) * np.linalg.norm(B))
    cn = np.linalg.norm(B, axis=0)
    e2 = np.abs(np.linalg.norm(QtB, axis=0) - cn).max() / cn.max()
    h.apply_q(dB, nb, ncols, params, work, h.make_exec(spin_limit=SPIN))
    e3 = rel(dB.cpu().numpy(), B)
    say("UNMQR nb %d (%d columns, %d right-hand sides): R^T (Q^T B)(0:N) - A^T B %.2e, column norms %.2e, "
        "Q Q^T B vs B %.2e" % (nb, ncols, nrhs, e1, e2, e3))
    assert e1 <= TOL_ID and e2 <= TOL_ID and e3 <= TOL_ID


@pytest.mark.parametrize("kind,nb", [("TSMQR", 64), ("TSMQR", 256), ("TTMQR", 64), ("TTMQR", 256)])
def test_update_kernels(cuda, kind, nb):
    """A 2 x 2 tile matrix: the second tile column goes through UNMQR and one
    kind of two-tile update kernel."""
    if kind == "TSMQR":
        params = flat_ts(nb)
        want = ["GEQRT", "TSMQR", "TSQRT", "UNMQR"]
    else:
        params = flat_tt(nb)
        want = ["GEQRT", "TTMQR", "TTQRT", "UNMQR"]
    M, N = 2 * nb, 2 * nb - 29  # ragged last tile column
    A = inputs.gaussian(M, N, 61)
    assert ops_of(M, N, nb, params) == want
    _, R, work = run(A, params)
    e1 = gram_err(R, A.T @ A)
    e2 = rel(oq.sign_normalize(R), oq.sign_normalize(oq.r_factor(A)))
    QtA = apply_qt_of(A, params, work)
    e3 = rel(np.triu(QtA[:N]), R)
    e4 = (np.linalg.norm(np.tril(QtA[:N], -1)) + np.linalg.norm(QtA[N:])) / np.linalg.norm(A)
    say("%s nb %d (%dx%d): R^T R - A^T A %.2e, R vs oracle %.2e, Q^T A vs [R; 0]: %.2e / %.2e" % (
        kind, nb, M, N, e1, e2, e3, e4))
    assert e1 <= TOL_ID and e2 <= TOL_R and e3 <= TOL_ID and e4 <= TOL_ID
