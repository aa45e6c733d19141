"""GPU tests of the boundary's contracts: workspaces shared between entry
points, the factorization signature, and factorization handles.

* A least-squares workspace holds its factorization where hqr_apply_qt,
  hqr_apply_q and hqr_solve look for it: Q^T B, Q B and the least-squares
  solution of new right-hand sides with it match the oracle (the first N rows
  of D Q^T B sign-normalised, the residual norms, x), as after hqr_factor.
* A workspace that holds another factorization (other tree, other shape) or
  none is refused: the apply launch stops before its first task, B is left
  as it was, and hqr_status reports HQR_ERR_FACTORS.
* hqr_factors handles from hqr_factor, hqr_lstsq and hqr_factor_f32 drive
  the same operations with the shape, parameters and workspace they carry.
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


def check_qtb(QtB, R, F, tau, B, N, tol=TOL):
    """First N rows of D Q^T B against the oracle's, and the residual norms."""
    ref = oq.apply_qt(F, tau, B)
    Rref = oq.r_of(F)
    top = signs(R)[:, None] * QtB[:N]
    top_ref = signs(Rref)[:, None] * ref[:N]
    e_top = np.linalg.norm(top - top_ref) / np.linalg.norm(top_ref)
    e_res = np.abs(np.linalg.norm(QtB[N:], axis=0) - np.linalg.norm(ref[N:], axis=0)).max() / np.linalg.norm(B)
    say("  Q^T B: top %.3e residual norms %.3e" % (e_top, e_res))
    assert e_top <= tol and e_res <= tol


@pytest.mark.parametrize("M,N,nb", [(2100, 513, 64), (2100, 513, 256), (1536, 448, 128)])
def test_lstsq_workspace_serves_apply_and_solve(cuda, M, N, nb):
    import paper_1110_1553_amd as h

    say("case lstsq workspace reused: %dx%d nb %d" % (M, N, nb))
    params = h.make_params(nb=nb, p=2, a=2, low="greedy", high="fibonacci", domino=1)
    ex = h.make_exec(spin_limit=SPIN)
    A = inputs.gaussian(M, N, 41)
    B1 = inputs.gaussian(M, 3, 42)
    dA, dB1 = dev(A), dev(B1)
    work = h.lstsq(dA, dB1, params, ex)
    R = np.triu(dA[:N, :N].cpu().numpy())
    F, tau = oq.factor(A)
    # Q^T of a new right-hand side with the least-squares workspace
    B2 = inputs.gaussian(M, 5, 43)
    dB2 = dev(B2)
    bwork = h.apply_qt(dB2, M, N, params, work, ex)
    check_qtb(dB2.cpu().numpy(), R, F, tau, B2, N)
    # Q (Q^T B) = B
    h.apply_q(dB2, M, N, params, work, ex, bwork=bwork)
    e_rt = np.linalg.norm(dB2.cpu().numpy() - B2) / np.linalg.norm(B2)
    say("  Q Q^T B - B: %.3e" % e_rt)
    assert e_rt <= TOL
    # least squares for further right-hand sides
    B3 = inputs.gaussian(M, 2, 44)
    dB3 = dev(B3)
    h.solve(dB3, M, N, params, work, ex)
    X = dB3.cpu().numpy()[:N]
    Xref = oq.lstsq(A, B3)
    e_x = np.linalg.norm(X - Xref) / np.linalg.norm(Xref)
    say("  solve: x %.3e" % e_x)
    assert e_x <= 1e-11


def test_apply_refuses_a_foreign_workspace(cuda):
    import torch

    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import _lib

    M, N = 1000, 300
    say("case signature: apply with other params / shape / an unfactored workspace")
    p1 = h.make_params(nb=64, p=2, a=2, low="greedy", high="binary", domino=1)
    p2 = h.make_params(nb=64, p=1, a=1, low="greedy")  # same tile grid, other tree
    ex = h.make_exec(spin_limit=SPIN)
    A = inputs.gaussian(M, N, 51)
    dA = dev(A)
    work = h.factor(dA, p1, ex)
    R = np.triu(dA[:N, :N].cpu().numpy())
    B = inputs.gaussian(M, 2, 52)
    for tag, (MM, NN, pp, ww) in {
        "other tree": (M, N, p2, work),
        "other shape": (M, N - 64, p1, work),
    }.items():
        dB = dev(B)
        with pytest.raises(h.HQRError) as e:
            h.apply_qt(dB, MM, NN, pp, ww, ex)
        say("  %s: code %d" % (tag, e.value.code))
        assert e.value.code == _lib.ERR_FACTORS
        assert np.array_equal(dB.cpu().numpy(), B)  # nothing was applied
    # a workspace that never held a factorization
    blank = h.Workspace(M, N, p1, device="cuda")
    blank.buf.zero_()
    dB = dev(B)
    with pytest.raises(h.HQRError) as e:
        h.solve(dB, M, N, p1, blank, ex)
    assert e.value.code == _lib.ERR_FACTORS
    # the right one still works afterwards
    dB = dev(B)
    h.apply_qt(dB, M, N, p1, work, ex)
    F, tau = oq.factor(A)
    check_qtb(dB.cpu().numpy(), R, F, tau, B, N)
    torch.cuda.synchronize()


def test_factor_handles(cuda):
    import torch

    import paper_1110_1553_amd as h

    M, N = 1300, 420
    say("case handles: hqr_factor / hqr_lstsq / hqr_factor_f32 -> hqr_factors_*")
    params = h.make_params(nb=128, p=2, a=2, low="greedy", high="fibonacci", domino=1)
    ex = h.make_exec(spin_limit=SPIN)
    A = inputs.gaussian(M, N, 61)
    F, tau = oq.factor(A)
    dA = dev(A)
    work, fac = h.factor(dA, params, ex, handle=True)
    MM, NN, prm, wptr, wbytes = fac.query()
    assert (MM, NN, prm.nb, prm.p, prm.a, wptr, wbytes) == (M, N, 128, 2, 2, work.ptr, work.bytes)
    R = np.triu(dA[:N, :N].cpu().numpy())
    B = inputs.gaussian(M, 4, 62)
    dB = dev(B)
    h.factors_run(fac, "apply_qt", dB, ex)
    check_qtb(dB.cpu().numpy(), R, F, tau, B, N)
    h.factors_run(fac, "apply_q", dB, ex)
    assert np.linalg.norm(dB.cpu().numpy() - B) / np.linalg.norm(B) <= TOL
    dB = dev(B)
    h.factors_run(fac, "solve", dB, ex)
    Xref = oq.lstsq(A, B)
    e_x = np.linalg.norm(dB.cpu().numpy()[:N] - Xref) / np.linalg.norm(Xref)
    say("  handle solve: x %.3e" % e_x)
    assert e_x <= 1e-11
    fac.close()
    # a handle from hqr_lstsq
    dA2, dB2 = dev(A), dev(inputs.gaussian(M, 1, 63))
    work2, fac2 = h.lstsq(dA2, dB2, params, ex, handle=True)
    dB = dev(B)
    h.factors_run(fac2, "apply_qt", dB, ex)
    check_qtb(dB.cpu().numpy(), R, F, tau, B, N)
    # a handle of FP32 factors: Q^T B in FP32 arithmetic, B itself double
    A32 = A.astype(np.float32).astype(np.float64)
    dA32 = h.colmajor(torch.from_numpy(np.ascontiguousarray(A32)).cuda().to(torch.float32))
    work3, fac3 = h.factor(dA32, params, ex, handle=True)
    R32 = np.triu(dA32[:N, :N].double().cpu().numpy())
    F32, tau32 = oq.factor(A32)
    dB = dev(B)
    h.factors_run(fac3, "apply_qt", dB, ex)
    tol32 = 10 * np.sqrt(M * N) * 2.0 ** -24
    check_qtb(dB.cpu().numpy(), R32, F32, tau32, B, N, tol=tol32)
    with pytest.raises(h.HQRError):
        h.factors_run(fac3, "solve", dev(B), ex)  # solve takes double factors only
    torch.cuda.synchronize()
