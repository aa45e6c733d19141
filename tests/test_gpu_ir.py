"""GPU parity of the mixed-precision least-squares solver (hqr_lstsq_ir):
FP32 tiled QR plus FP64 augmented-system refinement against the CPU
oracle's FP64 solution x = R^{-1} (Q^T b)(0:N).

The refinement runs until the backward error eta of the augmented system
is <= 1e-15 (a few units of u = 2^-53).  Both solutions are then backward
stable in FP64, so they differ by at most about kappa(A) u relative to
||x||: the tolerance is max(1e-11, 100 kappa u).  The refinement converges when kappa(A) times the
float unit roundoff is well below one; the cases go up to kappa = 1e6
(kappa u_f ~ 0.06).
"""
import sys

import numpy as np
import pytest

from oracle import qr as oq
from paper_1110_1553_amd import inputs

pytestmark = pytest.mark.gpu

SPIN = 4000000
U64 = 2.0 ** -53


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = [
    ("kappa1e6-nb64", 2048, 256, 1e-6, dict(nb=64, low="greedy")),
    ("kappa1e6-nb128-hqr", 3000, 384, 1e-6, dict(nb=128, p=2, a=4, low="greedy", high="fibonacci", domino=1)),
    ("kappa1e4-ragged-nb256", 1500, 300, 1e-4, dict(nb=256, p=1, a=2, low="greedy", high="greedy")),
    ("kappa1e2-square-nb64", 640, 640, 1e-2, dict(nb=64, low="binary")),
]


@pytest.mark.parametrize("tag,M,N,smin,prm", CASES, ids=[c[0] for c in CASES])
def test_ir_matches_oracle(cuda, tag, M, N, smin, prm):
    import torch

    import paper_1110_1553_amd as h

    say("case %s: %dx%d kappa %.0e %s" % (tag, M, N, 1 / smin, prm))
    A = inputs.graded_tall_device(M, N, 17, smin, device="cpu").numpy()
    rng = np.random.default_rng(18)
    b = A @ rng.standard_normal(N) + 1e-3 * rng.standard_normal(M)
    dA = h.colmajor(torch.from_numpy(np.ascontiguousarray(A)).cuda())
    A_before = dA.clone()
    db = torch.from_numpy(b).cuda()
    params = h.make_params(**prm)
    x, r, info = h.lstsq_ir(dA, db, params, h.make_exec(spin_limit=SPIN), tol=1e-15, residual=True)
    torch.cuda.synchronize()
    say("  iterations %d converged %s eta %.2e history %s" % (info["iterations"], info["converged"], info["eta"],
                                                             ["%.1e" % e for e in info["history"]]))
    assert info["converged"] and info["iterations"] <= 30
    assert torch.equal(dA, A_before)  # A is read only
    xr = oq.lstsq(A, b.reshape(-1, 1)).ravel()
    ex = np.linalg.norm(x.cpu().numpy() - xr) / np.linalg.norm(xr)
    rr = b - A @ xr
    er = np.linalg.norm(r.cpu().numpy() - rr) / np.linalg.norm(b)
    tol = max(1e-11, 100.0 / smin * U64)
    say("  x error %.3e (tolerance %.1e), residual error %.3e" % (ex, tol, er))
    assert ex <= tol and er <= tol
