"""GPU parity of the FP32 factorization (hqr_factor_f32) against the CPU
oracle.

The oracle factors the same float32 values in FP64.  Householder QR is
backward stable: the computed R is the exact R of A + dA with
||dA|| <= c(M, N) u ||A||, u = 2^-24, and for these iid Gaussian matrices
(M >= N, condition numbers below about 10) a relative perturbation of R of
the same order follows.  With c(M, N) taken as sqrt(M N) (the usual
rounding-error growth of blocked Householder QR) the tolerance is
10 sqrt(M N) u; the measured errors sit about two orders below it.
"""
import sys

import numpy as np
import pytest

from oracle import qr as oq
from paper_1110_1553_amd import inputs

pytestmark = pytest.mark.gpu

SPIN = 4000000
U32 = 2.0 ** -24


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = [
    ("flatTS-nb64", 512, 256, dict(nb=64, p=1, a=8, low="flat")),
    ("greedyTT-nb64-ragged", 1000, 300, dict(nb=64, low="greedy")),
    ("hqr-nb128-ragged", 1536, 449, dict(nb=128, p=3, a=2, low="greedy", high="fibonacci", domino=1)),
    ("hqr-nb256", 2100, 513, dict(nb=256, p=2, a=2, low="greedy", high="binary", domino=1)),
    ("binary-nb256-square", 768, 768, dict(nb=256, low="binary")),
    ("narrow-nb256", 900, 37, dict(nb=256, p=1, a=2, low="greedy", high="greedy")),
    ("flat-nb128-one-tile-row", 100, 100, dict(nb=128, p=1, a=1, low="flat")),
]


@pytest.mark.parametrize("tag,M,N,prm", CASES, ids=[c[0] for c in CASES])
def test_f32_factor_matches_oracle(cuda, tag, M, N, prm):
    import torch

    import paper_1110_1553_amd as h

    say("case %s: %dx%d %s" % (tag, M, N, prm))
    A = inputs.gaussian(M, N, 41).astype(np.float32)
    dA = h.colmajor(torch.from_numpy(np.ascontiguousarray(A)).cuda())
    params = h.make_params(**prm)
    h.factor(dA, params, h.make_exec(spin_limit=SPIN), timeout_s=60.0)
    R = np.triu(dA[:N, :N].cpu().numpy().astype(np.float64))
    Rref = oq.r_factor(A.astype(np.float64))
    err = np.linalg.norm(oq.sign_normalize(R) - oq.sign_normalize(Rref)) / np.linalg.norm(Rref)
    tol = 10.0 * np.sqrt(M * N) * U32
    say("  rel err %.3e (tolerance %.1e)" % (err, tol))
    assert np.all(np.isfinite(dA.cpu().numpy()))
    assert err <= tol
    # scheduling does not change a bit: one workgroup in list order gives the same result
    dA1 = h.colmajor(torch.from_numpy(np.ascontiguousarray(A)).cuda())
    h.factor(dA1, params, h.make_exec(workers=1, order=1, spin_limit=SPIN), timeout_s=60.0)
    assert torch.equal(dA, dA1)
