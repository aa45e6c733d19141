"""GPU parity of hqr_factor against the CPU oracle.

Every case factors a seeded synthetic matrix on the GPU through the C ABI and
compares the sign-normalised R with the oracle's unblocked Householder QR of
the same bytes: relative Frobenius error <= 1e-12 (R is unique up to row
signs for a full-rank matrix, and every elimination list computes the same
algebra in another order -- Section II of the paper).  Sizes span several
tiles, ragged edges (zero padding), all tree families and the hierarchical
composition; scheduling must not change a single bit.
"""
import sys

import numpy as np
import pytest

from oracle import qr as oq
from paper_1110_1553_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12
SPIN = 4000000  # polls before a stuck dependency is reported (seconds, not minutes)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def factor_on_gpu(A_np, params, exec_=None):
    import torch

    import paper_1110_1553_amd as h

    dA = h.colmajor(torch.from_numpy(np.ascontiguousarray(A_np)).cuda())
    if exec_ is None:
        exec_ = h.make_exec(spin_limit=SPIN)
    elif exec_.spin_limit == 0:
        exec_.spin_limit = SPIN
    work = h.factor(dA, params, exec_, timeout_s=60.0)
    torch.cuda.synchronize()
    return dA, work


def rel_err(R_gpu, R_ref):
    a, b = oq.sign_normalize(R_gpu), oq.sign_normalize(R_ref)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def check_case(M, N, seed, tag, **prm):
    import paper_1110_1553_amd as h

    say("case %s: %dx%d seed %d params %s" % (tag, M, N, seed, prm))
    A = inputs.gaussian(M, N, seed)
    params = h.make_params(**prm)
    dA, _ = factor_on_gpu(A, params)
    R = h.r_of(dA)
    assert np.all(np.isfinite(dA.cpu().numpy()))
    err = rel_err(R, oq.r_factor(A))
    say("  rel err %.3e" % err)
    assert err <= TOL, (tag, err)
    return dA


def test_small_flat_ts_512x256(hqr_lib, cuda):
    # 512 x 256, nb = 64 (8 x 4 tiles), flat tree with TS kernels
    check_case(512, 256, 1, "flatTS-512x256", nb=64, p=1, a=8, low="flat")


@pytest.mark.parametrize("low", ["flat", "binary", "greedy", "fibonacci"])
def test_tt_trees_nb64(hqr_lib, cuda, low):
    check_case(1024, 512, 2, "TT-" + low, nb=64, p=1, a=1, low=low)


@pytest.mark.parametrize("p,a,low,high,domino", [
    (4, 2, "greedy", "fibonacci", 1),
    (4, 2, "greedy", "fibonacci", 0),
    (3, 4, "flat", "binary", 1),
    (2, 3, "fibonacci", "greedy", 1),
    (8, 1, "binary", "flat", 0),
])
def test_hierarchical_nb64(hqr_lib, cuda, p, a, low, high, domino):
    check_case(1536, 448, 3, "hqr", nb=64, p=p, a=a, low=low, high=high, domino=domino)


@pytest.mark.parametrize("nb", [128, 256])
def test_larger_tiles(hqr_lib, cuda, nb):
    check_case(2048, 768, 4, "flatTS-nb%d" % nb, nb=nb, p=1, a=64, low="flat")
    check_case(2048, 768, 4, "greedyTT-nb%d" % nb, nb=nb, p=1, a=1, low="greedy")
    check_case(2048, 768, 4, "hqr-nb%d" % nb, nb=nb, p=2, a=2, low="greedy", high="fibonacci", domino=1)


def test_square(hqr_lib, cuda):
    check_case(1024, 1024, 5, "square-greedy", nb=128, p=1, a=1, low="greedy")
    check_case(1024, 1024, 5, "square-flatTS", nb=64, p=1, a=100, low="flat")


@pytest.mark.parametrize("M,N,nb", [(1000, 300, 64), (777, 777, 128), (4000, 100, 64), (300, 1, 64),
                                    (64, 64, 64), (65, 65, 64), (2100, 513, 256),
                                    # one tile column with 1, 2 or 3 of its 64-column blocks
                                    # holding no matrix column
                                    (900, 37, 256), (1300, 150, 256), (700, 130, 256)])
def test_ragged_and_edge_shapes(hqr_lib, cuda, M, N, nb):
    check_case(M, N, 6, "ragged", nb=nb, p=2, a=2, low="greedy", high="binary", domino=1)


def test_graded_square_matrix(hqr_lib, cuda):
    import paper_1110_1553_amd as h

    A = inputs.graded(768, seed=7, smin=1e-8)
    say("case graded 768x768 sigma 1..1e-8")
    dA, _ = factor_on_gpu(A, h.make_params(nb=128, p=1, a=1, low="greedy"))
    err = rel_err(h.r_of(dA), oq.r_factor(A))
    say("  rel err %.3e" % err)
    assert err <= TOL


def test_scheduling_does_not_change_bits(hqr_lib, cuda):
    import paper_1110_1553_amd as h

    A = inputs.gaussian(1536, 640, 8)
    prm = h.make_params(nb=64, p=3, a=2, low="greedy", high="fibonacci", domino=1)
    say("case bitwise: sequential (1 workgroup, list order) vs persistent")
    seq, _ = factor_on_gpu(A, prm, h.make_exec(workers=1, order=1))
    par, _ = factor_on_gpu(A, prm, h.make_exec())
    par2, _ = factor_on_gpu(A, prm, h.make_exec())
    prog, _ = factor_on_gpu(A, prm, h.make_exec(order=1))
    few, _ = factor_on_gpu(A, prm, h.make_exec(workers=7))
    s = seq.cpu().numpy()
    for other in (par, par2, prog, few):
        assert np.array_equal(s, other.cpu().numpy())


def test_watchdog_reports_and_exits(hqr_lib, cuda):
    import torch

    import paper_1110_1553_amd as h

    A = inputs.gaussian(1024, 512, 9)
    say("case watchdog: spin limit 1")
    dA = h.colmajor(torch.from_numpy(A).cuda())
    prm = h.make_params(nb=64, p=1, a=1, low="flat")
    work = h.factor(dA, prm, h.make_exec(spin_limit=1), check=False)
    st = h.status(work)
    assert st == 2  # HQR_ERR_WATCHDOG: some task had to wait at least once
    # the device is still usable afterwards
    dA2, _ = factor_on_gpu(A, prm)
    assert rel_err(h.r_of(dA2), oq.r_factor(A)) <= TOL
