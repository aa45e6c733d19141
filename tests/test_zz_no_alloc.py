"""The allocation-free least-squares entry point (hqr_lstsq_noalloc) against
hqr_lstsq: the same launches on the same inputs, with the workspace and the
task plan in the library's static device array instead of allocations.
Two calls in a row, the second on a smaller problem (the array keeps the
first call's contents), each compared with hqr_lstsq's R and solutions to
the FP64 parity bar (relative 1e-12; the kernels and their order are the
same, so the results are expected bit for bit); a problem beyond the array's
size is refused before anything is enqueued."""
import ctypes
import sys

import numpy as np
import pytest

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


def run_pair(M, N, nrhs, prm, seed):
    import torch

    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import _lib

    say("case no-alloc: %dx%d nrhs %d %s" % (M, N, nrhs, prm))
    params = h.make_params(**prm)
    ex = h.make_exec(spin_limit=SPIN)
    A = inputs.gaussian(M, N, seed)
    B = inputs.gaussian(M, nrhs, seed + 1)
    # the existing entry point, with its own workspace
    dA1, dB1 = dev(A), dev(B)
    h.lstsq(dA1, dB1, params, ex)
    # the allocation-free one through the C ABI
    dA2, dB2 = dev(A), dev(B)
    dinfo = torch.full((8,), -7, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    rc = _lib.lstsq_noalloc_ptr(dA2.data_ptr(), M, N, dA2.stride(1), dB2.data_ptr(), dB2.stride(1) if nrhs > 1 else M,
                                nrhs, params, ex, dinfo.data_ptr(), s.cuda_stream)
    assert rc == 0, rc
    torch.cuda.synchronize()
    info = dinfo.cpu().numpy()
    assert info[0] == 0, info
    R1 = np.triu(dA1[:N, :N].cpu().numpy())
    R2 = np.triu(dA2[:N, :N].cpu().numpy())
    X1, X2 = dB1.cpu().numpy()[:N], dB2.cpu().numpy()[:N]
    e_r = np.linalg.norm(R2 - R1) / np.linalg.norm(R1)
    e_x = np.linalg.norm(X2 - X1) / np.linalg.norm(X1)
    same = np.array_equal(dA1.cpu().numpy(), dA2.cpu().numpy()) and np.array_equal(dB1.cpu().numpy(),
                                                                                     dB2.cpu().numpy())
    say("  R %.3e  x %.3e  bitwise equal: %s" % (e_r, e_x, same))
    assert e_r <= TOL and e_x <= TOL


def test_noalloc_matches_lstsq_twice(cuda):
    # the second call is smaller: its layout and plan differ, the array still holds the first call's data
    run_pair(3000, 700, 3, dict(nb=128, p=2, a=2, low="greedy", high="fibonacci", domino=1), 81)
    run_pair(1500, 300, 1, dict(nb=128, p=2, a=2, low="greedy", high="fibonacci", domino=1), 83)
    # and a third with another tile size and tree
    run_pair(2100, 513, 2, dict(nb=256, p=1, a=4, low="greedy", high="greedy"), 85)


def test_noalloc_refuses_problems_beyond_the_array(cuda):
    import torch

    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import _lib

    params = h.make_params(nb=256)
    M, N = 16384, 1024
    assert h.lstsq_workspace_size(M, N, 1, params) > _lib.NOALLOC_SCRATCH_BYTES
    dA = torch.zeros((N, M), dtype=torch.float64, device="cuda").t()
    dB = torch.zeros((1, M), dtype=torch.float64, device="cuda").t()
    rc = _lib.lstsq_noalloc_ptr(dA.data_ptr(), M, N, M, dB.data_ptr(), M, 1, params, None, 0,
                                torch.cuda.current_stream().cuda_stream)
    assert rc == 3  # HQR_ERR_WORKSPACE
    assert "needs" in _lib.load().hqr_last_error().decode()
    # argument checks before any device work
    assert _lib.lstsq_noalloc_ptr(dA.data_ptr(), M, N, M - 1, dB.data_ptr(), M, 1, params, None, 0, 0) == -4
