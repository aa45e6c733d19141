"""Host side of the batched launch: the merged task list of a batch keeps
every problem's own dispatch order (so it is a topological order of the
union of the task graphs, Algorithm 2 per problem) and holds each problem's
tasks exactly once; the workspace covers every problem; bad arguments are
rejected before any device call."""
import ctypes
import random

import numpy as np
import pytest


def _single(h, M, N, params):
    nb = params.nb
    return h._lib.plan_tasks(-(-M // nb), -(-N // nb), params, 0)


@pytest.mark.parametrize("nb,low,high,p,a,domino", [
    (64, "greedy", "flat", 1, 1, 0),
    (64, "flat", "flat", 1, 1000, 0),
    (128, "greedy", "fibonacci", 2, 2, 1),
    (256, "binary", "greedy", 3, 1, 1),
])
def test_merge_keeps_each_problem_order(hqr_lib, nb, low, high, p, a, domino):
    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import _lib

    params = h.make_params(nb=nb, p=p, a=a, low=low, high=high, domino=domino)
    rng = random.Random(nb * 7 + p)
    M, N = [], []
    for _ in range(9):
        nt = rng.randint(1, 4)
        mt = rng.randint(nt, 12)
        M.append(mt * nb - (rng.randint(0, nb - 1) if nb == 64 else 0))
        N.append(nt * nb - (rng.randint(0, nb - 1) if nb == 64 else 0))  # ragged only where chunks = 1
        if N[-1] > M[-1]:
            N[-1] = M[-1]
    b = _lib.Batch(M, N, None, params)
    tasks, prob = b.tasks()
    assert np.bincount(prob, minlength=len(M)).tolist() == [len(_single(h, m, n, params)) for m, n in zip(M, N)]
    for q, (m, n) in enumerate(zip(M, N)):
        mine = tasks[prob == q]
        ref = _single(h, m, n, params)
        assert mine.tobytes() == ref.tobytes(), q
    assert b.workspace_size() > sum(h.workspace_size(m, n, params) for m, n in zip(M, N)) - 64 * 1024
    b.close()


def test_rhs_problems_and_workspace(hqr_lib):
    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import _lib

    params = h.make_params(nb=64, low="greedy")
    M, N, R = [700, 256, 1000], [200, 256, 64], [67, 0, 1]
    b = _lib.Batch(M, N, R, params)
    tasks, prob = b.tasks()
    counts = np.bincount(prob)
    # a problem with right-hand sides has the update tasks of its extra tile columns
    assert counts[0] > len(_single(h, 700, 200, params))
    assert counts[1] == len(_single(h, 256, 256, params))
    need = b.workspace_size()
    assert need >= sum(h.lstsq_workspace_size(m, n, r, params) if r else h.workspace_size(m, n, params)
                       for m, n, r in zip(M, N, R)) - 3 * 256
    assert _lib.lstsq_batched_workspace_size(M, N, R, params) == need
    b.close()


def test_batch_argument_checks(hqr_lib):
    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import _lib

    lib = _lib.load()
    p = h.make_params(nb=64)
    vp = ctypes.c_void_p
    arr = lambda xs, t=ctypes.c_int64: (t * len(xs))(*xs)  # noqa: E731
    out = vp()
    assert lib.hqr_batch_create(0, arr([1]), arr([1]), None, ctypes.byref(p), None, ctypes.byref(out)) == -1
    assert lib.hqr_batch_create(1, arr([100]), arr([200]), None, ctypes.byref(p), None, ctypes.byref(out)) == -3
    assert lib.hqr_batch_create(1, arr([0]), arr([0]), None, ctypes.byref(p), None, ctypes.byref(out)) == -2
    assert lib.hqr_batch_create(1, arr([100]), arr([50]), arr([-1], ctypes.c_int32), ctypes.byref(p), None,
                                ctypes.byref(out)) == -4
    bad = h.make_params(nb=96)
    assert lib.hqr_batch_create(1, arr([100]), arr([50]), None, ctypes.byref(bad), None, ctypes.byref(out)) == -5
    ex = h.make_exec(order=3)
    assert lib.hqr_batch_create(1, arr([100]), arr([50]), None, ctypes.byref(p), ctypes.byref(ex),
                                ctypes.byref(out)) == -6
    b = _lib.Batch([300, 200], [100, 200], [2, 0], p)
    need = b.workspace_size()
    ptrs = (ctypes.c_void_p * 2)(16, 16)
    # lda < M, missing right-hand sides, workspace too small: rejected on the host
    assert lib.hqr_batch_bind(b.handle, ptrs, arr([300, 100]), ptrs, arr([300, 200]), vp(16), need, None) == -3
    assert lib.hqr_batch_bind(b.handle, ptrs, arr([300, 200]), None, None, vp(16), need, None) == -4
    assert lib.hqr_batch_bind(b.handle, ptrs, arr([300, 200]), ptrs, arr([299, 0]), vp(16), need, None) == -5
    assert lib.hqr_batch_bind(b.handle, ptrs, arr([300, 200]), ptrs, arr([300, 0]), vp(16), need - 1, None) == -7
    # run before any bind
    assert lib.hqr_batch_run(b.handle, vp(16), need, None) == -2
    # the one-call form maps the same checks to its own argument positions
    L = lib.hqr_lstsq_batched
    assert L(1, ptrs, arr([100]), arr([200]), arr([100]), ptrs, arr([100]), None, ctypes.byref(p), None, vp(16),
             1 << 30, None) == -4
    assert L(1, ptrs, arr([300]), arr([100]), arr([200]), ptrs, arr([300]), arr([1], ctypes.c_int32),
             ctypes.byref(p), None, vp(16), 1 << 30, None) == -5
    b.close()
