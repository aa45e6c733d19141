"""GPU parity of the batched launch (hqr_batch_* / hqr_lstsq_batched).

Each problem of a batch runs the same tasks, in the same per-tile order, as
a launch of that problem alone, so R, V, Q^T B and the solutions must be
bitwise identical to hqr_lstsq / hqr_factor on the problem by itself; they
are also checked against the CPU oracle (sign-normalized R within 1e-12,
solutions within 1e-11, residual norms within 1e-12).  A graph-captured run
is replayed several times, with eager work in between, and every replay is
compared with the eager result.
"""
import sys

import numpy as np
import pytest

from oracle import qr as oq
from paper_1110_1553_amd import inputs

pytestmark = pytest.mark.gpu

SPIN = 4000000


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(X):
    import torch

    import paper_1110_1553_amd as h

    return h.colmajor(torch.from_numpy(np.ascontiguousarray(X)).cuda())


def signed_r(R):
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return d[:, None] * R


def check_against_oracle(A, B, Aout, Bout, tag):
    M, N = A.shape
    R = np.triu(Aout[:N, :N])
    Rref = oq.r_of(oq.factor(A)[0])
    e_r = np.linalg.norm(signed_r(R) - signed_r(Rref)) / np.linalg.norm(Rref)
    msg = "  %s %dx%d: R %.3e" % (tag, M, N, e_r)
    assert e_r <= 1e-12, msg
    if B is not None:
        X = Bout[:N]
        Xref = oq.lstsq(A, B)
        e_x = np.linalg.norm(X - Xref) / np.linalg.norm(Xref)
        rn = np.linalg.norm(Bout[N:], axis=0)
        rn_ref = np.linalg.norm(A @ Xref - B, axis=0)
        e_rn = np.abs(rn - rn_ref).max() / np.linalg.norm(B)
        msg += "  x %.3e  residual norms %.3e" % (e_x, e_rn)
        assert e_x <= 1e-11 and e_rn <= 1e-12, msg
    say(msg)


MIXES = [
    ("nb64-greedy", dict(nb=64, low="greedy"),
     [(700, 200, 3), (256, 256, 1), (1000, 64, 5), (333, 37, 2), (2048, 512, 1), (64, 64, 1), (129, 65, 0),
      (4000, 100, 70)]),
    ("nb64-hqr", dict(nb=64, p=2, a=2, low="greedy", high="fibonacci", domino=1),
     [(1500, 300, 1), (640, 128, 2), (97, 33, 1), (3000, 511, 4)]),
    ("nb128-flat", dict(nb=128, p=1, a=100, low="flat"), [(1024, 256, 1), (700, 300, 2), (300, 130, 0)]),
    ("nb256-hqr", dict(nb=256, p=2, a=1, low="greedy", high="binary", domino=0), [(2100, 513, 3), (600, 256, 1)]),
    ("nb256-narrow", dict(nb=256, p=1, a=4, low="greedy", high="greedy"),
     [(900, 37, 1), (1300, 150, 1), (5000, 333, 1), (256, 200, 1), (3000, 480, 2)]),
]


@pytest.mark.parametrize("tag,prm,shapes", MIXES, ids=[m[0] for m in MIXES])
def test_batch_matches_single_and_oracle(cuda, tag, prm, shapes):
    import torch

    import paper_1110_1553_amd as h

    say("batch %s: %s" % (tag, shapes))
    params = h.make_params(**prm)
    ex = h.make_exec(spin_limit=SPIN)
    As = [inputs.gaussian(m, n, 100 + q) for q, (m, n, r) in enumerate(shapes)]
    Bs = [inputs.gaussian(m, max(r, 1), 200 + q) for q, (m, n, r) in enumerate(shapes)]
    any_rhs = any(r > 0 for _, _, r in shapes)
    # problems without right-hand sides are factorizations: give them none
    dAs = [dev(A) for A in As]
    dBs = [dev(B if r > 0 else B[:, :0]) for B, (_, _, r) in zip(Bs, shapes)]
    solver = h.BatchedLstsq(dAs, dBs if any_rhs else None, params, ex)
    solver.run()
    st, first_zero = solver.status(timeout_s=60.0)
    assert st == 0 and (first_zero == -1).all()
    for q, (m, n, r) in enumerate(shapes):
        dA1 = dev(As[q])
        if r > 0:
            dB1 = dev(Bs[q])
            h.lstsq(dA1, dB1, params, ex)
            assert torch.equal(dBs[q], dB1), "B of problem %d differs from its single launch" % q
        else:
            h.factor(dA1, params, ex, timeout_s=60.0)
        assert torch.equal(dAs[q], dA1), "A of problem %d differs from its single launch" % q
        check_against_oracle(As[q], Bs[q] if r > 0 else None, dAs[q].cpu().numpy(),
                             dBs[q].cpu().numpy() if r > 0 else None, "problem %d" % q)
    torch.cuda.synchronize()


def test_one_call_form_and_request_shapes(cuda):
    """hqr_lstsq_batched on 40 requests drawn like a small serving mix."""
    import paper_1110_1553_amd as h

    m, n = inputs.request_shapes(40, 5, mlo=64, mhi=1500, nlo=8, nhi=200)
    say("one-call batch of %d requests, rows %d..%d cols %d..%d" % (len(m), m.min(), m.max(), n.min(), n.max()))
    params = h.make_params(nb=64, low="greedy")
    As = [inputs.gaussian(int(a), int(b), 300 + q) for q, (a, b) in enumerate(zip(m, n))]
    Bs = [inputs.gaussian(int(a), 1, 400 + q) for q, a in enumerate(m)]
    dAs, dBs = [dev(A) for A in As], [dev(B) for B in Bs]
    first_zero = h.lstsq_batched(dAs, dBs, params, h.make_exec(spin_limit=SPIN))
    assert (first_zero == -1).all()
    for q in range(len(m)):
        check_against_oracle(As[q], Bs[q], dAs[q].cpu().numpy(), dBs[q].cpu().numpy(), "request %d" % q)


def test_graph_capture_replays(cuda):
    """hqr_batch_run captured in a graph: three replays, each after the inputs
    are restored by eager copies and checked against the eager run."""
    import torch

    import paper_1110_1553_amd as h

    shapes = [(700, 200, 3), (1000, 64, 5), (256, 256, 1)]
    say("graph capture of a batch %s" % shapes)
    params = h.make_params(nb=64, low="greedy")
    ex = h.make_exec(spin_limit=SPIN)
    As = [dev(inputs.gaussian(m, n, 500 + q)) for q, (m, n, r) in enumerate(shapes)]
    Bs = [dev(inputs.gaussian(m, r, 600 + q)) for q, (m, n, r) in enumerate(shapes)]
    A0 = [A.clone() for A in As]
    B0 = [B.clone() for B in Bs]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        solver = h.BatchedLstsq(As, Bs, params, ex, stream=s)
        solver.run(stream=s)
    s.synchronize()
    st, fz = solver.status(stream=s, timeout_s=60.0)
    assert st == 0
    Aref = [A.clone() for A in As]
    Bref = [B.clone() for B in Bs]
    for A, a0 in zip(As, A0):
        A.copy_(a0)
    for B, b0 in zip(Bs, B0):
        B.copy_(b0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        solver.run(stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        for A, a0 in zip(As, A0):
            A.copy_(a0)
        for B, b0 in zip(Bs, B0):
            B.copy_(b0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        st, fz = solver.status(timeout_s=60.0)
        assert st == 0
        for q in range(len(shapes)):
            assert torch.equal(As[q], Aref[q]) and torch.equal(Bs[q], Bref[q]), "replay %d problem %d" % (rep, q)
        say("  replay %d identical to the eager run" % rep)
        _ = (torch.ones(1000, device="cuda") * rep).sum().item()  # eager work between replays


def test_rank_deficient_problem_is_reported(cuda):
    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import _lib

    shapes = [(400, 150, 1), (300, 100, 1), (500, 120, 2)]
    say("singular problem in a batch %s" % shapes)
    As = [inputs.gaussian(m, n, 700 + q) for q, (m, n, r) in enumerate(shapes)]
    As[1][:, 41] = 0.0
    Bs = [inputs.gaussian(m, r, 800 + q) for q, (m, n, r) in enumerate(shapes)]
    dAs, dBs = [dev(A) for A in As], [dev(B) for B in Bs]
    solver = h.BatchedLstsq(dAs, dBs, h.make_params(nb=64, low="greedy"), h.make_exec(spin_limit=SPIN))
    solver.run()
    st, first_zero = solver.status(timeout_s=60.0)
    assert st == _lib.ERR_SINGULAR
    assert first_zero.tolist() == [-1, 41, -1]
    # the same report written by the device into pinned host memory
    import torch

    words = torch.full((len(shapes) + 1,), 7, dtype=torch.int32, pin_memory=True)
    solver.batch.publish_status(solver.work.data_ptr(), words.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert words.tolist() == [_lib.ERR_SINGULAR, -1, 41, -1]
    for q in (0, 2):
        check_against_oracle(As[q], Bs[q], dAs[q].cpu().numpy(), dBs[q].cpu().numpy(), "problem %d" % q)


def test_export_all_matches_per_problem_export(cuda):
    """hqr_batch_export_all writes the same bytes as hqr_batch_export_factors
    problem by problem, and skips problems without a destination."""
    import torch

    import paper_1110_1553_amd as h

    shapes = [(900, 37, 1), (1300, 300, 1), (500, 120, 2), (700, 256, 0)]
    say("export of a batch's factors %s" % shapes)
    params = h.make_params(nb=256, p=1, a=2, low="greedy", high="greedy")
    As = [dev(inputs.gaussian(m, n, 900 + q)) for q, (m, n, r) in enumerate(shapes)]
    Bs = [dev(inputs.gaussian(m, max(r, 1), 950 + q)[:, :r]) for q, (m, n, r) in enumerate(shapes)]
    solver = h.BatchedLstsq(As, Bs, params, h.make_exec(spin_limit=SPIN))
    solver.run()
    s = torch.cuda.current_stream().cuda_stream
    one = [torch.zeros(h.workspace_size(m, n, params), dtype=torch.uint8, device="cuda") for m, n, r in shapes]
    for q, w in enumerate(one):
        solver.batch.export_factors(q, solver.work.data_ptr(), w.data_ptr(), w.numel(), s)
    allw = [torch.full((h.workspace_size(m, n, params),), 3, dtype=torch.uint8, device="cuda") for m, n, r in shapes]
    for w in allw[:3]:
        w.zero_()
    dsts = [w.data_ptr() for w in allw[:3]] + [0]
    solver.batch.export_all(solver.work.data_ptr(), dsts, [w.numel() for w in allw], s)
    torch.cuda.synchronize()
    for q in range(3):
        assert torch.equal(one[q], allw[q]), "problem %d" % q
    assert (allw[3] == 3).all()  # no destination: untouched
    st, _ = solver.status(timeout_s=60.0)
    assert st == 0

