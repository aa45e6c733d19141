"""Continuous-batching serving on the GPU: a Poisson trace of small
least-squares requests served by the scheduler over the batched launch.
Every request's factorization and solution must be bitwise identical to the
same request solved alone with hqr_lstsq (alone vs in a mix), and a sample
is checked against the CPU oracle."""
import sys

import numpy as np
import pytest

from oracle import qr as oq
from paper_1110_1553_amd import inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# nb = 64 with a Greedy tree, and the tile size and tree the serving
# benchmark's autotuner picks (nb = 256, TS domains of 4 under Greedy)
SERVE_CASES = [dict(tree=dict(nb=64, low="greedy"), mhi=2000, nhi=160, budget=24 << 20),
               dict(tree=dict(nb=256, a=4, low="greedy", high="greedy"), mhi=4000, nhi=400, budget=96 << 20)]


@pytest.mark.parametrize("case", SERVE_CASES, ids=["nb64-greedy", "nb256-ts4-greedy"])
def test_served_results_equal_lone_solves(cuda, case):
    import torch

    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import serve

    n_req = 60
    m, n = inputs.request_shapes(n_req, 9, mlo=64, mhi=case["mhi"], nlo=8, nhi=case["nhi"])
    gaps = inputs.arrival_gaps(n_req, 3000.0, 10)
    arrivals = np.cumsum(gaps)
    say("serving %d requests over %.1f ms, %s" % (n_req, arrivals[-1] * 1e3, case["tree"]))
    params = h.make_params(**case["tree"])
    As = [inputs.gaussian(int(a), int(b), 900 + q) for q, (a, b) in enumerate(zip(m, n))]
    Bs = [inputs.gaussian(int(a), 1, 1900 + q) for q, a in enumerate(m)]
    dev = lambda X: h.colmajor(torch.from_numpy(np.ascontiguousarray(X)).cuda())  # noqa: E731
    reqs = [serve.Request(q, dev(As[q]), dev(Bs[q]), float(arrivals[q])) for q in range(n_req)]
    # the budget in two slots forces several batches
    be = serve.GpuBackend(params, case["budget"], max_inflight=2, exec_=h.make_exec(spin_limit=4000000))
    sch = serve.Scheduler(be)
    lat = sch.run(reqs)
    torch.cuda.synchronize()
    sizes = [len(b["reqs"]) for b in sch.batches]
    say("batches %d, sizes %s, p50 %.2f ms p99 %.2f ms" % (len(sizes), sizes, np.percentile(lat, 50) * 1e3,
                                                       np.percentile(lat, 99) * 1e3))
    assert sum(sizes) == n_req and all(r.status == 0 and r.first_zero == -1 for r in reqs)
    assert (lat > 0).all()
    for q, r in enumerate(reqs):
        A1, B1 = dev(As[q]), dev(Bs[q])
        h.lstsq(A1, B1, params, h.make_exec(spin_limit=4000000))
        assert torch.equal(A1, r.A) and torch.equal(B1, r.B), "request %d differs from its lone solve" % q
    for q in range(0, n_req, 7):
        X = reqs[q].B.cpu().numpy()[: n[q]]
        Xref = oq.lstsq(As[q], Bs[q])
        e = np.linalg.norm(X - Xref) / np.linalg.norm(Xref)
        say("  request %d %dx%d: x error %.2e" % (q, m[q], n[q], e))
        assert e <= 1e-11


def test_overlap_and_resident_factors(cuda):
    """Batches admitted while another one runs (two slots, two streams), and
    factors kept on the device: a second right-hand side for a served
    request is solved with its resident factorization (hqr_solve)."""
    import torch

    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import serve

    n_req = 40
    m, n = inputs.request_shapes(n_req, 11, mlo=200, mhi=3000, nlo=16, nhi=200)
    arrivals = np.cumsum(inputs.arrival_gaps(n_req, 20000.0, 12))
    params = h.make_params(nb=64, low="greedy")
    As = [inputs.gaussian(int(a), int(b), 1100 + q) for q, (a, b) in enumerate(zip(m, n))]
    Bs = [inputs.gaussian(int(a), 1, 1200 + q) for q, a in enumerate(m)]
    dev = lambda X: h.colmajor(torch.from_numpy(np.ascontiguousarray(X)).cuda())  # noqa: E731
    reqs = [serve.Request(q, dev(As[q]), dev(Bs[q]), float(arrivals[q])) for q in range(n_req)]
    be = serve.GpuBackend(params, 48 << 20, max_inflight=2, exec_=h.make_exec(spin_limit=4000000),
                          factor_budget=1 << 30)
    sch = serve.Scheduler(be)
    lat = sch.run(reqs)
    torch.cuda.synchronize()
    b = sch.batches
    overlaps = sum(1 for i in range(1, len(b)) if b[i]["t_launch"] < b[i - 1]["t_done"])
    say("batches %d, launched while the previous one ran: %d, p50 %.2f ms" % (len(b), overlaps,
                                                                               np.percentile(lat, 50) * 1e3))
    assert len(b) > 1 and overlaps >= 1
    assert all(r.status == 0 for r in reqs)
    for q in (0, n_req // 2, n_req - 1):
        B2 = inputs.gaussian(int(m[q]), 2, 1300 + q)
        dB2 = dev(B2)
        assert be.solve_resident(q, int(m[q]), int(n[q]), dB2)
        torch.cuda.synchronize()
        X = dB2.cpu().numpy()[: n[q]]
        Xref = oq.lstsq(As[q], B2)
        e = np.linalg.norm(X - Xref) / np.linalg.norm(Xref)
        say("  request %d %dx%d: second right-hand side from resident factors, x error %.2e" % (q, m[q], n[q], e))
        assert e <= 1e-11
