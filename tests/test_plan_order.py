"""The dispatch order of the task plans is a topological order of the task
graph: replaying the plan in list order on one worker, with the counter
semantics of the persistent scheduler (per-tile, per-64-column sub-chunk
version counters; panel tasks wait for and publish every active sub-chunk
of their tiles, update tasks the sub-chunks they cover and the factored
tile's last active one), every wait is already satisfied when its task is
reached, and every tile ends with one bump per write."""
import collections

import numpy as np
import pytest

GEQRT, UNMQR, TSQRT, TSMQR, TTQRT, TTMQR = range(6)


def replay(tasks):
    cnt = collections.Counter()
    cols = [tasks[f].astype(np.int64).tolist() for f in ("op", "chunk", "row", "killer", "k", "j", "pad")]
    vs = tasks["v"].astype(np.int64).tolist()
    for n, (op, ch, i, piv, k, j, pad) in enumerate(zip(*cols)):
        v = vs[n]
        c0, cn, cv = ch, pad >> 8, pad & 0xFF
        if op in (GEQRT, TSQRT, TTQRT):
            for b in range(ch):  # ch = active sub-chunks of the tile column
                if op == GEQRT:
                    assert cnt[(i, k, b)] >= v[0], (n, "GEQRT block", b)
                else:
                    assert cnt[(piv, k, b)] >= v[0] and cnt[(i, k, b)] >= v[1], (n, "panel block", b)
            for b in range(ch):
                cnt[(i, k, b)] += 1
                if op != GEQRT:
                    cnt[(piv, k, b)] += 1
        else:
            assert cnt[(i, k, cv)] >= v[0], (n, "factored tile")
            for c in range(c0, c0 + cn):
                if op == UNMQR:
                    assert cnt[(i, j, c)] >= v[1], (n, "C", c)
                else:
                    assert cnt[(piv, j, c)] >= v[1] and cnt[(i, j, c)] >= v[2], (n, "C1/C2", c)
            for c in range(c0, c0 + cn):
                cnt[(i, j, c)] += 1
                if op != UNMQR:
                    cnt[(piv, j, c)] += 1
    return cnt


CASES = [
    (24, 24, dict(nb=256, p=1, a=24, low="flat")),
    (24, 24, dict(nb=256, p=1, a=1, low="greedy")),
    (24, 24, dict(nb=256, p=1, a=8, low="greedy", high="greedy")),
    (128, 8, dict(nb=256, p=8, a=4, low="greedy", high="fibonacci", domino=1)),
    (128, 8, dict(nb=256, p=1, a=1, low="binary")),
    (40, 12, dict(nb=128, p=3, a=2, low="fibonacci", high="binary", domino=1)),
    (30, 30, dict(nb=64, p=2, a=3, low="greedy", high="flat", coupling="binary", domino=1)),
]


@pytest.mark.parametrize("mt,nt,prm", CASES, ids=[str(c[:2]) + c[2]["low"] + str(c[2].get("a")) for c in CASES])
@pytest.mark.parametrize("order", [0, 1])
def test_plan_order_is_topological(hqr_lib, mt, nt, prm, order):
    import paper_1110_1553_amd as h

    params = h.make_params(**prm)
    tasks = h._lib.plan_tasks(mt, nt, params, order)
    cnt = replay(tasks)
    # the replay does catch an order that is not topological
    with pytest.raises(AssertionError):
        replay(tasks[::-1])
    # every panel tile column is fully published, and a tile is written once per elimination or update
    assert all(x > 0 for x in cnt.values())
    if order == 0:
        # the same multiset of tasks as program order
        ref = h._lib.plan_tasks(mt, nt, params, 1)
        assert np.array_equal(np.sort(tasks.view(np.void)), np.sort(ref.view(np.void)))
        assert replay(ref) == cnt


def test_batch_order_is_topological_per_problem(hqr_lib):
    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import _lib

    params = h.make_params(nb=128, p=1, a=4, low="greedy", high="greedy")
    b = _lib.Batch([3000, 1000, 700, 2500], [256, 512, 100, 384], [1, 0, 3, 2], params)
    tasks, prob = b.tasks()
    for q in range(4):
        replay(tasks[prob == q])
    b.close()
