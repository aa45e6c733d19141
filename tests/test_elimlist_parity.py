"""The library's C++ elimination-list generator against the independent
Python enumeration in oracle/elimlist.py: identical records (bit-exact),
the same kernel counts and weights, and the same verdicts of the validity
rules of Section II."""
import random

import numpy as np
import pytest

from oracle import elimlist as el

TREES = [el.FLAT, el.BINARY, el.GREEDY, el.FIBONACCI]


def ref_list(mt, nt, p, a, low, high, coupling, domino):
    return np.array(el.hqr_elimlist(mt, nt, p, a, low, high, coupling, domino), dtype=np.int32).reshape(-1, 6)


def lib_list(mt, nt, p, a, low, high, coupling, domino):
    import paper_1110_1553_amd as h

    return h.elimlist(mt, nt, h.make_params(nb=64, p=p, a=a, low=low, high=high, coupling=coupling, domino=domino))


CASES = [
    # (mt, nt, p, a, low, high, coupling, domino)
    (12, 3, 1, 1, el.FLAT, el.FLAT, el.CHAIN, 0),
    (12, 3, 1, 1, el.BINARY, el.FLAT, el.CHAIN, 0),
    (12, 3, 1, 1, el.GREEDY, el.FLAT, el.CHAIN, 0),
    (24, 10, 3, 2, el.GREEDY, el.FIBONACCI, el.CHAIN, 1),
    (8, 4, 1, 8, el.FLAT, el.FLAT, el.CHAIN, 0),            # 512x256, nb=64, flat tree, TS kernels
    (512, 8, 8, 4, el.GREEDY, el.FIBONACCI, el.CHAIN, 1),   # 131072x2048, nb=256, hierarchical
    (512, 8, 1, 512, el.FLAT, el.FLAT, el.CHAIN, 0),        # same shape, flat tree TS
    (512, 8, 1, 1, el.BINARY, el.FLAT, el.CHAIN, 0),        # same shape, binary tree TT
    (64, 64, 1, 1, el.GREEDY, el.FLAT, el.CHAIN, 0),        # 16384^2, nb=256, Greedy TT
    (64, 64, 1, 64, el.FLAT, el.FLAT, el.CHAIN, 0),         # 16384^2, flat tree TS
]


@pytest.mark.parametrize("case", CASES, ids=[str(c[:4]) for c in CASES])
def test_named_configurations_bit_exact(hqr_lib, case):
    a = lib_list(*case)
    b = ref_list(*case)
    assert a.shape == b.shape
    assert a.tobytes() == b.tobytes()


def test_random_sweep_bit_exact(hqr_lib):
    rng = random.Random(20240607)
    for _ in range(400):
        mt = rng.randint(1, 48)
        nt = rng.randint(1, min(mt, 14))
        case = (mt, nt, rng.randint(1, 7), rng.randint(1, 9), rng.choice(TREES), rng.choice(TREES),
                rng.choice(TREES + [el.CHAIN]), rng.randint(0, 1))
        a, b = lib_list(*case), ref_list(*case)
        assert a.tobytes() == b.tobytes(), case


def test_dag_counts_and_weight_match(hqr_lib):
    import paper_1110_1553_amd as h

    rng = random.Random(77)
    for _ in range(60):
        mt = rng.randint(1, 30)
        nt = rng.randint(1, min(mt, 10))
        p, a = rng.randint(1, 5), rng.randint(1, 6)
        low, high, cpl, dom = rng.choice(TREES), rng.choice(TREES), rng.choice(TREES + [el.CHAIN]), rng.randint(0, 1)
        st = h.dag_stats(mt, nt, h.make_params(nb=256, p=p, a=a, low=low, high=high, coupling=cpl, domino=dom))
        tasks = el.expand(mt, nt, el.hqr_elimlist(mt, nt, p, a, low, high, cpl, dom))
        counts = {op: sum(1 for t in tasks if t[0] == op) for op in h.OPS}
        assert st["count"] == counts
        assert st["weight"] == el.weight(tasks) == el.weight_formula(mt, nt)
        updates = sum(counts[o] for o in ("UNMQR", "TSMQR", "TTMQR"))
        assert st["device_tasks"] == len(tasks) + updates  # 2 column chunks of 128 at nb = 256


def test_task_counts_closed_form(hqr_lib):
    # flat TS on 8 x 4 tiles: sum over k of 1 GEQRT, 7 - k TSQRT, 3 - k UNMQR
    # and (7 - k)(3 - k) TSMQR = 32 + 21 + 12 + 5 tasks; 64 x 64 tiles: every
    # tile below the diagonal is killed once (2016 kills, plus 64 GEQRT under
    # flat TS, 2080 GEQRT under TT), each with its updates to the right
    import paper_1110_1553_amd as h

    assert h.dag_stats(8, 4, h.make_params(nb=64, a=8, low="flat"))["tasks"] == 70
    assert h.dag_stats(64, 64, h.make_params(nb=256, a=1, low="greedy"))["tasks"] == 176800
    assert h.dag_stats(64, 64, h.make_params(nb=256, a=64, low="flat"))["tasks"] == 89440


def test_validator_agrees_with_oracle(hqr_lib):
    import paper_1110_1553_amd as h

    recs = el.hqr_elimlist(10, 4, 2, 2, el.GREEDY, el.BINARY, el.CHAIN, 1)
    assert h.validate(10, 4, recs) == 0
    broken = [
        recs[:-1],                          # a tile never killed
        recs + [recs[3]],                   # a tile killed twice
        recs[1:] + recs[:1],                # a row not ready
        [(0, 1, 0, 1, 1, 1), (0, 2, 1, 1, 1, 2)] + [r for r in recs if r[0] > 0 or r[1] > 2],  # dead killer
    ]
    for b in broken:
        with pytest.raises(ValueError):
            el.validate(10, 4, b)
        assert h.validate(10, 4, b) != 0
    # TS victim used as a killer
    ts = [(0, 2, 0, el.TS, 0, 1), (0, 1, 2, el.TT, 1, 1)] + [r for r in recs if r[0] > 0 or r[1] > 2]
    with pytest.raises(ValueError):
        el.validate(10, 4, ts)
    assert h.validate(10, 4, ts) != 0
