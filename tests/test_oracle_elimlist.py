"""Pins of the elimination-list oracle against the paper's tables and text.

* Tables 1 and 3: flat tree killers and unit-model steps (all cells).
* Table 4: binary tree killers (all cells) and panel-0 steps.
* Table 5: Greedy killers and steps (all cells but the two garbled killer
  cells of panel 2, rows 5 and 6, pinned to the rule printed with the table).
* Section IV-B worked example (m=24, n=10, p=3, a=2): the named eliminations
  and their levels, the TS victims (odd local rows under the local diagonal)
  and tile (6,2) as cluster 0's local-diagonal survivor of panel 2.
* Section II: exactly one elimination per tile below the diagonal, validity
  rules, and the weight invariant 6 m n^2 - 2 n^3 for every list.
"""
import itertools
import os
import math
import random

import pytest

from oracle import elimlist as el


def read_table(path):
    rows = []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        rows.append(line.split())
    return rows


def table_cells(path, panels):
    """{(row, panel): (killer, step)} for the killed cells of a 3-panel table."""
    cells = {}
    for f in read_table(path):
        row = int(f[0])
        for k in range(panels):
            kk, st = f[1 + 2 * k], f[2 + 2 * k]
            if kk != "*":
                cells[(row, k)] = (int(kk), int(st) if st != "-" else None)
    return cells


def test_table1_flat_panel0(golden_dir):
    recs = el.hqr_elimlist(12, 1, low=el.FLAT)
    steps, kill = el.unit_steps(12, 1, recs), el.killers(recs)
    for (row, k), (kk, st) in table_cells(os.path.join(golden_dir, "table1_flat_panel0.txt"), 1).items():
        assert kill[(row, k)] == kk and steps[(row, k)] == st


def test_table3_flat_three_panels(golden_dir):
    recs = el.hqr_elimlist(12, 3, low=el.FLAT)
    steps, kill = el.unit_steps(12, 3, recs), el.killers(recs)
    cells = table_cells(os.path.join(golden_dir, "table3_flat_3panels.txt"), 3)
    assert len(cells) == len(recs) == 11 + 10 + 9
    for (row, k), (kk, st) in cells.items():
        assert kill[(row, k)] == kk, (row, k)
        assert steps[(row, k)] == st, (row, k)


def test_table4_binary_killers_and_panel0_steps(golden_dir):
    recs = el.hqr_elimlist(12, 3, low=el.BINARY)
    steps, kill = el.unit_steps(12, 3, recs), el.killers(recs)
    cells = table_cells(os.path.join(golden_dir, "table4_binary_3panels.txt"), 3)
    assert len(cells) == len(recs)
    for (row, k), (kk, st) in cells.items():
        assert kill[(row, k)] == kk, (row, k)
        if k == 0:
            assert steps[(row, k)] == st, (row, k)


def test_table5_greedy(golden_dir):
    recs = el.hqr_elimlist(12, 3, low=el.GREEDY)
    steps, kill = el.unit_steps(12, 3, recs), el.killers(recs)
    cells = table_cells(os.path.join(golden_dir, "table5_greedy_3panels.txt"), 3)
    # the two garbled cells: the pairing rule (z rows right above kill in natural order)
    garbled = {(5, 2): 3, (6, 2): 4}
    for (row, k), (kk, st) in cells.items():
        assert kill[(row, k)] == garbled.get((row, k), kk), (row, k)
        assert steps[(row, k)] == st, (row, k)
    # greedy rounds are its steps
    for (k, i, piv, kind, level, rnd) in recs:
        assert rnd == steps[(i, k)]


def test_hqr_worked_example(golden_dir):
    mt, nt, p, a = 24, 10, 3, 2
    for high in (el.FLAT, el.BINARY):
        recs = el.hqr_elimlist(mt, nt, p=p, a=a, low=el.GREEDY, high=high, coupling=el.CHAIN, domino=1)
        el.validate(mt, nt, recs)
        by = {(k, i): (piv, kind, level) for (k, i, piv, kind, level, _) in recs}
        for f in read_table(os.path.join(golden_dir, "hqr_example_m24_p3_a2.txt")):
            k, i, piv, level = map(int, f)
            assert by[(k, i)][0] == piv and by[(k, i)][2] == level
        # level-0 (TS) victims: odd local rows strictly under the local diagonal, killed by the tile above
        for (k, i, piv, kind, level, _) in recs:
            l, c = divmod(i, p)
            if level == 0:
                assert kind == el.TS and l % 2 == 1 and l > k and piv == i - p
            else:
                assert kind == el.TT
        for k in range(nt):
            for i in range(k + 1, mt):
                l = i // p
                if l > k and l % 2 == 1:
                    assert by[(k, i)][2] == 0
        # tile (6,2) is cluster 0's local-diagonal killer for panel 2: it survives levels 0 and 1
        # and is then killed at level 2 by cluster 0's top tile
        victims01 = {i for (k, i, _, _, level, _) in recs if k == 2 and level <= 1}
        killers01 = {piv for (k, _, piv, _, level, _) in recs if k == 2 and level <= 1 and piv % p == 0}
        assert 6 not in victims01 and 6 in killers01
        assert by[(2, 6)][2] == 2


@pytest.mark.parametrize("mt,nt", [(8, 4), (512, 8), (64, 64)])
def test_counts_one_elimination_per_tile(mt, nt):
    recs = el.hqr_elimlist(mt, nt, p=1, a=1, low=el.GREEDY)
    assert len(recs) == sum(mt - k - 1 for k in range(min(mt, nt)))


def test_named_special_cases():
    # p=1, a >= m: flat tree with TS kernels everywhere
    recs = el.hqr_elimlist(8, 4, p=1, a=8)
    assert all(kind == el.TS and piv == k for (k, i, piv, kind, _, _) in recs)
    tasks = el.expand(8, 4, recs)
    assert len(tasks) == 70
    # p=1, a=1: single low-level tree, TT kernels only
    recs = el.hqr_elimlist(12, 3, p=1, a=1, low=el.BINARY)
    assert all(kind == el.TT and level == 1 for (_, _, _, kind, level, _) in recs)


def test_fibonacci_construction_example():
    # 15 rows: groups of nominal sizes 1, 2, 3, 4, 5 from the top, the last one cut to 4 rows by the
    # end of the list; the bottom group goes first, each victim killed by the row g places above it
    trip = el.tree_fibonacci(list(range(15)))
    got = {v: (kk, r) for v, kk, r in trip}
    assert sorted(got) == list(range(1, 15))
    assert got[1] == (0, 5) and got[2] == (0, 4) and got[3] == (1, 4)
    assert [got[v] for v in (4, 5, 6)] == [(1, 3), (2, 3), (3, 3)]
    assert [got[v] for v in (7, 8, 9, 10)] == [(3, 2), (4, 2), (5, 2), (6, 2)]
    assert [got[v] for v in (11, 12, 13, 14)] == [(6, 1), (7, 1), (8, 1), (9, 1)]


def _fib_group(v):
    """Group of position v >= 1 in closed form: the least g with g (g + 1) / 2 >= v."""
    g = (math.isqrt(8 * v) - 1) // 2
    while g * (g + 1) // 2 < v:
        g += 1
    return g


def test_fibonacci_closed_form():
    # killer position v - g(v), round G - g(v) + 1 with G = g(s - 1), for every list length
    for s in range(1, 200):
        trip = el.tree_fibonacci(list(range(s)))
        assert len(trip) == s - 1
        G = _fib_group(s - 1) if s > 1 else 0
        for v, kk, r in trip:
            g = _fib_group(v)
            assert (kk, r) == (v - g, G - g + 1), (s, v)


def test_fibonacci_panels_shift_one_row():
    # the cited scheme repeats each column's pattern one row lower in the next column: in a
    # single-tree run, the killer of row i in panel k is one more than the killer of row i - 1 in
    # panel k - 1 (a wrong group offset anywhere breaks this for some list length)
    for mt in range(2, 48):
        for nt in (1, 2, min(mt, 5), mt):
            recs = el.hqr_elimlist(mt, nt, p=1, a=1, low=el.FIBONACCI)
            el.validate(mt, nt, recs)
            killer = {(k, i): piv for (k, i, piv, _, _, _) in recs}
            for (k, i), piv in killer.items():
                if k > 0:
                    assert piv == killer[(k - 1, i - 1)] + 1, (mt, nt, k, i)


TREES = [el.FLAT, el.BINARY, el.GREEDY, el.FIBONACCI]


def _random_params(rng):
    mt = rng.randint(1, 40)
    nt = rng.randint(1, min(mt, 12))
    return dict(mt=mt, nt=nt, p=rng.randint(1, 6), a=rng.randint(1, 9), low=rng.choice(TREES),
                high=rng.choice(TREES), coupling=rng.choice(TREES + [el.CHAIN]), domino=rng.randint(0, 1))


def test_random_lists_valid_and_weight_invariant():
    rng = random.Random(1234)
    for _ in range(300):
        prm = _random_params(rng)
        mt, nt = prm.pop("mt"), prm.pop("nt")
        recs = el.hqr_elimlist(mt, nt, **prm)
        el.validate(mt, nt, recs)
        assert el.weight(el.expand(mt, nt, recs)) == el.weight_formula(mt, nt)


def test_validator_rejects_bad_lists():
    recs = el.hqr_elimlist(6, 3, low=el.FLAT)
    with pytest.raises(ValueError):
        el.validate(6, 3, recs[:-1])  # a tile never killed
    with pytest.raises(ValueError):
        el.validate(6, 3, recs + [recs[0]])  # killed twice
    bad = list(recs)
    # kill row 1 of panel 1 before row 1 is ready (swap a panel-0 elimination to the end)
    first = bad.pop(0)
    bad.append(first)
    with pytest.raises(ValueError):
        el.validate(6, 3, bad)
    # a killer that is already zero: kill (2,0) with row 1 after (1,0) was killed by 0
    bad2 = [(0, 1, 0, el.TT, 1, 1), (0, 2, 1, el.TT, 1, 2)] + [r for r in recs if r[0] > 0 or r[1] > 2]
    with pytest.raises(ValueError):
        el.validate(6, 3, bad2)
