"""Elimination-list oracle (test infrastructure only).

A pure-Python enumeration of the elimination lists that drive the tiled QR,
written from the paper's definitions:

* Section II, Algorithm 1: a tiled QR of an m x n tile matrix is the ordered
  list of eliminations elim(i, killer(i,k), k); its validity rules (each
  (i,k), i>k, killed once; both rows ready; killer still alive) are checked
  by :func:`validate`.
* Section II, the weight paragraph: kernel weights in units of b^3/3 flops
  (GEQRT 4, UNMQR 6, TSQRT 6, TSMQR 12, TTQRT 2, TTMQR 6) and the invariant
  total 6 m n^2 - 2 n^3 (:func:`weight`).
* Section III-A/B: the flat tree (Tables 1 and 3), the binary tree
  (Table 4) and the Greedy reduction (Table 5); the Fibonacci scheme is only
  named by the paper -- the construction used here is the reading recorded
  in the design notes, pinned by the property of the cited scheme (each
  panel repeats the previous one a row lower) and by a closed form of its
  groups, not by values the paper prints.
* Section IV: the hierarchical composition HQR with TS domains of a tiles
  (level 0), a low-level tree (level 1), the coupling ("domino") tree
  (level 2) and the high-level tree (level 3), rows mapped cyclically on a
  virtual grid of p clusters; worked example of Section IV-B.
* Algorithm 2: expansion of each elimination into kernels (:func:`expand`).
* The coarse unit-time model of Section III (each elimination takes one
  time unit) gives the "Step" columns of Tables 1, 3, 4 and 5
  (:func:`unit_steps`).

A record is the 6-tuple (k, victim, killer, kind, level, round) with kind
0 = TS, 1 = TT.  This module shares no code with the GPU library's C++
generator; the two are compared record by record.
"""
from typing import Dict, List, Sequence, Tuple

FLAT, BINARY, GREEDY, FIBONACCI, CHAIN = 0, 1, 2, 3, 4
TREE_NAMES = {FLAT: "flat", BINARY: "binary", GREEDY: "greedy", FIBONACCI: "fibonacci", CHAIN: "chain"}
TS, TT = 0, 1

Record = Tuple[int, int, int, int, int, int]

# ---------------------------------------------------------------- static trees
# Each tree reduces an ascending participant list L = [r0 < r1 < ...] into r0
# and returns (victim, killer, round) triples.


def tree_flat(L: Sequence[int]):
    """Flat tree (Section III-A, Table 1): the first row kills every other
    row, top to bottom, one per round."""
    return [(L[j], L[0], j) for j in range(1, len(L))]


def tree_binary(L: Sequence[int]):
    """Binary tree (Section III-A, Table 4): at distance d = 1, 2, 4, ... the
    row at position j (j a multiple of 2d) kills the row at position j + d."""
    out = []
    s = len(L)
    d, rnd = 1, 1
    while d < s:
        for j in range(0, s, 2 * d):
            if j + d < s:
                out.append((L[j + d], L[j], rnd))
        d *= 2
        rnd += 1
    return out


def tree_fibonacci(L: Sequence[int]):
    """Fibonacci scheme of order 1 (named in Sections III-C and V, where it
    is credited to Modi and Clarke; its construction is not given in the
    paper -- reading of the design notes).

    Positions 1..s-1 are cut, from the top, into consecutive groups of
    nominal sizes 1, 2, 3, ... (the last group may be cut short by the end of
    the list).  With G groups, group g is killed in round G - g + 1 (bottom
    group first), and the victim at position v of group g is killed by
    position v - g, the row g places above it.  The killer of a position
    depends on the position only, not on the length of the list, so the next
    panel's list (one row shorter, starting one row lower) gets the same
    pattern shifted down by one row: the property of the cited scheme that
    each column repeats the previous one a row lower.  The victims of a round
    and their killers are distinct rows that are still alive (the killers of
    group g lie in groups g - 1 and g - 2)."""
    s = len(L)
    groups = []
    pos, size = 1, 1
    while pos < s:
        z = min(size, s - pos)
        groups.append((pos, z, size))
        pos += z
        size += 1
    G = len(groups)
    out = []
    for g, (start, z, nominal) in enumerate(groups, 1):
        for v in range(start, start + z):
            out.append((L[v], L[v - nominal], G - g + 1))
    return out


def tree_chain(L: Sequence[int]):
    """Domino chain (Section IV-B, level 2): bottom first, each row is killed
    by the row right above it.  The paper shows the domino level on one
    example only, whose coupling lists hold two rows; for longer lists this
    chain is a reading (design notes, D1), pinned by that example alone."""
    s = len(L)
    return [(L[j], L[j - 1], s - j) for j in range(s - 1, 0, -1)]


def greedy_panel(L: Sequence[int], ready: Dict[int, int]):
    """One panel of the Greedy reduction (Section III-B, Table 5).

    At step s every row of the panel that is ready (killed in the previous
    panel at a step < s, or never killed there) and still alive takes part;
    the bottom floor(r/2) of these r rows are killed by the floor(r/2) rows
    right above them, paired in natural order.  Returns (victim, killer, step)
    triples."""
    alive = list(L)
    out = []
    s = 0
    while len(alive) > 1:
        s += 1
        A = sorted(r for r in alive if ready.get(r, 0) < s)
        n = len(A)
        z = n // 2
        dead = set()
        for j in range(z):
            out.append((A[n - z + j], A[n - 2 * z + j], s))
            dead.add(A[n - z + j])
        alive = [r for r in alive if r not in dead]
    return out


def _static_tree(kind: int, L: Sequence[int]):
    if kind == FLAT:
        return tree_flat(L)
    if kind == BINARY:
        return tree_binary(L)
    if kind == FIBONACCI:
        return tree_fibonacci(L)
    if kind == CHAIN:
        return tree_chain(L)
    raise ValueError("unknown static tree kind %r" % kind)


class _TreeRunner:
    """Runs a tree kind on successive panels, carrying the Greedy readiness of
    each (level, group) from one panel to the next."""

    def __init__(self):
        self.prev: Dict[Tuple[int, int], Dict[int, int]] = {}
        self.cur: Dict[Tuple[int, int], Dict[int, int]] = {}

    def next_panel(self):
        self.prev, self.cur = self.cur, {}

    def run(self, kind: int, level: int, group: int, L: Sequence[int]):
        if len(L) < 2:
            return []
        if kind == GREEDY:
            trip = greedy_panel(L, self.prev.get((level, group), {}))
            mem = self.cur.setdefault((level, group), {})
            for v, _, s in trip:
                mem[v] = s
            return trip
        return _static_tree(kind, L)


# ------------------------------------------------------------ HQR composition

def hqr_elimlist(mt: int, nt: int, p: int = 1, a: int = 1, low: int = FLAT, high: int = FLAT,
                 coupling: int = CHAIN, domino: int = 0) -> List[Record]:
    """Elimination list of the hierarchical algorithm (Section IV).

    Rows are mapped cyclically onto p virtual clusters: cluster c(i) = i mod p,
    local index l(i) = i // p.  For panel k and cluster c:
      Loc = {l : k <= l p + c < mt}, top tile t = min Loc (the p top tiles
      are the global rows k .. k+p-1);
      with the coupling level (domino = 1) S = {l in Loc : l >= k} (on or
      below the local diagonal) and the level-2 list is [t] + {l : t < l <= k};
      without it S = Loc.
      level 0 (TS): s0 = min S; every l in S other than s0 is killed by
        h = max(a * (l // a), s0) when h != l (domains of a tiles);
      level 1 (low tree, TT) over [s0] + {l in S : l > s0, a | l};
      level 2 (coupling tree, TT) over the level-2 list;
      level 3 (high tree, TT) over the sorted top tiles of all clusters.
    Records are emitted per panel in the canonical order: level 0 by
    (cluster, killer, victim), levels 1 and 2 by (cluster, round, victim),
    level 3 by (round, victim)."""
    if mt < 1 or nt < 1 or p < 1 or a < 1:
        raise ValueError("bad sizes")
    runner = _TreeRunner()
    recs: List[Record] = []
    for k in range(min(mt, nt)):
        runner.next_panel()
        lv0, lv1, lv2 = [], [], []
        tops = []
        for c in range(p):
            Loc = [l for l in range(0, (mt - c + p - 1) // p) if k <= l * p + c < mt]
            if not Loc:
                continue
            t = Loc[0]
            tops.append(t * p + c)
            if domino:
                S = [l for l in Loc if l >= k]
                L2 = [t] + [l for l in Loc if t < l <= k]
            else:
                S = list(Loc)
                L2 = []
            g = lambda l, c=c: l * p + c  # noqa: E731  local -> global row
            if S:
                s0 = S[0]
                for l in S[1:]:
                    h = max(a * (l // a), s0)
                    if h != l:
                        lv0.append((c, g(h), g(l), l - h))
                L1 = [s0] + [l for l in S if l > s0 and l % a == 0]
                for v, kk, r in runner.run(low, 1, c, [g(l) for l in L1]):
                    lv1.append((c, r, v, kk))
            if len(L2) > 1:
                for v, kk, r in runner.run(coupling, 2, c, [g(l) for l in L2]):
                    lv2.append((c, r, v, kk))
        lv3 = [(r, v, kk) for v, kk, r in runner.run(high, 3, 0, sorted(tops))]
        for c, kk, v, r in sorted(lv0):
            recs.append((k, v, kk, TS, 0, r))
        for c, r, v, kk in sorted(lv1):
            recs.append((k, v, kk, TT, 1, r))
        for c, r, v, kk in sorted(lv2):
            recs.append((k, v, kk, TT, 2, r))
        for r, v, kk in sorted(lv3):
            recs.append((k, v, kk, TT, 3, r))
    return recs


# ---------------------------------------------------------------- validation

def validate(mt: int, nt: int, recs: Sequence[Record]) -> None:
    """Raise ValueError unless the list obeys the rules of Section II:
    every tile (i,k), i > k, k < min(m,n), is killed exactly once; when
    elim(i, piv, k) runs, rows i and piv have been zeroed in every panel
    k' < k and piv has not been killed in panel k yet.  In addition a TS
    victim must still be a square tile: it is never a killer in that panel."""
    K = min(mt, nt)
    killed = set()
    for idx, (k, i, piv, kind, level, rnd) in enumerate(recs):
        if not (0 <= k < K and k <= piv < mt and k < i < mt and piv != i):
            raise ValueError("record %d out of range: %r" % (idx, recs[idx]))
        if (i, k) in killed:
            raise ValueError("tile (%d,%d) killed twice" % (i, k))
        if (piv, k) in killed:
            raise ValueError("killer %d of (%d,%d) is already zero" % (piv, i, k))
        for row in (i, piv):
            for kp in range(k):
                if row > kp and (row, kp) not in killed:
                    raise ValueError("row %d not ready for panel %d" % (row, k))
        killed.add((i, k))
    for k in range(K):
        for i in range(k + 1, mt):
            if (i, k) not in killed:
                raise ValueError("tile (%d,%d) never killed" % (i, k))
    ts_victims = {(k, i) for (k, i, piv, kind, _, _) in recs if kind == TS}
    for (k, i, piv, kind, _, _) in recs:
        if (k, piv) in ts_victims:
            raise ValueError("TS victim %d used as a killer in panel %d" % (piv, k))


# ------------------------------------------------------------ kernel expansion

WEIGHT = {"GEQRT": 4, "UNMQR": 6, "TSQRT": 6, "TSMQR": 12, "TTQRT": 2, "TTMQR": 6}


def expand(mt: int, nt: int, recs: Sequence[Record]):
    """Kernel tasks of a list (Algorithm 2).  In each panel k, every row r >= k
    that is not a TS victim is triangularised once (GEQRT(r,k) and its
    UNMQR(r,k,j) for j > k) before its first elimination; a TS elimination is
    TSQRT + TSMQR(j > k), a TT elimination TTQRT + TTMQR(j > k).  Tasks are
    tuples (name, row, killer, k, j) with -1 for unused fields."""
    tasks = []
    K = min(mt, nt)
    by_panel: Dict[int, List[Record]] = {}
    for r in recs:
        by_panel.setdefault(r[0], []).append(r)
    for k in range(K):
        pr = by_panel.get(k, [])
        ts = {i for (_, i, _, kind, _, _) in pr if kind == TS}
        for r in range(k, mt):
            if r in ts:
                continue
            tasks.append(("GEQRT", r, -1, k, -1))
            for j in range(k + 1, nt):
                tasks.append(("UNMQR", r, -1, k, j))
        for (_, i, piv, kind, _, _) in pr:
            q, u = ("TSQRT", "TSMQR") if kind == TS else ("TTQRT", "TTMQR")
            tasks.append((q, i, piv, k, -1))
            for j in range(k + 1, nt):
                tasks.append((u, i, piv, k, j))
    return tasks


def weight(tasks) -> int:
    return sum(WEIGHT[t[0]] for t in tasks)


def weight_formula(mt: int, nt: int) -> int:
    """6 m n^2 - 2 n^3 for m >= n (Section II)."""
    return 6 * mt * nt * nt - 2 * nt ** 3


# ------------------------------------------------------------ unit-time model

def unit_steps(mt: int, nt: int, recs: Sequence[Record]) -> Dict[Tuple[int, int], int]:
    """Step at which each tile (i,k) is zeroed when every elimination takes
    one time unit and starts as soon as both rows are ready (zeroed in the
    previous panel) and have finished their earlier eliminations of the same
    panel (Section III, coarse-grain model)."""
    steps: Dict[Tuple[int, int], int] = {}
    by_panel: Dict[int, List[Record]] = {}
    for r in recs:
        by_panel.setdefault(r[0], []).append(r)
    for k in range(min(mt, nt)):
        last: Dict[int, int] = {}
        for (_, i, piv, _, _, _) in by_panel.get(k, []):
            ready_i = steps.get((i, k - 1), 0) if k > 0 else 0
            ready_p = steps.get((piv, k - 1), 0) if k > 0 else 0
            s = 1 + max(ready_i, ready_p, last.get(i, 0), last.get(piv, 0))
            steps[(i, k)] = s
            last[i] = s
            last[piv] = s
    return steps


def killers(recs: Sequence[Record]) -> Dict[Tuple[int, int], int]:
    return {(i, k): piv for (k, i, piv, _, _, _) in recs}
