"""Autotuning of the tile size and the elimination tree, keyed by shape only.

The candidates are tile sizes nb in {64, 128, 256} (the inner blocking is
fixed at 16 by the tile kernels) crossed with the trees of Sections III-IV
of the paper: TT kernels only under a Greedy tree (a = 1), TS domains of a
tiles whose heads are reduced by a Greedy tree (a = 2, 4, 8, 16), and the
flat tree with TS kernels (a = number of tile rows).  Each candidate is
timed on seeded synthetic inputs of the requested shapes through the same
entry points that serve them (one batched launch, or one hqr_factor), and
the fastest is kept in a cache whose key holds only the shapes, bucketed to
tile granularity.  Every candidate computes the same factorization (to
rounding), so the choice affects speed only.
"""
import json
import os
import time

from . import _lib

TREES = (
    dict(a=1, low="greedy"),
    dict(a=2, low="greedy", high="greedy"),
    dict(a=4, low="greedy", high="greedy"),
    dict(a=8, low="greedy", high="greedy"),
    dict(a=16, low="greedy", high="greedy"),
    dict(a=1 << 20, low="flat"),
)
TILES = (64, 128, 256)


def candidates(tiles=TILES, trees=TREES):
    return [dict(nb=nb, **t) for nb in tiles for t in trees]


def _bucket(M, N, q=64):
    # tile-granular shape key: every tile size in TILES divides 256
    return (-(-int(M) // q) * q, -(-int(N) // q) * q)


class Autotuner:
    """Best parameters per shape key; ``path`` (optional) persists the cache
    as JSON."""

    def __init__(self, path=None, reps=2):
        self.path = path
        self.reps = reps
        self.cache = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.cache = {k: v for k, v in json.load(f).items()}

    def _save(self):
        if self.path:
            with open(self.path, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)

    @staticmethod
    def batch_key(shapes, nrhs):
        return "batch:" + ",".join("%dx%dx%d" % (_bucket(m, n) + (int(r),))
                                   for (m, n), r in sorted(zip(shapes, nrhs)))

    def tune_batch(self, shapes, nrhs=None, device="cuda", cands=None, seed=7):
        """Fastest parameters for one batched launch over `shapes` ((M, N)
        pairs) with nrhs[q] right-hand sides each (default 1).  Returns
        (params dict, {candidate label: seconds})."""
        import torch

        from . import BatchedLstsq, colmajor, make_exec, make_params
        from . import inputs

        nrhs = list(nrhs) if nrhs is not None else [1] * len(shapes)
        key = self.batch_key(shapes, nrhs)
        if key in self.cache:
            return self.cache[key]["params"], self.cache[key]["times"]
        A0 = [colmajor(inputs.gaussian_device(int(m), int(n), seed + q, device)) for q, (m, n) in enumerate(shapes)]
        B0 = [colmajor(inputs.gaussian_device(int(m), max(int(r), 1), seed + 50000 + q, device)[:, :int(r)])
              for q, ((m, n), r) in enumerate(zip(shapes, nrhs))]
        As = [x.clone() for x in A0]
        Bs = [x.clone() for x in B0]
        any_rhs = any(r > 0 for r in nrhs)
        times = {}
        stream = torch.cuda.current_stream(device)
        for c in (cands or candidates()):
            solver = BatchedLstsq(As, Bs if any_rhs else None, make_params(**c), make_exec(), stream=stream)
            best = float("inf")
            for rep in range(self.reps + 1):
                for x, y in zip(As, A0):
                    x.copy_(y)
                for x, y in zip(Bs, B0):
                    x.copy_(y)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                solver.run(stream)
                e1.record(stream)
                e1.synchronize()
                if rep > 0:
                    best = min(best, e0.elapsed_time(e1) / 1e3)
            st, _ = solver.status(stream)
            if st not in (0, _lib.ERR_SINGULAR):
                raise _lib.HQRError("autotune candidate %s" % c, st)
            times[json.dumps(c, sort_keys=True)] = best
            del solver
        best_c = min(times, key=times.get)
        self.cache[key] = {"params": json.loads(best_c), "times": times}
        self._save()
        return self.cache[key]["params"], times

    def tune_factor(self, M, N, device="cuda", cands=None, seed=7):
        """Fastest parameters for hqr_factor of one M x N matrix."""
        import torch

        from . import Workspace, colmajor, factor, make_exec, make_params
        from . import inputs

        key = "factor:%dx%d" % _bucket(M, N)
        if key in self.cache:
            return self.cache[key]["params"], self.cache[key]["times"]
        A0 = colmajor(inputs.gaussian_device(int(M), int(N), seed, device))
        A = A0.clone()
        stream = torch.cuda.current_stream(device)
        times = {}
        for c in (cands or candidates()):
            p = make_params(**c)
            work = Workspace(M, N, p, device=device)
            best = float("inf")
            for rep in range(self.reps + 1):
                A.copy_(A0)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                factor(A, p, make_exec(), work=work, stream=stream, check=False)
                e1.record(stream)
                e1.synchronize()
                if rep > 0:
                    best = min(best, e0.elapsed_time(e1) / 1e3)
            times[json.dumps(c, sort_keys=True)] = best
            del work
        best_c = min(times, key=times.get)
        self.cache[key] = {"params": json.loads(best_c), "times": times}
        self._save()
        return self.cache[key]["params"], times
