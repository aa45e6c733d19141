"""Continuous-batching least-squares serving on one GPU.

Requests (A_q: M_q x N_q, b_q: M_q x nrhs_q, both already in device memory)
arrive over time and wait in a FIFO queue.  Whenever fewer than
``max_inflight`` batches are on the GPU and requests are waiting, the
scheduler admits requests from the head of the queue while the batch
workspace still fits in one slot of the HBM budget (the budget is split into
``max_inflight`` workspace slots, allocated once), plans the batch on the
host and launches it as one batched launch (copy-in, one persistent launch
over the union of the task graphs, back substitution, copy-out).  Each
workspace slot has its own stream: a batch admitted while another runs is
launched at once, and its persistent workgroups take the compute units that
the running batch releases as its task list drains, so the two overlap on
the device.  A request completes with the end event of its batch; its
latency is that time minus its arrival time.

With a factor budget, the factorization of every served request (its T
factors and factored tiles) is copied out of the batch workspace into a
workspace of its own and kept on the device, least recently used first out
when the budget is full, so that later right-hand sides for the same matrix
are solved without factoring again (``GpuBackend.solve_resident``).

A request's results do not depend on the batch it was served in: each
problem of a batched launch runs the same tasks in the same per-tile order
as a launch of that problem alone, so they are bitwise identical.

The scheduling logic is separate from the GPU backend (``GpuBackend``) so
that it can be exercised with a simulated backend.
"""
import collections
import time

import numpy as np

from . import _lib


class FactorStore:
    """Device-resident factorizations under a byte budget, least recently
    used evicted first."""

    def __init__(self, budget_bytes):
        self.budget = int(budget_bytes)
        self.used = 0
        self.items = collections.OrderedDict()  # rid -> (bytes, object)
        self.evicted = 0

    def put(self, rid, nbytes, obj):
        if nbytes > self.budget:
            return False
        while self.used + nbytes > self.budget and self.items:
            _, (b, _) = self.items.popitem(last=False)
            self.used -= b
            self.evicted += 1
        self.items[rid] = (nbytes, obj)
        self.used += nbytes
        return True

    def get(self, rid):
        if rid not in self.items:
            return None
        self.items.move_to_end(rid)
        return self.items[rid][1]


class GpuBackend:
    """Launches batches through hqr_batch_*, one stream per workspace slot,
    with the slots carved out of one preallocated device buffer."""

    def __init__(self, params, budget_bytes, max_inflight=2, device="cuda", exec_=None, factor_budget=0):
        import torch

        self.params = params
        self.exec_ = exec_ if exec_ is not None else _lib.make_exec()
        self.device = torch.device(device)
        # every stream is created by torch at the default priority and is
        # non-blocking with respect to the null stream; `side` serves the
        # solves with kept factorizations
        self.streams = [torch.cuda.Stream(self.device) for _ in range(max_inflight)]
        self.stream = self.streams[0]
        self.side = torch.cuda.Stream(self.device)
        self.store = FactorStore(factor_budget) if factor_budget > 0 else None
        self.slots = max_inflight
        self.slot_bytes = (int(budget_bytes) // max_inflight) & ~255
        self.pool = torch.empty(self.slot_bytes * max_inflight, dtype=torch.uint8, device=self.device)
        self.free = list(range(max_inflight))
        # per slot, pinned host words into which a batch's last kernel writes
        # its status: a finished batch is read without a device-to-host copy
        # (which would queue behind the other slot's persistent launch)
        self.status_host = [None] * max_inflight
        self._ws = {}
        self.t0_event = None

    # -- sizes -------------------------------------------------------------
    def request_bytes(self, M, N, nrhs):
        """Workspace estimate of one request inside a batch (its tiles, T
        factors and counters, plus room for its task records)."""
        key = (int(M), int(N), int(nrhs))
        b = self._ws.get(key)
        if b is None:
            nb = self.params.nb
            mt, nt, nrt = -(-M // nb), -(-N // nb), -(-nrhs // nb)
            tasks = mt * nt * (nt + nrt) * 4 + 64  # above the update and panel task count of any tree
            b = _lib.lstsq_workspace_size(M, N, nrhs, self.params) if nrhs > 0 else _lib.workspace_size(M, N, self.params)
            b += tasks * 28 + 512
            self._ws[key] = b
        return b

    # -- clock ---------------------------------------------------------------
    def start_clock(self):
        import torch

        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_event.record(self.stream)
        self.t0_host = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0_host

    def sleep(self, dt):
        time.sleep(dt)

    # -- batches -------------------------------------------------------------
    def launch(self, reqs):
        """Plans, binds and launches the batch; returns a handle, or None
        when its workspace exceeds a slot (the caller shrinks the batch)."""
        import torch

        M = [r.A.shape[0] for r in reqs]
        N = [r.A.shape[1] for r in reqs]
        nrhs = [r.B.shape[1] for r in reqs]
        batch = _lib.Batch(M, N, nrhs, self.params, self.exec_)
        need = batch.workspace_size()
        if need > self.slot_bytes:
            batch.close()
            return None
        slot = self.free.pop(0)
        st = self.streams[slot]
        base = self.pool.data_ptr() + slot * self.slot_bytes
        batch.bind([r.A.data_ptr() for r in reqs], [max(r.A.stride(1), r.A.shape[0]) for r in reqs],
                   [r.B.data_ptr() for r in reqs], [max(r.B.stride(1), r.B.shape[0]) for r in reqs],
                   base, self.slot_bytes, st.cuda_stream)
        batch.run(base, self.slot_bytes, st.cuda_stream)
        words = self.status_host[slot]
        if words is None or words.numel() < len(reqs) + 1:
            words = torch.zeros(max(len(reqs) + 1, 4097), dtype=torch.int32, pin_memory=True)
            self.status_host[slot] = words
        batch.publish_status(base, words.data_ptr(), st.cuda_stream)
        kept = []
        if self.store is not None:
            from . import Workspace

            with torch.cuda.stream(st):
                for r in reqs:
                    kept.append((r, Workspace(r.M, r.N, self.params, device=self.device)))
            batch.export_all(base, [w.ptr for _, w in kept], [w.bytes for _, w in kept], st.cuda_stream)
        end = torch.cuda.Event(enable_timing=True)
        end.record(st)
        return {"batch": batch, "slot": slot, "base": base, "end": end, "kept": kept}

    def done(self, h):
        """Completion time (seconds since start_clock) or None if running."""
        if not h["end"].query():
            return None
        t = self.t0_event.elapsed_time(h["end"]) / 1e3
        words = self.status_host[h["slot"]].numpy()[: h["batch"].count + 1].copy()
        h["status"], h["first_zero"] = int(words[0]), words[1:]
        h["batch"].close()
        self.free.append(h["slot"])
        for r, w in h.get("kept", []):
            self.store.put(r.rid, w.bytes, w)
        return t

    def solve_resident(self, rid, M, N, B):
        """Least squares for new right-hand sides B (M x nrhs, column-major,
        overwritten as hqr_solve does) with the kept factorization of
        request rid; returns False if it was evicted."""
        import torch

        from . import solve

        w = self.store.get(rid) if self.store is not None else None
        if w is None:
            return False
        # the kept workspace was allocated on a slot stream: tell the caching
        # allocator that the side stream uses it too, so that an eviction
        # does not hand its memory to new work while the solve still reads it;
        # the solve's own scratch is allocated on the side stream
        w.buf.record_stream(self.side)
        B.record_stream(self.side)
        with torch.cuda.stream(self.side):
            solve(B, M, N, self.params, w, self.exec_, stream=self.side)
        return True


class Request:
    __slots__ = ("rid", "A", "B", "M", "N", "nrhs", "arrival", "done", "status", "first_zero")

    def __init__(self, rid, A, B, arrival):
        self.rid, self.A, self.B, self.arrival = rid, A, B, arrival
        self.M, self.N = A.shape
        self.nrhs = B.shape[1]
        self.done = None
        self.status = None
        self.first_zero = None


class Scheduler:
    """FIFO admission under a per-slot byte budget and continuous batching
    over a backend with ``backend.slots`` workspace slots (at most that many
    batches in flight)."""

    def __init__(self, backend, max_batch=4096, poll_s=20e-6):
        self.backend = backend
        self.max_inflight = backend.slots
        self.max_batch = max_batch
        self.poll_s = poll_s
        self.batches = []

    def admit(self, queue):
        """Requests for the next batch: the longest FIFO prefix whose
        estimated workspace fits a slot (at least the head)."""
        out, used = [], 0
        cap = self.backend.slot_bytes
        while queue and len(out) < self.max_batch:
            r = queue[0]
            b = self.backend.request_bytes(r.M, r.N, r.nrhs)
            if out and used + b > cap:
                break
            out.append(queue.popleft())
            used += b
        return out

    def run(self, requests):
        """Serves `requests` (sorted by arrival, seconds from the start) in
        real time; returns the per-request latencies (seconds)."""
        be = self.backend
        queue = collections.deque()
        inflight = []
        nxt, finished = 0, 0
        n = len(requests)
        be.start_clock()
        while finished < n:
            now = be.now()
            while nxt < n and requests[nxt].arrival <= now:
                queue.append(requests[nxt])
                nxt += 1
            # retire finished batches (in launch order)
            while inflight:
                t = be.done(inflight[0]["h"])
                if t is None:
                    break
                b = inflight.pop(0)
                fz = b["h"].get("first_zero")
                for q, r in enumerate(b["reqs"]):
                    r.done = t
                    r.status = b["h"].get("status", 0)
                    r.first_zero = int(fz[q]) if fz is not None else -1
                finished += len(b["reqs"])
                b["t_done"] = t
            if queue and len(inflight) < self.max_inflight:
                reqs = self.admit(queue)
                h = be.launch(reqs)
                while h is None and len(reqs) > 1:  # the estimate was short: give back the tail
                    half = len(reqs) // 2
                    for r in reversed(reqs[half:]):
                        queue.appendleft(r)
                    reqs = reqs[:half]
                    h = be.launch(reqs)
                if h is None:
                    raise RuntimeError("request %d does not fit a workspace slot" % reqs[0].rid)
                rec = {"reqs": reqs, "h": h, "t_launch": be.now()}
                inflight.append(rec)
                self.batches.append(rec)
                continue
            if not inflight and not queue and nxt < n:
                wait = requests[nxt].arrival - be.now()
                if wait > 0:
                    be.sleep(min(wait, 1e-3))
            elif inflight:
                be.sleep(self.poll_s)
        return np.array([r.done - r.arrival for r in requests])


def summarize(latencies, requests, span_s):
    lat = np.asarray(latencies)
    return {
        "requests": len(requests),
        "solves_per_s": len(requests) / span_s,
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "max_ms": float(lat.max() * 1e3),
        "span_s": span_s,
    }
