"""The continuous-batching scheduler (paper_1110_1553_amd.serve) against a
simulated GPU: every request is served exactly once and in FIFO order,
batches respect the workspace budget and the in-flight limit, a batch whose
real workspace is larger than estimated is split, and latencies follow the
simulated service times."""
import numpy as np
import pytest

from paper_1110_1553_amd import serve


class SimBackend:
    """A GPU that runs batches one after another; a batch takes
    `per_batch` seconds plus `per_byte` seconds per byte of its requests.
    Virtual clock: sleep() advances it."""

    def __init__(self, slot_bytes, slots=2, per_batch=1e-3, per_byte=1e-9, real_factor=1.0):
        self.slot_bytes, self.slots = slot_bytes, slots
        self.per_batch, self.per_byte, self.real_factor = per_batch, per_byte, real_factor
        self.t = 0.0
        self.gpu_free_at = 0.0
        self.inflight = 0
        self.max_seen = 0
        self.launched = []

    def request_bytes(self, M, N, nrhs):
        return M * N * 8

    def start_clock(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += dt

    def launch(self, reqs):
        real = sum(self.request_bytes(r.M, r.N, r.nrhs) for r in reqs) * self.real_factor
        if len(reqs) > 1 and real > self.slot_bytes:
            return None
        start = max(self.t, self.gpu_free_at)
        end = start + self.per_batch + self.per_byte * real
        self.gpu_free_at = end
        self.inflight += 1
        self.max_seen = max(self.max_seen, self.inflight)
        self.launched.append([r.rid for r in reqs])
        return {"end": end, "n": len(reqs)}

    def done(self, h):
        if self.t < h["end"]:
            return None
        self.inflight -= 1
        h["status"], h["first_zero"] = 0, np.full(h["n"], -1)
        return h["end"]


class Mat:
    def __init__(self, M, N):
        self.shape = (M, N)


def make_requests(n, rate, seed, mmax=4096):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    out = []
    for q in range(n):
        M = int(rng.integers(64, mmax))
        N = int(rng.integers(8, min(M, 512) + 1))
        out.append(serve.Request(q, Mat(M, N), Mat(M, 1), float(t[q])))
    return out


@pytest.mark.parametrize("slots", [1, 2, 3])
def test_every_request_served_once_in_fifo_order(slots):
    reqs = make_requests(400, rate=2000.0, seed=slots)
    be = SimBackend(slot_bytes=64 << 20, slots=slots)
    sch = serve.Scheduler(be)
    lat = sch.run(reqs)
    flat = [rid for b in be.launched for rid in b]
    assert flat == list(range(len(reqs)))           # FIFO, each once
    assert be.max_seen <= slots
    assert (lat > 0).all()
    for b in sch.batches:                            # admission respects the slot budget
        est = sum(be.request_bytes(r.M, r.N, r.nrhs) for r in b["reqs"])
        assert len(b["reqs"]) == 1 or est <= be.slot_bytes
        assert all(r.done >= r.arrival for r in b["reqs"])
        assert all(b["t_launch"] >= r.arrival for r in b["reqs"])
    s = serve.summarize(lat, reqs, max(r.done for r in reqs))
    assert s["p99_ms"] >= s["p50_ms"] > 0


def test_light_load_serves_requests_alone():
    # arrivals far apart: each request is a batch of its own and waits only its service time
    reqs = make_requests(50, rate=10.0, seed=4)
    be = SimBackend(slot_bytes=64 << 20, slots=2, per_batch=1e-3, per_byte=0.0)
    lat = serve.Scheduler(be).run(reqs)
    assert all(len(b) == 1 for b in be.launched)
    assert np.allclose(lat, 1e-3, atol=25e-6)


def test_heavy_load_forms_batches_and_underestimates_are_split():
    reqs = make_requests(300, rate=1e6, seed=5)   # all arrive at once
    # the real workspace is 3x the estimate: the scheduler must split batches it admitted
    be = SimBackend(slot_bytes=32 << 20, slots=2, real_factor=3.0)
    sch = serve.Scheduler(be)
    sch.run(reqs)
    flat = [rid for b in be.launched for rid in b]
    assert flat == list(range(len(reqs)))
    assert max(len(b) for b in be.launched) > 1
    for b in be.launched:
        real = sum(reqs[r].M * reqs[r].N * 8 * 3.0 for r in b)
        assert len(b) == 1 or real <= be.slot_bytes


def test_max_batch_limits_batch_size():
    reqs = make_requests(100, rate=1e6, seed=6, mmax=200)
    be = SimBackend(slot_bytes=1 << 30, slots=1)
    serve.Scheduler(be, max_batch=7).run(reqs)
    assert max(len(b) for b in be.launched) == 7


def test_factor_store_keeps_the_most_recent_within_budget():
    st = serve.FactorStore(100)
    for rid in range(6):
        assert st.put(rid, 30, "f%d" % rid)
    # 3 fit: 3, 4, 5 remain
    assert [st.get(r) is not None for r in range(6)] == [False, False, False, True, True, True]
    assert st.used == 90 and st.evicted == 3
    st.get(3)                       # 3 becomes the most recently used
    st.put(6, 30, "f6")             # evicts 4
    assert st.get(4) is None and st.get(3) == "f3" and st.get(6) == "f6"
    assert not st.put(7, 101, "too big")
