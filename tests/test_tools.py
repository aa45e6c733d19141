"""CPU tests of the measurement helpers: the per-task timeline summary and
the benchmark's parity measure (no GPU: synthetic stamps and matrices)."""
import numpy as np

from paper_1110_1553_amd import timeline


def test_task_work_counts_kernel_weights():
    nb = 256
    b3 = nb ** 3 / 3.0
    # Section II weights in units of nb^3/3; an update task over half the
    # columns carries half its tile's weight
    assert timeline.task_work(0, nb, nb)[0] == 4 * b3
    assert timeline.task_work(2, nb, nb)[0] == 6 * b3
    assert timeline.task_work(4, nb, nb)[0] == 2 * b3
    assert timeline.task_work(3, nb, nb // 2)[0] == 6 * b3
    assert timeline.task_work(1, nb, nb // 2)[0] == 3 * b3
    assert timeline.task_work(5, nb, nb // 2)[0] == 3 * b3
    # bytes: TSQRT reads and writes a triangle and a square plus its T
    tile = nb * nb * 8
    assert timeline.task_work(2, nb, nb)[1] == 2 * (tile / 2 + tile) + nb * 16 * 8


def _plan(ops, chunks, pads):
    dt = np.dtype([("op", "u1"), ("chunk", "u1"), ("pad", "<u2")])
    t = np.zeros(len(ops), dtype=dt)
    t["op"], t["chunk"], t["pad"] = ops, chunks, pads
    return t


def test_summarize_shares_and_rates():
    # two workgroups over 10 us: wg 0 runs a GEQRT for 4 us after 1 us of
    # waiting, wg 1 a TSMQR chunk (two sub-chunks) for 8 us after 2 us
    tl = np.array([[0, 100, 500, 0], [0, 200, 1000, 1]], dtype=np.uint64)  # 100 MHz stamps
    tasks = _plan([0, 3], [4, 0], [0, 2 << 8])
    s = timeline.summarize(tl, tasks, 256)
    assert s["workers"] == 2
    assert abs(s["span_ms"] - 0.01) < 1e-12
    assert abs(s["run_share"] - (4 + 8) / 20.0) < 1e-12
    assert abs(s["wait_share"] - (1 + 2) / 20.0) < 1e-12
    assert abs(s["run_share"] + s["wait_share"] + s["idle_share"] - 1.0) < 1e-12
    g = s["kernels"]["GEQRT"]
    assert g["count"] == 1 and abs(g["run_us_mean"] - 4.0) < 1e-9
    assert abs(g["tflops_per_cu"] - 4 * 256 ** 3 / 3.0 / 4e-6 / 1e12) < 1e-9
    t = s["kernels"]["TSMQR"]
    assert abs(t["flops_per_task"] - 6 * 256 ** 3 / 3.0) < 1e-3


def test_bench_parity_is_sign_invariant():
    import bench

    rng = np.random.default_rng(3)
    R = np.triu(rng.standard_normal((40, 40)))
    D = np.diag(np.where(rng.random(40) < 0.5, -1.0, 1.0))
    # the same R up to row signs, below-diagonal garbage ignored
    Rg = D @ R + np.tril(rng.standard_normal((40, 40)), -1)
    assert bench.r_parity(Rg, R) < 1e-15
    Rb = R.copy()
    Rb[3, 7] += 1e-6 * np.linalg.norm(R)
    assert bench.r_parity(Rb, R) > 5e-7
