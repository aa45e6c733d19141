"""Per-task timeline of one factorization, summarised per tile kernel.

Runs one factorization with the library's per-task clock stamps on
(HQR_TIMELINE=1: when a workgroup took the task, when its inputs were ready,
when it finished; 100 MHz real-time clock) and reports, per kernel (GEQRT,
UNMQR, TSQRT, TSMQR, TTQRT, TTMQR): the task count, the mean running time,
the mean wait for inputs, the algorithmic flops and bytes of a task and the
rates they give (TFLOP/s on one compute unit; GB/s of HBM traffic for the
panel kernels, whose columns are sequential), plus the share of the
workgroups' time spent running, waiting and between tasks.

Algorithmic work per task (nb = b):
* flops: the kernel weights of Section II of the paper in units of b^3/3
  (GEQRT 4, UNMQR 6, TSQRT 6, TSMQR 12, TTQRT 2, TTMQR 6); an update task
  covering w of the b columns of its tile carries w / b of its tile's weight.
* bytes: every tile element the kernel must read and write once (a triangle
  counts half a tile) and its T factors (b x 16 per tile, written by the
  panel kernels, read by the update kernels).

Usage::

    python -m paper_1110_1553_amd.timeline --M 131072 --N 2048 --nb 256 \\
        --p 8 --a 4 --low greedy --high fibonacci --domino 1 [--graded] [--json out.json] \\
        [--raw out.npz]

``--raw`` also saves the per-task stamps (``tl``: picked, ready, done,
workgroup | XCD << 16) next to the plan's fields, in dispatch order.
"""
import argparse
import json
import os
import sys

OPS = ("GEQRT", "UNMQR", "TSQRT", "TSMQR", "TTQRT", "TTMQR")
WEIGHT = (4, 6, 6, 12, 2, 6)
CLOCK_HZ = 100e6


def task_work(op, nb, width, esize=8):
    """(flops, bytes) of one task: op index, tile size, columns covered."""
    tile = nb * nb * esize
    tbytes = nb * 16 * esize
    frac = width / nb
    flops = WEIGHT[op] * nb ** 3 / 3.0 * frac
    if op == 0:    # GEQRT: the tile in and out, T out
        b = 2 * tile + tbytes
    elif op == 2:  # TSQRT: killer triangle and victim square in and out, T out
        b = 2 * (tile / 2 + tile) + tbytes
    elif op == 4:  # TTQRT: two triangles in and out, T out
        b = 2 * tile + tbytes
    elif op == 1:  # UNMQR: V (unit lower triangle) and T in, the chunk in and out
        b = tile / 2 + tbytes + 2 * tile * frac
    elif op == 3:  # TSMQR: V (square) and T in, two chunks in and out
        b = tile + tbytes + 4 * tile * frac
    else:          # TTMQR: V (triangle) and T in, two chunks in and out
        b = tile / 2 + tbytes + 4 * tile * frac
    return flops, b


def summarize(tl, tasks, nb, esize=8):
    """tl: (ntasks, 4) uint64 timeline in dispatch order; tasks: the plan
    (structured array with fields op, chunk, pad)."""
    import numpy as np

    picked = tl[:, 0].astype(np.float64)
    ready = tl[:, 1].astype(np.float64)
    done = tl[:, 2].astype(np.float64)
    wg = (tl[:, 3] & 0xFFFF).astype(np.int64)
    t0 = picked.min()
    span = (done.max() - t0) / CLOCK_HZ
    workers = int(wg.max()) + 1
    run = (done - ready) / CLOCK_HZ
    wait = (ready - picked) / CLOCK_HZ
    out = {"tasks": int(len(tl)), "workers": workers, "span_ms": 1e3 * span,
           "run_share": float(run.sum() / (workers * span)), "wait_share": float(wait.sum() / (workers * span))}
    out["idle_share"] = 1.0 - out["run_share"] - out["wait_share"]
    per = {}
    for op in range(6):
        sel = tasks["op"] == op
        n = int(sel.sum())
        if n == 0:
            continue
        if op in (0, 2, 4):
            widths = np.minimum(tasks["chunk"][sel].astype(np.int64) * 64, nb)  # active columns of the panel
        else:
            widths = (tasks["pad"][sel].astype(np.int64) >> 8) * 64              # sub-chunks covered
        fl = np.array([task_work(op, nb, int(w), esize)[0] for w in widths])
        by = np.array([task_work(op, nb, int(w), esize)[1] for w in widths])
        r = run[sel]
        per[OPS[op]] = {
            "count": n,
            "run_us_mean": 1e6 * float(r.mean()),
            "run_us_median": 1e6 * float(np.median(r)),
            "wait_us_mean": 1e6 * float(wait[sel].mean()),
            "busy_share": float(r.sum() / (workers * span)),
            "tflops_per_cu": float(fl.sum() / r.sum() / 1e12),
            "gbytes_per_s_per_task": float(by.sum() / r.sum() / 1e9),
            "flops_per_task": float(fl.mean()),
            "bytes_per_task": float(by.mean()),
        }
    out["kernels"] = per
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--M", type=int, required=True)
    ap.add_argument("--N", type=int, required=True)
    ap.add_argument("--nb", type=int, default=256)
    ap.add_argument("--p", type=int, default=1)
    ap.add_argument("--a", type=int, default=1)
    ap.add_argument("--low", default="greedy")
    ap.add_argument("--high", default="flat")
    ap.add_argument("--coupling", default="chain")
    ap.add_argument("--domino", type=int, default=0)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--graded", action="store_true", help="U diag(sigma) V^T (square only) instead of N(0,1)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--json", default=None)
    ap.add_argument("--raw", default=None, help="save the per-task stamps and the plan (numpy .npz)")
    args = ap.parse_args()
    os.environ["HQR_TIMELINE"] = "1"  # read by the library at its first launch
    import torch

    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import _lib, inputs

    dev = torch.device("cuda:0")
    params = h.make_params(nb=args.nb, p=args.p, a=args.a, low=args.low, high=args.high, coupling=args.coupling,
                           domino=args.domino)
    if args.graded:
        A0 = h.colmajor(inputs.graded_device(args.M, args.seed, 1e-8, dev))
    else:
        A0 = h.colmajor(inputs.gaussian_device(args.M, args.N, args.seed, dev))
    work = h.Workspace(args.M, args.N, params, device=dev)
    stream = torch.cuda.current_stream(dev)
    A = A0.clone()
    for _ in range(args.warmup + 1):
        A.copy_(A0)
        h.factor(A, params, work=work, stream=stream)
    tl = _lib.timeline(stream.cuda_stream)
    tasks = _lib.plan_tasks(-(-args.M // args.nb), -(-args.N // args.nb), params)
    if len(tasks) != len(tl):
        raise RuntimeError("timeline and plan disagree (%d vs %d tasks)" % (len(tl), len(tasks)))
    s = summarize(tl, tasks, args.nb)
    s["workload"] = vars(args)
    print("span %.3f ms, %d workgroups: running %.1f%%, waiting %.1f%%, between tasks %.1f%%" % (
        s["span_ms"], s["workers"], 100 * s["run_share"], 100 * s["wait_share"], 100 * s["idle_share"]))
    print("%-6s %7s %10s %10s %9s %8s %10s %10s" % ("kernel", "count", "run us", "median us", "wait us", "busy %",
                                                    "TF/s/CU", "GB/s"))
    for k, v in s["kernels"].items():
        print("%-6s %7d %10.1f %10.1f %9.1f %8.1f %10.3f %10.1f" % (
            k, v["count"], v["run_us_mean"], v["run_us_median"], v["wait_us_mean"], 100 * v["busy_share"],
            v["tflops_per_cu"], v["gbytes_per_s_per_task"]))
    if args.json:
        with open(args.json, "w") as f:
            json.dump(s, f, indent=1)
    if args.raw:
        import numpy as np

        np.savez_compressed(args.raw, tl=tl, **{f: tasks[f] for f in tasks.dtype.names})
    sys.stdout.flush()


if __name__ == "__main__":
    main()
