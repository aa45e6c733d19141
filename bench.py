#!/usr/bin/env python3
"""Benchmark of the tiled hierarchical Householder QR on one MI355X.

A step is one factorization (hqr_factor: one persistent GPU launch running
every tile kernel of the elimination list) of a synthetic matrix already
resident in HBM.  The headline workload is the tall-skinny FP64 QR of a
131072 x 2048 iid N(0,1) matrix with 256 x 256 tiles and the hierarchical
tree (TS domains of 4 tiles, Greedy low level, domino coupling level,
Fibonacci high level, 8 virtual clusters).  Throughput is reported in GFLOP/s
of the Householder count 2MN^2 - 2N^3/3 (the total weight of any elimination
list, Section II of the paper), next to the FP64 matrix peak of MI355X.

Next to the headline line it measures (keys "lstsq" and "serving"):
* least squares of a 32768 x 2048 matrix with condition number 1e6 (one
  hqr_lstsq: factorization with the right-hand side carried along, then back
  substitution): solves per second;
* continuous-batching serving of 4096 least-squares requests (rows uniform
  in [256, 16384], columns uniform in [32, 512], one right-hand side,
  Poisson arrivals at 0.8 of the measured saturated throughput, 8 GiB
  workspace budget in two slots with a stream each, factors of served
  requests kept on the device within 32 GiB, tile size and tree autotuned
  on the first 64 requests): solves per second and p50/p99 latency.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6  # MI355X dense FP64 (matrix and vector)
PEAK_FP32_TFLOPS = 157.3  # MI355X dense FP32 matrix

# HBM bytes per launch of persistent_kernel<double, 256> from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE), each scaled by what the counter reads for the
# copy-in kernel of known size.  Valid only for the kernel source they were
# measured on (first 16 hex digits of the SHA-256 of csrc/kernels.hip).
TRAFFIC = {
    "tall-hqr": {"kernels_sha256": "577485b801b01c3a", "read": 39.80e9, "write": 21.33e9,
                 "profile": "profiles/persistent_kernel_tall-hqr.md"},
    "square-flat": {"kernels_sha256": "577485b801b01c3a", "read": 176.60e9, "write": 94.48e9,
                    "profile": "profiles/persistent_kernel_square-flat.md"},
}


def kernels_sha():
    import hashlib

    path = os.path.join(ROOT, "paper_1110_1553_amd", "csrc", "kernels.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_for(name):
    t = TRAFFIC.get(name)
    if t is None or t["kernels_sha256"] != kernels_sha():
        return None
    return t["read"] + t["write"]
METRIC = "QR GFLOP/s & % FP64 MFMA peak; lstsq solves/sec + p50/p99 latency"

HQR = dict(nb=256, p=8, a=4, low="greedy", high="fibonacci", coupling="chain", domino=1)
WORKLOADS = {
    "tall-hqr": dict(M=131072, N=2048, seed=2, gen="gaussian", params=HQR,
                     label="tall-skinny FP64 QR 131072x2048 iid N(0,1), nb=256, hierarchical tree "
                           "(TS domains a=4, Greedy low, domino coupling, Fibonacci high, p=8)"),
    "tall-flat": dict(M=131072, N=2048, seed=2, gen="gaussian", params=dict(nb=256, p=1, a=512, low="flat"),
                      label="tall-skinny FP64 QR 131072x2048, nb=256, FlatTree with TS kernels"),
    "tall-binary": dict(M=131072, N=2048, seed=2, gen="gaussian", params=dict(nb=256, p=1, a=1, low="binary"),
                        label="tall-skinny FP64 QR 131072x2048, nb=256, BinaryTree with TT kernels"),
    "square-greedy": dict(M=16384, N=16384, seed=3, gen="graded", params=dict(nb=256, p=1, a=1, low="greedy"),
                          label="square FP64 QR 16384^2, sigma logspaced 1..1e-8, nb=256, Greedy with TT kernels"),
    "tall-hqr-f32": dict(M=131072, N=2048, seed=2, gen="gaussian", params=HQR, dtype="f32",
                         label="tall-skinny FP32 QR 131072x2048 iid N(0,1) (FP32 tile kernels), nb=256, hierarchical "
                               "tree (TS domains a=4, Greedy low, domino coupling, Fibonacci high, p=8)"),
    "square-flat": dict(M=16384, N=16384, seed=3, gen="graded", params=dict(nb=256, p=1, a=64, low="flat"),
                        label="square FP64 QR 16384^2, sigma logspaced 1..1e-8, nb=256, FlatTree with TS kernels"),
}


def qr_flops(M, N):
    return 2.0 * M * N * N - 2.0 * N ** 3 / 3.0


def make_input(w, device):
    from paper_1110_1553_amd import inputs

    if w["gen"] == "gaussian":
        return inputs.gaussian_device(w["M"], w["N"], w["seed"], device)
    return inputs.graded_device(w["M"], w["seed"], 1e-8, device)


def mean_std(xs):
    m = sum(xs) / len(xs)
    v = sum((x - m) ** 2 for x in xs) / (len(xs) - 1) if len(xs) > 1 else 0.0
    return m, v ** 0.5


def host_plan_ms(M, N, params):
    """Host time of the elimination list, task graph and dispatch order (hqr_plan_tasks builds them
    from scratch; hqr_factor caches the result per shape and tree)."""
    from paper_1110_1553_amd import _lib

    nb = params.nb
    t = time.perf_counter()
    _lib.plan_tasks((M + nb - 1) // nb, (N + nb - 1) // nb, params)
    return 1e3 * (time.perf_counter() - t)


def run_workload(name, steps, warmup, device, keep_result=False):
    import torch

    import paper_1110_1553_amd as h

    w = WORKLOADS[name]
    M, N = w["M"], w["N"]
    params = h.make_params(**w["params"])
    plan_ms = host_plan_ms(M, N, params)
    pristine = h.colmajor(make_input(w, device))
    f32 = w.get("dtype") == "f32"
    if f32:
        pristine = h.colmajor(pristine.to(torch.float32))
    work = h.Workspace(M, N, params, device=device, f32=f32)
    stream = torch.cuda.current_stream(device)
    # warm-up: builds and uploads the task plan, loads the code object
    scratch = torch.empty_like(pristine)
    for _ in range(warmup):
        scratch.copy_(pristine)
        h.factor(scratch, params, work=work, stream=stream)
    del scratch
    copies = [pristine.clone() for _ in range(steps)]
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    # events around the persistent launch alone (recorded by the library on the same stream)
    kb = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ke = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for e in kb + ke:
        e.record(stream)  # creates the underlying hipEvent
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    for s in range(steps):
        starts[s].record(stream)
        ex = h.make_exec(ev_begin=kb[s].cuda_event, ev_end=ke[s].cuda_event)
        h.factor(copies[s], params, exec_=ex, work=work, stream=stream, check=False)
        ends[s].record(stream)
    torch.cuda.synchronize(device)
    wall = time.perf_counter() - t0
    status = h.status(work, stream)
    if status != 0:
        raise RuntimeError("device status %d in workload %s" % (status, name))
    ev = [starts[s].elapsed_time(ends[s]) / 1e3 for s in range(steps)]
    kev = [kb[s].elapsed_time(ke[s]) / 1e3 for s in range(steps)]
    fl = qr_flops(M, N)
    launch_s, launch_std = mean_std(ev)
    kernel_s, kernel_std = mean_std(kev)
    peak = PEAK_FP32_TFLOPS if f32 else PEAK_FP64_TFLOPS
    out = {
        "workload": name,
        "label": w["label"],
        "M": M, "N": N,
        "params": w["params"],
        "steps": steps, "warmup": warmup,
        "wall_s": wall,
        "ms_per_step": 1e3 * wall / steps,
        "gflops": fl * steps / wall / 1e9,
        "launch_s": launch_s,
        "launch_ms_std": 1e3 * launch_std,
        "launch_s_min": min(ev),
        "launch_s_max": max(ev),
        "tflops_launch": fl / launch_s / 1e12,
        "kernel_s": kernel_s,
        "kernel_ms_std": 1e3 * kernel_std,
        "tflops_kernel": fl / kernel_s / 1e12,
        "host_plan_ms": plan_ms,
    }
    out["frac_peak"] = out["tflops_launch"] / peak
    out["frac_peak_kernel"] = out["tflops_kernel"] / peak
    result = copies[0] if keep_result else None
    host_sample = None
    if keep_result:
        host_sample = pristine.cpu().numpy()
    del copies, pristine, work
    torch.cuda.empty_cache()
    return out, result, host_sample


def run_lstsq(device, M=32768, N=2048, seed=4, reps=5):
    """FP64 least squares on the tall graded matrix (kappa = 1e6)."""
    import torch

    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import inputs

    # TS domains of 2 tiles: the fastest hierarchical tree for 128 tile rows (a = 4 and 8, p = 1..16, and
    # plain Greedy / Binary trees measured 0.3-4.7 ms slower)
    params = h.make_params(nb=256, p=4, a=2, low="greedy", high="fibonacci", domino=1)
    A0 = h.colmajor(inputs.graded_tall_device(M, N, seed, 1e-6, device))
    g = torch.Generator(device=device)
    g.manual_seed(seed + 1)
    xs = torch.randn((N, 1), generator=g, device=device, dtype=torch.float64)
    b0 = h.colmajor(A0 @ xs + 1e-10 * torch.randn((M, 1), generator=g, device=device, dtype=torch.float64))
    work = h.Workspace(M, N, params, device=device, nrhs=1)
    stream = torch.cuda.current_stream(device)
    A, b = A0.clone(), b0.clone()
    times = []
    for r in range(reps + 1):
        A.copy_(A0)
        b.copy_(b0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        h.lstsq(A, b, params, work=work, stream=stream, check=False)
        e1.record(stream)
        e1.synchronize()
        if r > 0:
            times.append(e0.elapsed_time(e1) / 1e3)
    if h.status(work, stream) != 0:
        raise RuntimeError("device status %d in the least-squares workload" % h.status(work, stream))
    x = b[:N].clone()
    # the refined-residual measure: eta = ||A^T (b - A x)|| / (||A||_2 (||A||_2 ||x|| + ||b||)), with ||A||_2 = 1
    # by construction (largest singular value 1)
    nA = torch.linalg.matrix_norm(A0, 2).item()

    def eta_l1(xv):
        xv = xv.reshape(-1, 1)
        rv = b0 - A0 @ xv
        return (A0.t() @ rv).norm().item() / (nA * (nA * xv.norm().item() + b0.norm().item()))

    t = sum(times) / len(times)
    out = {"workload": "FP64 least squares %dx%d, kappa 1e6, one right-hand side, nb=256 hierarchical tree "
                       "(TS domains a=2, Greedy low, domino coupling, Fibonacci high, p=4)" % (M, N),
           "solves_per_s": 1.0 / t, "ms_per_solve": 1e3 * t,
           "gflops": (qr_flops(M, N) + 4.0 * M * N) / t / 1e9,
           "forward_error_vs_x_true": ((x - xs).norm() / xs.norm()).item(),
           "eta": eta_l1(x)}
    # the same problem with an FP32 factorization refined in FP64 (hqr_lstsq_ir)
    # the refinement keeps TS domains of 4 tiles: at a = 2 the FP32 factors needed one correction more at
    # eta <= 1e-12 (37.1 against 35.0 ms)
    pf = h.make_params(nb=256, p=4, a=4, low="greedy", high="fibonacci", domino=1)
    del A, b, work
    torch.cuda.empty_cache()
    out["ir"] = []
    for tol in (1e-12, 1e-15):
        tir = []
        for r in range(3):
            torch.cuda.synchronize(device)
            t0 = time.perf_counter()
            xi, info = h.lstsq_ir(A0, b0.reshape(-1), pf, max_iter=30, tol=tol, stream=stream)
            torch.cuda.synchronize(device)
            if r > 0:
                tir.append(time.perf_counter() - t0)
        ti = sum(tir) / len(tir)
        out["ir"].append({
            "method": "FP32 tiled QR + FP64 augmented-system refinement, stop at backward error <= %g" % tol,
            "ms_per_solve": 1e3 * ti, "solves_per_s": 1.0 / ti, "iterations": info["iterations"],
            "converged": info["converged"], "eta_augmented": info["eta"], "eta": eta_l1(xi),
            "forward_error_vs_x_true": ((xi - xs.reshape(-1)).norm() / xs.norm()).item(),
            "difference_vs_fp64_solution": ((xi - x.reshape(-1)).norm() / x.norm()).item()})
    del A0, b0
    torch.cuda.empty_cache()
    # BF16 products (FP32 accumulation) under the same refinement, at three condition numbers: it converges
    # only while kappa times the bfloat16 unit roundoff (2^-8) is well below one
    out["bf16"] = []
    pb = h.make_params(nb=256, p=4, a=4, low="greedy", high="fibonacci", domino=1, precision="bf16")
    for kap in (1e2, 1e4, 1e6):
        Ak = h.colmajor(inputs.graded_tall_device(M, N, seed, 1.0 / kap, device))
        bk = (Ak @ xs + 1e-10 * torch.randn((M, 1), generator=g, device=device, dtype=torch.float64)).reshape(-1)
        bk = bk.contiguous()
        torch.cuda.synchronize(device)
        t0 = time.perf_counter()
        xb, info = h.lstsq_ir(Ak, bk, pb, max_iter=30, tol=1e-12, stream=stream)
        torch.cuda.synchronize(device)
        tb = time.perf_counter() - t0
        xf, _ = h.lstsq_ir(Ak, bk, h.make_params(nb=256, p=4, a=4, low="greedy", high="fibonacci", domino=1),
                           max_iter=30, tol=1e-15, stream=stream)
        out["bf16"].append({
            "kappa": kap, "method": "BF16 products, FP32 accumulation, FP64 refinement, stop at <= 1e-12 or 30",
            "ms_per_solve": 1e3 * tb, "iterations": info["iterations"], "converged": info["converged"],
            "eta_augmented": info["eta"], "eta_history": info["history"],
            "forward_error_vs_x_true": ((xb - xs.reshape(-1)).norm() / xs.norm()).item(),
            "difference_vs_refined_fp32_solution": ((xb - xf).norm() / xf.norm()).item()})
        del Ak, bk
    torch.cuda.empty_cache()
    return out


def run_serving(device, count=4096, budget_gib=8, seed=5, load=0.8, tune_sample=64):
    """Continuous-batching serving of a Poisson stream of least-squares requests."""
    import numpy as np
    import torch

    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import inputs, serve, tune

    m, n = inputs.request_shapes(count, seed)
    tuner = tune.Autotuner()
    best, _ = tuner.tune_batch(list(zip(m[:tune_sample], n[:tune_sample])), [1] * tune_sample, device=device)
    params = h.make_params(**best)
    print("bench: serving params %s" % best, file=sys.stderr, flush=True)

    def make_requests(arrivals):
        reqs = []
        for q in range(count):
            A = inputs.gaussian_device(int(m[q]), int(n[q]), 100000 + q, device)
            B = inputs.gaussian_device(int(m[q]), 1, 200000 + q, device)
            reqs.append(serve.Request(q, A, B, float(arrivals[q])))
        torch.cuda.synchronize(device)
        return reqs

    be = serve.GpuBackend(params, budget_gib << 30, max_inflight=2, device=device, factor_budget=32 << 30)
    # saturated throughput: every request waiting at the start
    reqs = make_requests(np.zeros(count))
    sch = serve.Scheduler(be)
    sch.run(reqs)
    span = max(r.done for r in reqs)
    sat = count / span
    del reqs, sch
    be.store = serve.FactorStore(32 << 30)  # the second run starts with no resident factors
    # Poisson arrivals at `load` times that rate
    arrivals = np.cumsum(inputs.arrival_gaps(count, load * sat, seed + 1))
    reqs = make_requests(arrivals)
    sch = serve.Scheduler(be)
    lat = sch.run(reqs)
    bad = sum(1 for r in reqs if r.status != 0)
    s = serve.summarize(lat, reqs, max(r.done for r in reqs))
    # the plain FP64 path on the same requests: one hqr_lstsq per request, back to back on one stream
    nseq = min(count, 256)
    seq_reqs = [(inputs.gaussian_device(int(m[q]), int(n[q]), 100000 + q, device),
                 inputs.gaussian_device(int(m[q]), 1, 200000 + q, device)) for q in range(nseq)]
    stream = torch.cuda.current_stream(device)
    for A, B in seq_reqs[:4]:
        h.lstsq(A.clone(), B.clone(), params, stream=stream, check=False)
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    for A, B in seq_reqs:
        h.lstsq(A, B, params, stream=stream, check=False)
    torch.cuda.synchronize(device)
    seq_rate = nseq / (time.perf_counter() - t0)
    del seq_reqs
    flops = float(sum(qr_flops(int(a), int(b)) + 4.0 * a * b for a, b in zip(m, n)))
    out = {"workload": "%d least-squares requests, rows U[256,16384], cols U[32,512], 1 rhs, Poisson arrivals" % count,
           "params": best, "budget_GiB": budget_gib, "saturated_solves_per_s": sat,
           "saturated_gflops": flops / span / 1e9, "arrival_rate_per_s": load * sat,
           "solves_per_s": s["solves_per_s"], "p50_ms": s["p50_ms"], "p99_ms": s["p99_ms"],
           "plain_fp64_sequential_solves_per_s": seq_rate,
           "plain_fp64_sequential_sample": "the first %d requests, one hqr_lstsq each (same tile size and tree)" % nseq,
           "batches": len(sch.batches), "mean_batch": count / len(sch.batches), "failed": bad,
           "batches_launched_while_another_ran": sum(1 for i in range(1, len(sch.batches))
                                                     if sch.batches[i]["t_launch"] < sch.batches[i - 1]["t_done"]),
           "resident_factorizations": len(be.store.items), "resident_GiB": be.store.used / 2 ** 30,
           "evicted": be.store.evicted}
    del reqs, sch, be
    torch.cuda.empty_cache()
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sample):
    """The oracle (unblocked Householder QR) on the whole benchmark matrix with the host's threads (up
    to 16), and on its leading 16384 x 512 block with one thread.  Returns the record and the
    oracle's factored array (its upper triangle is R)."""
    import numpy as np

    from oracle import qr as oq

    threads = max(1, min(16, os.cpu_count() or 1))
    A = np.asfortranarray(sample)
    m, n = A.shape
    t = time.perf_counter()
    F, _ = oq.factor(A, nthreads=threads)
    dt = time.perf_counter() - t
    ms, ns = min(m, 16384), min(n, 512)
    t = time.perf_counter()
    oq.factor(np.asfortranarray(A[:ms, :ns]), nthreads=1)
    dt1 = time.perf_counter() - t
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    rec = {"value": qr_flops(m, n) / dt / 1e9, "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
           "sample": "oracle QR of the whole %dx%d benchmark matrix, copied to the host (%.1f s on %d threads)"
                     % (m, n, dt, threads),
           "cpu_model": cpu_model(), "nproc": os.cpu_count(), "cpus_available": avail,
           "single_thread": {"value": qr_flops(ms, ns) / dt1 / 1e9, "unit": "GFLOP/s",
                             "sample": "oracle QR of the leading %dx%d block, 1 thread (%.1f s)" % (ms, ns, dt1)}}
    return rec, F


def r_parity(R_gpu, F_ref):
    """Relative Frobenius error of the sign-normalised R against the oracle's."""
    import numpy as np

    n = R_gpu.shape[1]
    Rg, Rr = np.triu(R_gpu[:n, :n]), np.triu(F_ref[:n, :n])
    dg = np.where(np.diagonal(Rg) < 0, -1.0, 1.0)
    dr = np.where(np.diagonal(Rr) < 0, -1.0, 1.0)
    return float(np.linalg.norm(Rg * dg[:, None] - Rr * dr[:, None]) / np.linalg.norm(Rr))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tall-hqr", choices=sorted(WORKLOADS))
    ap.add_argument("--secondary", default="square-flat,square-greedy,tall-flat,tall-binary,tall-hqr-f32",
                    help="comma-separated workloads also timed (--sec-steps steps each after 2 warm-ups); empty "
                         "for none")
    ap.add_argument("--sec-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", type=int, default=4096, help="requests in the serving trace (0: skip serving)")
    ap.add_argument("--no-lstsq", action="store_true", help="skip the least-squares measurement")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    device = torch.device("cuda:0")
    torch.cuda.set_device(device)
    primary, result, host_sample = run_workload(args.workload, args.steps, args.warmup, device, keep_result=True)
    R_gpu = result[:primary["N"], :primary["N"]].cpu().numpy() if result is not None else None
    del result
    print("bench: %s %.3f ms/step (kernel %.3f ms)" % (args.workload, primary["ms_per_step"],
                                                      1e3 * primary["kernel_s"]), file=sys.stderr, flush=True)
    secondary = []
    for name in [s for s in args.secondary.split(",") if s]:
        if name == args.workload:
            continue
        res, _, _ = run_workload(name, args.sec_steps, 2, device)
        print("bench: %s %.3f ms/step (kernel %.3f +- %.3f ms)" % (name, res["ms_per_step"], 1e3 * res["kernel_s"],
                                                                  res["kernel_ms_std"]), file=sys.stderr, flush=True)
        secondary.append({k: res[k] for k in ("workload", "label", "steps", "warmup", "ms_per_step", "gflops",
                                              "tflops_launch", "frac_peak", "launch_ms_std", "kernel_s",
                                              "kernel_ms_std", "tflops_kernel", "frac_peak_kernel",
                                              "host_plan_ms")})
    lstsq = None
    if not args.no_lstsq:
        lstsq = run_lstsq(device)
        print("bench: lstsq %.3f ms/solve" % lstsq["ms_per_solve"], file=sys.stderr, flush=True)
    serving = None
    if args.serve > 0:
        serving = run_serving(device, count=args.serve)
        print("bench: serving %.0f solves/s p50 %.2f ms p99 %.2f ms" % (
            serving["solves_per_s"], serving["p50_ms"], serving["p99_ms"]), file=sys.stderr, flush=True)
    cpu = None
    parity = None
    if not args.no_cpu_baseline and host_sample is not None:
        cpu, F_ref = cpu_baseline(host_sample)
        print("bench: cpu baseline %s" % cpu["sample"], file=sys.stderr, flush=True)
        if R_gpu is not None and primary["params"].get("precision", "fp64") == "fp64" and \
                WORKLOADS[args.workload].get("dtype") != "f32":
            err = r_parity(R_gpu, F_ref)
            parity = {"rel_err_R": err, "tol": 1e-12, "ok": bool(err <= 1e-12),
                      "reference": "sign-normalised R of the oracle's QR of the same %dx%d matrix (the "
                                   "cpu_baseline run), against the R of the first timed step"
                                   % (primary["M"], primary["N"])}
            print("bench: parity of R against the oracle %.3e" % err, file=sys.stderr, flush=True)
        del F_ref
    w = WORKLOADS[args.workload]
    f32 = w.get("dtype") == "f32"
    peak = PEAK_FP32_TFLOPS if f32 else PEAK_FP64_TFLOPS
    line = {
        "metric": METRIC,
        "value": round(primary["gflops"], 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(primary["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if f32 else "f64",
        "data": "synthetic",
        "config": {"workload": w["label"], "M": w["M"], "N": w["N"], "tree": w["params"],
                   "frac_peak": round(primary["frac_peak"], 4)},
        "roofline": {"bound": "mfma", "achieved": round(primary["tflops_kernel"], 3), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(primary["frac_peak_kernel"], 4),
                     "traffic": traffic_for(args.workload), "traffic_unit": "bytes per launch (HBM read + write)",
                     "kernel": "persistent_kernel<%s, 256> (all tile kernels of one factorization)" % (
                         "float" if f32 else "double"),
                     "flops_per_launch": qr_flops(primary["M"], primary["N"]),
                     "kernel_ms": round(1e3 * primary["kernel_s"], 3),
                     "kernel_ms_std": round(primary["kernel_ms_std"], 3),
                     "timing": "HIP events recorded by the library right before and after the persistent launch "
                               "(hqr_exec.ev_begin/ev_end), mean over the timed steps",
                     "whole_call_ms": round(1e3 * primary["launch_s"], 3),
                     "whole_call_frac": round(primary["frac_peak"], 4)},
        "host_plan_ms": round(primary["host_plan_ms"], 2),
        "parity": parity,
        "cpu_baseline": cpu,
        "secondary": secondary,
        "lstsq": lstsq,
        "serving": serving,
    }
    print(json.dumps(line), flush=True)
    if parity is not None and not parity["ok"]:
        print("bench.py: R differs from the oracle's by %.3e (> 1e-12)" % parity["rel_err_R"], file=sys.stderr)
        sys.exit(1)


if __name__ == "__main__":
    main()
