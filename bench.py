#!/usr/bin/env python3
"""Node relaxations solved per second at 1e-6 relative gap on one MI355X.

Workload (one step): 256 least-squares node relaxations of the k-sparse, box-constrained ridge
GLM that share one design X (n = 20000, p = 10000, Toeplitz-correlated Gaussian rows with
rho = 0.5, standardised columns, stored in BF16), k = 10, M = 2, lambda2 = 1e-3, each node with
random fixed-zero / fixed-in sets of sizes uniform in [0, 20] / [0, 10]. Every node is solved to
an FP64-certified relative gap <= 1e-6.

The step runs the batched mixed-precision engine (BF16 MFMA products with FP32 accumulation
around FP64 base points) when the library has it, else the plain FP64 per-node path; the plain
FP64 per-node path is also timed on a subset of the same nodes as the comparator.

Prints one JSON line (see the printed keys). Inputs are resident in HBM before the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2502_09502_amd import _lib, synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
WORKLOAD = ("256 least-squares node relaxations sharing X: n=20000, p=10000, BF16 X "
            "(Toeplitz rho=0.5, standardised), k=10, M=2, lambda2=1e-3, |Z0|~U[0,20], "
            "|Z1|~U[0,10], FP64-certified rel. gap 1e-6")
KERNEL_NAMES = {0: "k_xt (plain X^T pass)", 1: "k_xb (plain X pass)",
                2: "k_gemm_bf16<1, RT> (batched X^T pass)",
                3: "k_gemm_bf16<0, RT> (batched X pass)",
                4: "k_gemm_f64 (FP64 certification X pass)"}


def algorithmic_bytes(which: int, n: int, p: int, sx: int, nodes: int) -> float:
    """Bytes a launch must move at minimum: X once, plus the vectors it reads and writes."""
    if which == 0:  # h = X^T grad f(u_gamma): X, u^t, u^{t-1}, y, h
        return n * p * sx + 8.0 * (3 * n + p)
    if which == 1:  # u = X beta: X, beta, u, y
        return n * p * sx + 8.0 * (p + 2 * n)
    if which == 2:  # batched X^T pass: X, BF16 operand (nodes x n), FP32 output (nodes x p)
        return n * p * sx + nodes * (2.0 * n + 4.0 * p)
    if which == 3:  # batched X pass: X, BF16 operand (nodes x p), FP32 output (nodes x n)
        return n * p * sx + nodes * (2.0 * p + 4.0 * n)
    return n * p * sx + nodes * 8.0 * (n + p)


MFMA_BF16_PEAK_TFLOPS = 2500.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_gemm_bf16_c4_traffic.md")
TRAFFIC_SOURCES = ("paper_2502_09502_amd/csrc/gemm_bf16.h",)  # the product kernels and their main loop


def tiling_desc(code):
    """A product's tiling from the engine's code (split-K, plus 100 for the 128-row tile and 200
    for the 64-row tile)."""
    code = int(code)
    if code <= 0:
        return None
    return f"{256 >> min(code // 100, 2)} rows x 256 nodes per workgroup, split-K {code % 100}"


def measured_traffic(key: str, tiling=None):
    """HBM bytes per launch from the committed counter summary, or None when the kernel sources
    changed since the counters were taken, when the counters were taken on another tiling of the
    product than the one in use (tiling: its code), or when there is no summary."""
    import hashlib
    try:
        h = hashlib.sha256()
        for f in TRAFFIC_SOURCES:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        vals = {}
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if ":" in line and not line.startswith(("|", "#", "`")):
                    k, v = line.split(":", 1)
                    vals[k.strip()] = v.strip()
        if vals.get("source_sha256_16") != h.hexdigest()[:16]:
            return None
        tkey = key.replace("traffic_bytes_", "tiling_")
        if tiling is not None and tkey in vals and int(vals[tkey]) != int(tiling):
            return None
        return float(vals[key])
    except (OSError, KeyError, ValueError):
        return None


def roofline(ctx, n, p, sx, nodes, which):
    """Roofline of one kernel from its live HIP-event timing over the timed region."""
    ms, cnt = ctx.kernel_stats(which)
    if cnt == 0:
        return None
    avg_s = ms / cnt / 1e3
    nbytes = algorithmic_bytes(which, n, p, sx, nodes)
    achieved = nbytes / avg_s / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
           "kernel": KERNEL_NAMES[which], "avg_launch_us": round(avg_s * 1e6, 2),
           "launches": cnt, "bytes_per_launch": nbytes}
    if which in (2, 3):
        code_x, code_xt = ctx.kernel_stats(14)  # the tilings the engine's autotuner chose
        code = int(code_xt if which == 2 else code_x)
        out["tiling"] = tiling_desc(code)
        out["traffic"] = measured_traffic("traffic_bytes_xt_pass" if which == 2 else
                                          "traffic_bytes_x_pass", tiling=code)
        tflops = 2.0 * n * p * nodes / avg_s / 1e12
        out["mfma_context"] = {"achieved_tflops": round(tflops, 1),
                               "peak_tflops": MFMA_BF16_PEAK_TFLOPS,
                               "frac": round(tflops / MFMA_BF16_PEAK_TFLOPS, 4)}
    return out


_CPU_JOB = {}  # set before the workers fork; never pickled


def _cpu_worker(i):
    """Oracle solve of node i in a worker process with one BLAS thread (forked: the design is
    shared with the parent, copy-on-write)."""
    d, sets, L = _CPU_JOB["d"], _CPU_JOB["sets"], _CPU_JOB["L"]
    z0, z1 = sets[i]
    import oracle
    from threadpoolctl import threadpool_limits

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        r = oracle.solve_node(d.X, d.y, "ls", d.lam2, d.M, d.k, z0, z1, tol=1e-6, L=L)
        return r.iters, r.status, time.perf_counter() - t0


def host_cores() -> int:
    """Cores this process may run on, at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(d, sets, nodes_per_core=2):
    """The oracle on the host cores, node-parallel: one process per core, each with one BLAS
    thread, solving whole nodes (Alg. 3 to the FP64-certified 1e-6 gap) of the workload's first
    nodes_per_core x cores node sets; solves/s = nodes / wall time. The oracle's own Lipschitz
    constant (an eigen-solver on X^T X) is computed first, outside the timed region. Runs before
    the GPU is touched, so the forked workers inherit no device state."""
    import multiprocessing as mp

    import oracle

    cores = host_cores()
    t_l = time.perf_counter()
    L = oracle.lipschitz(d.X, "ls")
    t_l = time.perf_counter() - t_l
    work = list(range(min(len(sets), nodes_per_core * cores)))
    _CPU_JOB.update(d=d, sets=sets, L=L)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(processes=cores) as pool:
        out = pool.map(_cpu_worker, work, chunksize=1)
    t = time.perf_counter() - t0
    _CPU_JOB.clear()
    iters = sum(o[0] for o in out)
    conv = sum(1 for o in out if o[1] == oracle.CONVERGED)
    print(f"# cpu baseline: {len(work)} nodes on {cores} processes in {t:.1f} s", file=sys.stderr,
          flush=True)
    return {"value": len(work) / t, "unit": "solves/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"oracle (FP64 NumPy) solves of the workload's first {len(work)} nodes "
                       f"to the certified 1e-6 gap ({conv} converged), one process per core "
                       f"with one BLAS thread each, {iters} iterations in {t:.1f} s; the "
                       f"oracle's L = {L:.6g} from its own eigen-solver ({t_l:.1f} s, untimed)")}


SERVE_WORKLOAD = ("serving: Poisson stream (mean 2000/s) of node relaxations over 3 resident "
                  "datasets p in {1000, 5000, 20000}, n = 2p, FP32 X (BF16 copies on the device), "
                  "least squares and logistic 50/50, |Z0|~U[0,30], |Z1|~U[0,10], k=10, M=2, "
                  "lambda2=1e-3, FP64-certified rel. gap 1e-6")


def serve(args):
    """Continuous-batching server under a Poisson request stream; latency is completion time
    minus arrival time (including the wait for the polling loop to pick the request up)."""
    sizes = [int(v) for v in args.serve_sizes.split(",")]
    ctx = _lib.Context(0)
    t_setup = time.perf_counter()
    probs = []
    for p in sizes:
        X32, y_ls, y_log = synth.serving_dataset(p)
        pair = []
        for loss, y in (("ls", y_ls), ("logistic", y_log)):
            pair.append((p, loss, _lib.Problem(ctx, X32, y, loss=loss, lam2=1e-3, M=2.0, k=10)))
        if not args.no_share:
            # the logistic relaxation shares the least-squares problem's engine: one pass over
            # the design per iteration advances the nodes of both
            pair[0][2].share_design(pair[1][2])
        probs += pair
        del X32
    print(f"# serving setup {time.perf_counter() - t_setup:.1f}s", file=sys.stderr, flush=True)
    N = args.requests
    rng = np.random.default_rng([3, 5])
    which = rng.integers(0, len(probs), size=N)
    sets = {p: synth.node_sets(p, 10, N, 30, config_id=5) for p in sizes}
    specs = []
    for i in range(N):
        p, loss, prob = probs[int(which[i])]
        z0, z1 = sets[p][i]
        specs.append((prob, prob.node(Z0=z0, Z1=z1, tol=1e-6, max_iter=5000, precision="mixed")))
    arrivals = synth.poisson_arrivals(N, args.rate)
    # warm the engines (setup of the BF16 copies and of the graphs is not request latency)
    srv = _lib.Server(ctx, 0, 256)
    for prob_i in range(len(probs)):
        prob = probs[prob_i][2]
        srv.submit(prob, prob.node(tol=1e-6, precision="mixed"))
    got = 0
    while got < len(probs):
        got += len(srv.poll(256))
    arrival_of = {}
    p_of = {}
    lat = []
    lat_by_p = {p: [] for p in sizes}
    statuses = {}
    i = 0
    t0 = time.perf_counter()
    t_last = t0
    while len(lat) < N:
        now = time.perf_counter() - t0
        while i < N and arrivals[i] <= now:
            prob, spec = specs[i]
            t = srv.submit(prob, spec)
            arrival_of[t] = arrivals[i]
            p_of[t] = prob.p
            i += 1
        for t, r, _ in srv.poll(256):
            done_t = time.perf_counter() - t0
            lat.append(done_t - arrival_of.pop(t))
            lat_by_p[p_of.pop(t)].append(lat[-1])
            statuses[r.status] = statuses.get(r.status, 0) + 1
            t_last = time.perf_counter()
        if i < N and not srv.stats()["running"] and not srv.stats()["queued"]:
            time.sleep(max(0.0, arrivals[i] - (time.perf_counter() - t0)))
    elapsed = t_last - t0
    srv.close()
    lat_ms = 1e3 * np.asarray(lat)
    out = {
        "metric": "node relaxations solved/sec at 1e-6 gap, batched vs plain; p50/p99 latency",
        "value": round(N / elapsed, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": round(1e3 * elapsed, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-mfma/fp32-acc + fp64 bound",
        "data": "synthetic",
        "config": {"workload": SERVE_WORKLOAD, "requests": N, "rate_per_s": args.rate,
                   "sizes": sizes, "engine": "server",
                   "engines": "one per problem" if args.no_share else "one per dataset"},
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 3),
                       "p99": round(float(np.percentile(lat_ms, 99)), 3),
                       "max": round(float(lat_ms.max()), 3)},
        "latency_ms_by_dataset": {
            str(p): {"requests": len(v),
                     "p50": round(float(np.percentile(1e3 * np.asarray(v), 50)), 3),
                     "p99": round(float(np.percentile(1e3 * np.asarray(v), 99)), 3)}
            for p, v in lat_by_p.items() if v},
        "statuses": statuses,
        "offered_rate_per_s": args.rate,
    }
    print(json.dumps(out))


PROX_WORKLOAD = ("standalone prox of g (Fig. 1 setting): gamma ~ N(0, I_p), k=10, M=1, rho=1, "
                 "p = 100 * 2^i, a batch of vectors per size")


def prox_workload(args):
    """The prox kernel alone (Alg. 1 through the Moreau identity): per-vector latency (one
    vector per launch) and batched throughput, kernel time from HIP events; the oracle's prox on
    five seeds per size as the CPU baseline."""
    ctx = _lib.Context(0)
    sizes = [100 * 2 ** i for i in range(args.prox_max_i + 1)]
    batch = args.prox_batch
    rows = []
    cpu_s = 0.0
    cpu_n = 0
    for p in sizes:
        W = np.stack([np.random.default_rng([4, p, s]).standard_normal(p) for s in range(batch)])
        _lib.prox_node_batch(ctx, W[:1], 1.0, 1.0, 10)  # warm-up
        ctx.set_profiling(True)
        ctx.kernel_stats(8, reset=True)
        for _ in range(5):
            _lib.prox_node_batch(ctx, W[:1], 1.0, 1.0, 10)
        ms1, n1 = ctx.kernel_stats(8, reset=True)
        for _ in range(3):
            _lib.prox_node_batch(ctx, W, 1.0, 1.0, 10)
        msb, nb = ctx.kernel_stats(8, reset=True)
        ctx.set_profiling(False)
        row = {"p": p, "gpu_us_one_vector": round(1e3 * ms1 / n1, 2),
               "gpu_us_per_vector_batched": round(1e3 * msb / nb / batch, 3),
               "gpu_vectors_per_s_batched": round(nb * batch / (msb / 1e3), 1)}
        if not args.no_cpu:
            import oracle
            t0 = time.perf_counter()
            for s in range(5):
                oracle.prox_g(W[s], 1.0, 1.0, 10)
            t = time.perf_counter() - t0
            cpu_s += t
            cpu_n += 5
            row["oracle_ms_per_vector"] = round(1e3 * t / 5, 3)
        rows.append(row)
    last = rows[-1]
    out = {
        "metric": "prox evaluations per second (standalone prox workload)",
        "value": last["gpu_vectors_per_s_batched"],
        "unit": "prox/s",
        "n_gpus": 1,
        "steps": 3,
        "warmup": 1,
        "ms_per_step": round(last["gpu_us_per_vector_batched"] * batch / 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": PROX_WORKLOAD, "batch": batch, "p_max": sizes[-1]},
        "sizes": rows,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = {"value": round(cpu_n / cpu_s, 3), "unit": "prox/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"oracle prox (stack PAVA) on 5 seeds per size, all sizes "
                                         f"pooled: {cpu_n} vectors in {cpu_s:.2f} s"}
    print(json.dumps(out))


SINGLE_WORKLOADS = {
    "c1": ("least-squares root relaxation, plain FP64: n=200, p=50, k=5, M=2, lambda2=1e-3, "
           "Toeplitz rho=0.5 standardised X, FP64-certified rel. gap 1e-6",
           [("c1", "f64")]),
    "c2": ("least-squares root relaxation, single iterate (HBM-bound GEMV path): n=10000, "
           "p=5000, k=10, M=2, lambda2=1e-3, Toeplitz rho=0.5 standardised X in FP64 and in FP32, "
           "FP64-certified rel. gap 1e-6",
           [("c2_f64", "f64"), ("c2_f32", "f64")]),
    "c3": ("logistic root relaxation: n=20000, p=10000, k=10, M=2, lambda2=1e-3, Toeplitz rho=0.5 "
           "standardised X in FP32, labels Bernoulli(sigmoid(X beta*)); plain FP64 iterates vs "
           "BF16-X MFMA corrections with FP32 accumulation and FP64 bounds, FP64-certified rel. "
           "gap 1e-6",
           [("c3", "f64"), ("c3", "mixed")]),
}


def _oracle_sample(d, budget_s=20.0):
    """The oracle's root solve on the host cores (NumPy BLAS on all of them), run to convergence
    or stopped at an iteration cap chosen so that it takes about budget_s seconds: returns
    (seconds, iterations, converged, gap, seconds per iteration)."""
    import oracle

    L = oracle.lipschitz(d.X, d.loss)
    t0 = time.perf_counter()
    oracle.solve_node(d.X, d.y, d.loss, d.lam2, d.M, d.k, tol=1e-6, max_iter=2, L=L)
    per_iter = (time.perf_counter() - t0) / 2
    cap = max(3, int(budget_s / max(per_iter, 1e-6)))
    t0 = time.perf_counter()
    r = oracle.solve_node(d.X, d.y, d.loss, d.lam2, d.M, d.k, tol=1e-6, max_iter=cap, L=L)
    t = time.perf_counter() - t0
    return t, r.iters, r.status == oracle.CONVERGED, r.gap_rel, t / max(r.iters, 1)


def single_workload(args):
    """One root relaxation per dataset, solved to the FP64-certified 1e-6 gap: wall time of a
    whole solve (median of 5 after 3 warm-up solves, inputs resident in HBM), iterations, and the
    achieved bandwidth of the products from HIP events in one more, profiled solve."""
    desc, runs = SINGLE_WORKLOADS[args.workload]
    ctx = _lib.Context(0)
    rows = []
    cpu = None
    cache = {}
    for name, prec in runs:
        if name not in cache:
            cache.clear()
            cache[name] = synth.make_config(name)
        d = cache[name]
        if not args.no_cpu and cpu is None and prec == "f64":
            t, it, conv, gap, spi = _oracle_sample(d)
            cpu = {"config": name, "seconds": t, "iters": it, "converged": conv, "gap": gap,
                   "s_per_iter": spi}
        prob = _lib.Problem(ctx, d.X_store, d.y, loss=d.loss, lam2=d.lam2, M=d.M, k=d.k)
        for _ in range(3):
            prob.solve(tol=1e-6, precision=prec)
        times, res = [], None
        for _ in range(5):
            t0 = time.perf_counter()
            res = prob.solve(tol=1e-6, precision=prec)
            times.append(time.perf_counter() - t0)
        for w in range(10):
            ctx.kernel_stats(w, reset=True)
        ctx.set_profiling(True)
        prob.solve(tol=1e-6, precision=prec)
        ctx.set_profiling(False)
        sx = d.X_store.dtype.itemsize
        row = {"config": name, "x_dtype": {8: "f64", 4: "f32", 2: "bf16"}[sx], "path": prec,
               "time_to_tol_s": round(statistics.median(times), 5),
               "times_s": [round(t, 5) for t in times], "iters": res.iters,
               "restarts": res.restarts, "gap_rel": res.gap_rel, "status": res.status,
               "primal": res.primal, "lower_bound": res.lower_bound}
        kernels = {}
        for which in ((0, 1) if prec == "f64" else (2,)):
            r = roofline(ctx, d.n, d.p, sx if prec == "f64" else 2, 1 if prec == "f64" else 256,
                         which)
            if r is not None:
                kernels[KERNEL_NAMES[which]] = r
        row["kernels"] = kernels
        rows.append(row)
        prob.close()
        print(f"# {name} {prec}: {row['time_to_tol_s'] * 1e3:.1f} ms, {res.iters} iterations, "
              f"gap {res.gap_rel:.2e}", file=sys.stderr, flush=True)
    head = rows[0]
    dom = head["kernels"].get(KERNEL_NAMES[0])
    out = {
        "metric": "time to 1e-6 relative gap, one root relaxation",
        "value": head["time_to_tol_s"],
        "unit": "s",
        "n_gpus": 1,
        "steps": 5,
        "warmup": 3,
        "ms_per_step": round(head["time_to_tol_s"] * 1e3, 3),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "runs": [f"{n}/{p}" for n, p in runs]},
        "roofline": dom,
        "results": rows,
    }
    if cpu is not None:
        est = cpu["s_per_iter"] * head["iters"]
        out["cpu_baseline"] = {
            "value": round(cpu["seconds"] if cpu["converged"] else est, 3), "unit": "s",
            "cores": host_cores(), "kind": "oracle",
            "sample": (f"oracle (FP64 NumPy, BLAS on the host cores) on the {cpu['config']} root "
                       f"node: {cpu['iters']} iterations in {cpu['seconds']:.1f} s, "
                       + ("run to the certified 1e-6 gap" if cpu["converged"] else
                          f"stopped at its iteration cap (gap {cpu['gap']:.1e}); value = its "
                          f"{cpu['s_per_iter']:.3f} s per iteration x the GPU path's "
                          f"{head['iters']} iterations"))}
    print(json.dumps(out))


def copy_calibration(nbytes: int) -> None:
    """One plain device-to-device copy of a known size through the HIP runtime's copy kernel
    (the reference for the traffic counters)."""
    import ctypes

    hip = ctypes.CDLL("libamdhip64.so")
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    for ptr in (a, b):
        if hip.hipMalloc(ctypes.byref(ptr), ctypes.c_size_t(nbytes)) != 0:
            raise RuntimeError("hipMalloc failed")
    try:
        if hip.hipMemset(a, 1, ctypes.c_size_t(nbytes)) != 0 or hip.hipDeviceSynchronize() != 0:
            raise RuntimeError("hipMemset failed")
        if hip.hipMemcpy(b, a, ctypes.c_size_t(nbytes), 3) != 0:  # device to device
            raise RuntimeError("hipMemcpy failed")
        if hip.hipDeviceSynchronize() != 0:
            raise RuntimeError("hipDeviceSynchronize failed")
    finally:
        hip.hipFree(a)
        hip.hipFree(b)
    print(f"# copy calibration: {nbytes} bytes", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nodes", type=int, default=256)
    ap.add_argument("--plain-nodes", type=int, default=16,
                    help="nodes of the plain FP64 per-node comparator")
    ap.add_argument("--stream-batches", type=int, default=4,
                    help="batched: batches of --nodes nodes streamed through the engine's slots in "
                         "one call after the timed steps (0: skip)")
    ap.add_argument("--check-every", type=int, default=2,
                    help="batched: dual-monitor period of the mixed-precision nodes (iterations; "
                         "the plain FP64 comparator keeps 1)")
    ap.add_argument("--mode", choices=["auto", "batched", "plain"], default="auto")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-nodes-per-core", type=int, default=2,
                    help="cpu_baseline: oracle node solves per host core (one process per core)")
    ap.add_argument("--workload", choices=["batched", "serve", "prox", "c1", "c2", "c3"],
                    default="batched",
                    help="batched: the 256-node step (default); serve: the request stream; "
                         "prox: the standalone prox workload; c1, c2, c3: one root relaxation "
                         "(least squares tiny; FP64/FP32; logistic plain vs BF16-X)")
    ap.add_argument("--prox-batch", type=int, default=256, help="prox: vectors per launch")
    ap.add_argument("--prox-max-i", type=int, default=10,
                    help="prox: sizes p = 100 * 2^i for i = 0..this (Fig. 1 runs to i = 10)")
    ap.add_argument("--requests", type=int, default=3000,
                    help="serve: number of requests (3000 at 2000/s: 1.5 s of arrivals, long "
                         "enough for the engines to reach their steady occupancy)")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve: mean arrivals per second")
    ap.add_argument("--serve-sizes", default="1000,5000,20000", help="serve: dataset p values")
    ap.add_argument("--no-share", action="store_true",
                    help="serve: an engine per problem (the two losses of a dataset apart)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="after the run, one device copy of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (nodes shard "
              "across GPUs with no per-iteration communication; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "prox":
        prox_workload(args)
        return
    if args.workload in SINGLE_WORKLOADS:
        single_workload(args)
        if args.copy_bytes > 0:
            copy_calibration(args.copy_bytes)
        return
    if args.workload == "serve":
        # one hardware queue per resident engine's stream (six engines, the context's stream and
        # the retirement copies), read by the HIP runtime when it starts (no HIP call has been
        # made yet): with the default four, a small design's kernels wait behind a large
        # design's in a shared queue
        os.environ.setdefault("GPU_MAX_HW_QUEUES", "8")
        serve(args)
        if args.copy_bytes > 0:
            copy_calibration(args.copy_bytes)
        return

    t_setup = time.perf_counter()
    d = synth.make_config("c4")
    sets = synth.node_sets(d.p, d.k, args.nodes, 20, config_id=4)
    # the oracle on the host cores first: its workers are forked before any device call
    cpu = None if args.no_cpu else cpu_baseline(d, sets, args.cpu_nodes_per_core)
    ctx = _lib.Context(0)
    prob = _lib.Problem(ctx, d.X_store, d.y, loss="ls", lam2=d.lam2, M=d.M, k=d.k)
    L = prob.L
    print(f"# setup {time.perf_counter() - t_setup:.1f}s  L={L:.6g}", file=sys.stderr, flush=True)

    # the batched engine's working-precision dual monitor only decides when a node asks for its
    # FP64 certificate; every second iteration is enough (and faster); the FP64 path evaluates
    # its bound every iteration
    def specs(prec):
        ce = args.check_every if prec == "mixed" else 1
        return [prob.node(Z0=z0, Z1=z1, tol=1e-6, precision=prec, check_every=ce)
                for z0, z1 in sets]

    mode = args.mode
    engine_setup_ms = None
    if mode in ("auto", "batched"):
        # the first batched solve builds the engine (BF16 copies, split-K tuning, graphs and, for
        # least squares, the FP64 Gram matrix); its time is reported, not part of a step
        t_eng = time.perf_counter()
        try:
            prob.solve_batch(specs("mixed")[:1])
            engine_setup_ms = (time.perf_counter() - t_eng) * 1e3
            mode = "batched"
        except _lib.CglError:
            if mode == "batched":
                raise
            mode = "plain"
    step_specs = specs("mixed" if mode == "batched" else "f64")

    # the solutions of every step land in one host buffer that persists across steps, as a
    # branch-and-bound caller's would (its pages are mapped before the timed region)
    out = np.empty((len(step_specs), d.p))
    out.fill(0.0)
    for _ in range(args.warmup):
        prob.solve_batch(step_specs, out=out)
    # timed steps: the production path (graph-captured chunks), with only the host wall time of
    # the engine's phases recorded (batched engine)
    ctx.set_profiling(True, phases_only=True)
    for w in range(16):
        ctx.kernel_stats(w, reset=True)
    t0 = time.perf_counter()
    results = []
    for _ in range(args.steps):
        results = prob.solve_batch(step_specs, out=out)
    t1 = time.perf_counter()
    ctx.set_profiling(False)
    elapsed = t1 - t0
    value = args.steps * len(step_specs) / elapsed
    phases = None
    if mode == "batched":
        phases = {}
        for w, name in ((5, "iteration_chunks"), (6, "certification_rounds"),
                        (7, "admission_retirement"), (10, "chunks_gpu"),
                        (11, "certification_rounds_gpu")):
            ms, cnt = ctx.kernel_stats(w, reset=True)
            phases[name] = {"ms_per_step": round(ms / args.steps, 3), "count_per_step": cnt / args.steps}
        phases["reorders_per_step"] = ctx.kernel_stats(12, reset=True)[1] / args.steps
        # cycles of the timed steps (one X pass each) and the share of the columns they read:
        # the X pass reads only the operand's nonzero prefix of the support-first column order
        frac, passes = ctx.kernel_stats(9, reset=True)
        if passes:
            cycles = passes / args.steps
            phases["x_pass_kernel"] = {"count_per_step": cycles,
                                       "mean_columns_read": round(frac / passes, 4),
                                       "tiling": tiling_desc(ctx.kernel_stats(14)[0])}
            for name in ("iteration_chunks", "chunks_gpu"):
                phases[name]["us_per_cycle"] = round(1e3 * phases[name]["ms_per_step"] / cycles, 1)
    # one more step, untimed, with kernel events on the roofline's kernel (its launches then run
    # outside graphs): the kernel's live average launch time and the per-cycle kernel figures
    for w in range(12):
        ctx.kernel_stats(w, reset=True)
    ctx.set_profiling(True)
    prob.solve_batch(step_specs, out=out)
    ctx.set_profiling(False)
    roof = roofline(ctx, d.n, d.p, 2, len(step_specs), 2 if mode == "batched" else 0)
    if roof is not None:
        roof["timed_in"] = "one extra profiled step after the timed steps (same nodes)"
    if mode == "batched":
        for w, name in ((2, "xt_pass_kernel"), (4, "fp64_pass_kernel")):
            ms, cnt = ctx.kernel_stats(w)
            phases[name] = {"ms_per_step": round(ms, 3), "count_per_step": cnt,
                            "from": "the profiled step"}
    ok = all(r.status == "converged" and r.gap_rel <= 1e-6 for r in results)
    iters = [r.iters for r in results]
    print(f"# {mode}: {value:.2f} solves/s, all certified: {ok}, iterations median "
          f"{statistics.median(iters)} max {max(iters)}", file=sys.stderr, flush=True)

    # continuous batching, as a branch-and-bound driver feeds the engine: several batches of
    # nodes of the same kind in one call, each node admitted into a slot as soon as one frees, so
    # the tail of one batch overlaps the next (a warm-up call first, then the measured one)
    stream = None
    if mode == "batched" and args.stream_batches > 0:
        csets = synth.node_sets(d.p, d.k, args.stream_batches * len(step_specs), 20, seed=3,
                                config_id=4)
        cspecs = [prob.node(Z0=z0, Z1=z1, tol=1e-6, precision="mixed",
                            check_every=args.check_every) for z0, z1 in csets]
        cout = np.empty((len(cspecs), d.p))
        cout.fill(0.0)
        prob.solve_batch(cspecs[: len(step_specs)], out=cout[: len(step_specs)])
        ctx.set_profiling(True, phases_only=True)
        for w in range(16):
            ctx.kernel_stats(w, reset=True)
        tc0 = time.perf_counter()
        cres = prob.solve_batch(cspecs, out=cout)
        tc = time.perf_counter() - tc0
        ctx.set_profiling(False)
        cphases = {}
        for w, name in ((5, "iteration_chunks"), (6, "certification_rounds"),
                        (7, "admission_retirement"), (10, "chunks_gpu"),
                        (11, "certification_rounds_gpu")):
            ms, cnt = ctx.kernel_stats(w, reset=True)
            cphases[name] = {"ms": round(ms, 3), "count": cnt}
        frac, passes = ctx.kernel_stats(9, reset=True)
        if passes:
            cphases["x_pass_kernel"] = {"count": passes, "mean_columns_read": round(frac / passes, 4)}
        cphases["reorders"] = ctx.kernel_stats(12, reset=True)[1]
        cphases["admissions"] = ctx.kernel_stats(13, reset=True)[1]
        cit = [r.iters for r in cres]
        stream = {"solves_per_s": round(len(cspecs) / tc, 1), "nodes": len(cspecs),
                  "batches": args.stream_batches, "ms": round(1e3 * tc, 2),
                  "all_certified": all(r.status == "converged" and r.gap_rel <= 1e-6 for r in cres),
                  "iterations": {"median": statistics.median(cit), "max": max(cit)},
                  "phases": cphases,
                  "note": "one call; nodes fill slots as they free (not the headline value)"}
        print(f"# stream of {len(cspecs)} nodes: {stream['solves_per_s']} solves/s", file=sys.stderr,
              flush=True)

    # plain FP64 per-node comparator on the first nodes (each solve is its own latency)
    plain = None
    if mode == "batched" and args.plain_nodes > 0:
        pspecs = specs("f64")[: args.plain_nodes]
        lat = []
        pres = []
        tp0 = time.perf_counter()
        for s in pspecs:
            ts = time.perf_counter()
            pres += prob.solve_batch([s])
            lat.append(time.perf_counter() - ts)
        tp = time.perf_counter() - tp0
        plain = {"solves_per_s": len(pspecs) / tp, "nodes": len(pspecs),
                 "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                 "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                 "iterations": {"median": statistics.median([r.iters for r in pres]),
                                "max": max(r.iters for r in pres)},
                 "restarts": {"median": statistics.median([r.restarts for r in pres]),
                              "max": max(r.restarts for r in pres)},
                 "batched_same_nodes": {
                     "iterations_median": statistics.median([r.iters for r in results[:len(pspecs)]]),
                     "restarts_median": statistics.median([r.restarts for r in results[:len(pspecs)]])}}

    out = {
        "metric": "node relaxations solved/sec at 1e-6 gap, batched vs plain; p50/p99 latency",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-mfma/fp32-acc + fp64 bound" if mode == "batched" else "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "nodes": len(step_specs), "n": d.n, "p": d.p,
                   "x_dtype": "bf16", "engine": mode,
                   "monitor_every": args.check_every if mode == "batched" else 1},
        "all_certified": ok,
        "iterations": {"median": statistics.median(iters), "p99": float(np.percentile(iters, 99)),
                       "max": max(iters)},
        "restarts": {"median": statistics.median([r.restarts for r in results]),
                     "max": max(r.restarts for r in results)},
        "roofline": roof,
    }
    if phases is not None:
        out["phases"] = phases
    if engine_setup_ms is not None:
        out["engine_setup_ms"] = round(engine_setup_ms, 1)
    if mode == "plain":
        out["latency_ms"] = {"note": "per-node solve time on the plain path, sequential",
                             "p50": round(1e3 * elapsed / args.steps / len(step_specs), 3)}
    if stream is not None:
        out["continuous_batching"] = stream
    if plain is not None:
        out["plain_fp64_per_node"] = plain
        out["speedup_vs_plain"] = round(value / plain["solves_per_s"], 2)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))
    if args.copy_bytes > 0:
        copy_calibration(args.copy_bytes)


if __name__ == "__main__":
    main()
