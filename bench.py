#!/usr/bin/env python3
"""Benchmark of the dense 3-way MTTKRP / CP-ALS hot path on one MI355X.

Default workload (N=1): the 1024 x 1024 x 1024 FP32 tensor (4 GiB), rank-64
CP model plus N(0, 1e-3) noise, R = 64 factors iid N(0,1) (synthetic,
seeded).  The headline path is the bf16x3 contraction (each FP32 operand
split into bf16 hi + lo, three bf16 MFMA products, FP32 accumulation); the
plain FP32 path (FP32 MFMA) and the bf16x6 path (three bf16 terms per
operand, six products: FP32-level error) are timed beside it on the same
tensor.  One step
= one CP-ALS sweep on the device: for each mode an MTTKRP (for FP32 tensors
with K >= 8R the mode-1 and mode-2 MTTKRPs come from one shared contraction
Y = X x3 C, the dimension tree, so the sweep reads X twice) followed by the
FP64 Gram / LDL^T (Cholesky) inverse / solve / normalise update.

``value`` is the algorithmic MTTKRP rate of the headline sweep: 3 x 2*I*J*K*R
flop per sweep (the three MTTKRPs a sweep defines) over the measured sweep
time; the flops the dimension tree actually executes are in ``detail``.

Also measured live, with HIP events on the stream the library launches on:
each mode's MTTKRP on its own for both paths, and the kernel that takes the
largest share of the headline sweep (the roofline object).  The FP64 oracle
runs on the host cores as ``cpu_baseline`` (timed on a bounded sample); its
full MTTKRPs also give each path's per-mode error over every output row.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]
                    [--workload cp1024_r64|cp512_r32|cp768_r128_sliced|cp64_r8|serve|copy|
                                coo64k_nnz64m_r64|coo64k_nnz64m_r64_zipf|nway4_128_r32]
                    [--prec fp32|bf16x3|bf16x6|fp8] [--compare fp32[,bf16x6]|none] [--no-cpu-baseline]

``--workload cp768_r128_sliced`` (FP8 e4m3, per-slice scales) also runs the
workload's 20 CP-ALS sweeps and reports their fit and model against the
oracle's 20 sweeps (``tests/golden/cp768_r128_als.json``, written by the
oracle).  ``--workload serve`` runs the serving workload instead (see
serve_bench); the ``coo*`` workloads run sparse CP-ALS (see sparse_bench) and
``nway4_128_r32`` four-way CP-ALS (see nway_bench).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Dense MFMA peaks per path, in algorithmic flops: bf16x3 issues three bf16
# MFMA products per product of the definition, bf16x6 six, FP8 two e4m3 ones.
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2516.6, "fp8": 5033.2}
PEAK_TFLOPS = {"fp32": 157.3, "bf16x3": 2516.6 / 3.0, "bf16x6": 2516.6 / 6.0, "fp8": 5033.2 / 2.0}
DEFAULT_PREC = {"cp64_r8": "fp32", "cp512_r32": "fp32", "cp1024_r64": "bf16x3", "cp768_r128_sliced": "fp8"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(dims, R, mode, prec):
    """Bytes an MTTKRP must move: the tensor in its storage format, the two
    input factors and the output (FP32); FP8 adds the slice exponents."""
    I, J, K = dims
    elem = 1 if prec == "fp8" else 4
    others = [d for m, d in enumerate(dims) if m != mode]
    b = I * J * K * elem + 4 * R * sum(others) + 4 * dims[mode] * R
    if prec == "fp8":
        b += 4 * I
    return b


# The dense contraction kernels that a traffic record can describe are built
# from these sources and the headers they include.
DENSE_KERNEL_SOURCES = ("mttkrp_kernels.hip", "dimtree.hip")


def kernel_source_files():
    """DENSE_KERNEL_SOURCES and, transitively, the library headers they
    include (the public header excepted: it declares, it builds nothing)."""
    import re
    d = os.path.join(ROOT, "paper_2411_04785_amd", "csrc")
    seen, todo = set(), list(DENSE_KERNEL_SOURCES)
    while todo:
        f = todo.pop()
        if f in seen or not os.path.exists(os.path.join(d, f)):
            continue
        seen.add(f)
        todo += re.findall(r'^#include "([A-Za-z0-9_]+\.h)"', open(os.path.join(d, f)).read(), flags=re.M)
    return sorted(seen)


def kernel_sources_hash():
    """sha256 prefix of the dense contraction kernels' sources (to tell
    whether a recorded counter measurement still describes the built
    kernels)."""
    import hashlib
    d = os.path.join(ROOT, "paper_2411_04785_amd", "csrc")
    src = b"".join(open(os.path.join(d, f), "rb").read() for f in kernel_source_files())
    return hashlib.sha256(src).hexdigest()[:16]


def recorded_traffic(workload, prec, kernel=None):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE runs, or None if none match this workload and kernel or the
    kernel sources changed since.  A record holds either one kernel
    ("kernel", "traffic_bytes_per_launch_mean") or several
    ("traffic_bytes_per_launch": {kernel: bytes})."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{prec}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_sources_sha256_16") != kernel_sources_hash():
        return None
    per = rec.get("traffic_bytes_per_launch")
    if per is not None:
        return per.get(kernel) if kernel is not None else None
    if kernel is not None and rec.get("kernel", kernel) != kernel:
        return None
    return rec["traffic_bytes_per_launch_mean"]


def ytree_bytes(dims, R):
    """Bytes the dimension tree's Y kernel must move: X (FP32), C, B, Y
    (I*J x R FP32, written) and its partial rows of M1 (J / 256 slices below
    R = 65, J / 128 above; the Y kernel forms them when J is a multiple of
    that)."""
    I, J, K = dims
    rows = 256 if R <= 64 else 128
    parts = J // rows if J % rows == 0 else 0
    return 4 * I * J * K + 4 * K * R + 4 * J * R + 4 * I * J * R + 4 * parts * I * R


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline(X, facs, reps=3):
    """The FP64 oracle on the host: each mode's full MTTKRP once (the
    references for the per-mode errors), then the mode-0 MTTKRP `reps` more
    times; the reported rate is the median of those `reps` timings."""
    import oracle
    I, J, K = X.shape
    R = facs[0].shape[1]
    flop = 2.0 * I * J * K * R
    refs, ref_s = [], []
    for mode in range(3):
        t0 = time.perf_counter()
        refs.append(oracle.mttkrp(X, facs, mode))
        ref_s.append(time.perf_counter() - t0)
        log(f"[bench] oracle mode {mode}: {ref_s[-1]:.2f} s")
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        oracle.mttkrp(X, facs, 0)
        ts.append(time.perf_counter() - t0)
    med = float(np.median(ts))
    out = {"value": round(flop / med / 1e9, 2), "unit": "GFLOP/s", "cores": int(blas_threads()), "kind": "oracle",
           "sample": f"FP64 oracle mode-1 MTTKRP of the same {I}x{J}x{K} tensor, R={R} (unfolding x explicit "
                     f"Khatri-Rao product, BLAS), median of {reps} runs: {', '.join(f'{t:.2f}' for t in ts)} s",
           "all_modes_s": [round(t, 3) for t in ref_s]}
    if I * J * K <= 512**3:
        try:
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1, user_api="blas"):
                t0 = time.perf_counter()
                oracle.mttkrp(X, facs, 0)
                t1 = time.perf_counter() - t0
            out["single_thread_value"] = round(flop / t1 / 1e9, 2)
        except Exception:
            pass
    return out, refs


def serve_cpu_baseline(reqs, inputs, done, n=6, seed=5):
    """The FP64 oracle's CP-ALS on a seeded sample of the served requests
    (same inputs, same sweep count), timed on the host: requests/s of the
    oracle, and each sampled request's served fit against the oracle's."""
    import oracle
    g = np.random.default_rng(seed)
    pick = sorted(g.choice(len(reqs), size=min(n, len(reqs)), replace=False).tolist())
    t_all, diffs = 0.0, []
    for q in pick:
        r = reqs[q]
        X, init = inputs[q]
        t0 = time.perf_counter()
        fa, la, _ = oracle.cp_als(X, init, r.sweeps, fit_every_sweep=False)
        t_all += time.perf_counter() - t0
        diffs.append(abs(done[r.rid]["fit"] - oracle.fit(X, fa, la)))
    cpu = {"value": round(len(pick) / t_all, 3), "unit": "req/s", "cores": int(blas_threads()), "kind": "oracle",
           "sample": f"FP64 oracle CP-ALS ({reqs[0].sweeps} sweeps, LU solves) of {len(pick)} seeded requests "
                     f"of the stream (ids {pick}), {t_all:.2f} s"}
    return cpu, [float(f"{d:.2e}") for d in diffs]


def serve_bench(args):
    """Open-loop serving run; prints one JSON line.

    A scheduler thread dispatches each request at its Poisson arrival time
    to a pool of submitter threads (the library copies the request into
    pinned memory inside mtk_server_submit, with Python's lock released), so
    one large request's copy does not delay the next arrival.  Latency is
    completion minus scheduled arrival; the submitters' lateness (start of
    the submit call minus scheduled arrival) is reported on its own."""
    import threading
    from concurrent.futures import ThreadPoolExecutor

    from paper_2411_04785_amd import synth
    from paper_2411_04785_amd.mttkrp import Server

    reqs = synth.make_requests(args.requests, args.rate)
    pool = synth.NoisePool()
    log(f"[serve] generating {len(reqs)} requests")
    t0 = time.perf_counter()
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        inputs = list(ex.map(lambda r: synth.request_tensor(r, pool), reqs))
    log(f"[serve] generated in {time.perf_counter() - t0:.1f} s "
        f"({sum(x.nbytes for x, _ in inputs) / 1e9:.1f} GB)")
    prec = args.prec or "fp32"
    srv = Server(0, budget_bytes=int(args.budget), max_slots=args.slots)
    # Warm the kernels (first launches load code objects) with one small request.
    srv.submit(-1, inputs[0][0], inputs[0][1], prec, sweeps=1)
    while not srv.poll(timeout_s=1.0):
        pass
    done = {}
    lateness = {}
    subs = ThreadPoolExecutor(8)

    def submit(r, X, init, sched):
        lateness[r.rid] = time.perf_counter() - sched
        srv.submit(r.rid, X, init, prec, sweeps=r.sweeps)

    def scheduler():
        start = time.perf_counter()
        for r, (X, init) in zip(reqs, inputs):
            sched = start + r.arrival_s
            delay = sched - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            subs.submit(submit, r, X, init, sched)

    th = threading.Thread(target=scheduler)
    tw = time.perf_counter()
    th.start()
    while len(done) < len(reqs):
        for res in srv.poll(timeout_s=0.5):
            done[res["id"]] = res
    th.join()
    subs.shutdown()
    wall = time.perf_counter() - tw
    stats = srv.stats()
    srv.close()
    log(f"[serve] open loop: {len(reqs)} requests in {wall:.2f} s; {stats}")

    # Closed loop on the first requests of the same stream: keep 2 x slots
    # requests outstanding; the completion rate is the saturation throughput.
    nsat = min(len(reqs), args.sat_requests)
    srv = Server(0, budget_bytes=int(args.budget), max_slots=args.slots)
    srv.submit(-1, inputs[0][0], inputs[0][1], prec, sweeps=1)
    while not srv.poll(timeout_s=1.0):
        pass
    nxt = got = inflight = 0
    ts = time.perf_counter()
    while got < nsat:
        while inflight < 2 * args.slots and nxt < nsat:
            X, init = inputs[nxt]
            srv.submit(reqs[nxt].rid, X, init, prec, sweeps=reqs[nxt].sweeps)
            nxt += 1
            inflight += 1
        for _ in srv.poll(timeout_s=0.5):
            got += 1
            inflight -= 1
    sat = nsat / (time.perf_counter() - ts)
    sat_stats = srv.stats()
    srv.close()
    log(f"[serve] closed loop: {nsat} requests at {sat:.1f} req/s")
    # Latency: completion (server clock) minus scheduled arrival.
    lat = np.array([done[r.rid]["t_done"] - done[r.rid]["t_submit"] + lateness[r.rid] for r in reqs])
    late = np.array([lateness[r.rid] for r in reqs])
    status_bad = sum(1 for r in reqs if done[r.rid]["status"] != 0)
    cpu, fit_diffs = (None, None)
    if not args.no_cpu_baseline:
        log("[serve] FP64 oracle on a seeded sample of the requests")
        cpu, fit_diffs = serve_cpu_baseline(reqs, inputs, done)

    def ms(v):
        return round(1e3 * float(v), 2)

    line = {
        "metric": "served CP-ALS requests/s (open loop) with p50/p99 latency",
        "value": round(len(reqs) / wall, 2), "unit": "req/s", "n_gpus": 1, "steps": len(reqs), "warmup": 1,
        "ms_per_step": round(1e3 * wall / len(reqs), 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if prec == "fp32" else prec, "data": "synthetic",
        "config": {"workload": f"serve: {len(reqs)} requests, Poisson {args.rate}/s, dims U[32,384]^3, "
                               f"R in {{8,16,32,64}}, N(0,1e-4) noise, 10 sweeps, budget {args.budget:.3g} B, "
                               f"{args.slots} slots", "prec": prec},
        "latency_ms": {"p50": ms(np.percentile(lat, 50)), "p99": ms(np.percentile(lat, 99)),
                       "max": ms(lat.max()), "mean": ms(lat.mean())},
        "cpu_baseline": cpu,
        "detail": {"wall_s": round(wall, 3), "offered_rate": args.rate, "failed": status_bad,
                   "submit_lateness_ms": {"p50": ms(np.percentile(late, 50)), "p99": ms(np.percentile(late, 99)),
                                          "max": ms(late.max())},
                   "saturation_req_s": round(sat, 2), "saturation_requests": nsat,
                   "scheduler_steps": stats["steps"], "max_requests_per_step": stats["max_batch"],
                   "saturation_max_requests_per_step": sat_stats["max_batch"],
                   "peak_bytes_in_use": stats["peak_bytes_in_use"], "device_bytes": stats["device_bytes"],
                   "fit_abs_err_vs_oracle_sample": fit_diffs},
    }
    print(json.dumps(line), flush=True)


def copy_bench(args):
    """A plain device copy of 512 MiB (the size of the 512^3 FP32 tensor),
    timed with HIP events: the calibration run for the HBM byte counters."""
    import torch
    n = 512 * 512 * 512
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(max(1, args.warmup)):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    print(json.dumps({"metric": "device copy GB/s (read + write)", "value": round(2 * n * 4 / ms / 1e6, 1),
                      "unit": "GB/s", "bytes_read_per_copy": n * 4, "bytes_written_per_copy": n * 4,
                      "ms_per_copy": round(ms, 4), "steps": args.steps}), flush=True)




SPARSE_WORKLOADS = {
    # dims, nnz, R, Zipf exponent of the mode-0 index (None: uniform)
    "coo64k_nnz64m_r64": ((1 << 16,) * 3, 1 << 26, 64, None),
    "coo64k_nnz64m_r64_zipf": ((1 << 16,) * 3, 1 << 26, 64, 1.2),
}


def coo_bytes(dims, nnz, R, mode):
    """Bytes a mode-n sparse MTTKRP must move: the entries in the library's
    form (16 bytes each), the two gathered factors once, the output once."""
    others = [d for m, d in enumerate(dims) if m != mode]
    return 16 * nnz + 4 * R * sum(others) + 4 * R * dims[mode]


def sparse_bench(args):
    """Sparse CP-ALS on one MI355X: a step is one sweep (mttkrp_coo and
    gram_solve for modes 0, 1, 2) over a seeded sparse tensor already in the
    library's form on the device."""
    import torch
    import oracle
    from paper_2411_04785_amd import synth
    from paper_2411_04785_amd.mttkrp import Context
    dims, nnz, R, skew = SPARSE_WORKLOADS[args.workload]
    t0 = time.perf_counter()
    idx, vals = synth.coo(dims, nnz, seed=2411, skew=skew)
    facs = synth.gaussian_factors(2412, synth.STREAM_INIT, dims, R)
    log(f"[bench] {args.workload}: inputs drawn in {time.perf_counter() - t0:.1f} s")
    ctx = Context(0)
    stream = torch.cuda.current_stream()
    di = [torch.from_numpy(i).cuda() for i in idx]
    dv = torch.from_numpy(vals).cuda()
    f0 = [torch.from_numpy(f.astype(np.float32)).cuda() for f in facs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t = ctx.coo_create(dims, di, dv)
    create_s = time.perf_counter() - t0
    del di, dv
    mode_ms, outs = [], []
    for mode in range(3):
        out = ctx.mttkrp_coo(t, f0, mode)
        if mode == 0:
            gpu_warm(torch, lambda: ctx.mttkrp_coo(t, f0, 0, out=out))
        mode_ms.append(time_calls(torch, stream, lambda: ctx.mttkrp_coo(t, f0, mode, out=out), args.mode_reps))
        outs.append(out.cpu().numpy().astype(np.float64))
        log(f"[bench] mode {mode}: {mode_ms[-1] * 1e3:.1f} us per sparse MTTKRP")
    # Sampled output rows of every mode against the oracle over their entries.
    g = np.random.default_rng(5)
    worst = 0.0
    for mode in range(3):
        rows = np.unique(g.integers(0, dims[mode], 32))
        sel = np.isin(idx[mode], rows)
        sub = [i[sel] for i in idx]
        ref = oracle.mttkrp_coo(sub, vals[sel], dims, facs, mode)[rows]
        s_abs = oracle.mttkrp_coo(sub, np.abs(vals[sel]), dims, [np.abs(f) for f in facs], mode)[rows]
        n = np.bincount(sub[mode], minlength=dims[mode])[rows].astype(np.float64)
        bound = (n[:, None] + 3.0) * 2.0 ** -24 * s_abs
        worst = max(worst, float((np.abs(outs[mode][rows] - ref) / np.maximum(bound, 1e-300)).max()))
    fd = [f.clone() for f in f0]
    lam = torch.ones(R, dtype=torch.float64, device="cuda")
    ctx.als_sweep_coo(t, fd, lam, max(1, args.warmup))
    torch.cuda.synchronize()
    e0, e1 = _events(torch, stream)
    e0.record(stream)
    ctx.als_sweep_coo(t, fd, lam, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    flop_mttkrp = 3.0 * nnz * R
    value = 3 * flop_mttkrp / (ms_step * 1e-3) / 1e9
    m = int(np.argmax(mode_ms))
    nbytes = coo_bytes(dims, nnz, R, m)
    ach = nbytes / (mode_ms[m] * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": f"mode-{m + 1} sparse MTTKRP (coo_mttkrp_kernel + zero fill + carry levels)",
            "avg_launch_us": round(mode_ms[m] * 1e3, 2), "algorithmic_bytes": int(nbytes),
            "factor_row_gather_bytes": int(8 * R * nnz),
            "factor_row_gather_GBs": round(8 * R * nnz / (mode_ms[m] * 1e-3) / 1e9, 1)}
    cpu = None
    if not args.no_cpu_baseline:
        ns = 1 << 22
        sub = [i[:ns] for i in idx]
        ts = []
        for _ in range(3):
            c0 = time.perf_counter()
            oracle.mttkrp_coo(sub, vals[:ns], dims, facs, 0)
            ts.append(time.perf_counter() - c0)
        med = float(np.median(ts))
        cpu = {"value": round(3.0 * ns * R / med / 1e9, 3), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
               "sample": f"FP64 oracle mode-1 sparse MTTKRP (numpy gather + unbuffered scatter-add) of the first "
                         f"{ns} entries of the same tensor, R={R}, median of 3 runs: "
                         f"{', '.join(f'{x:.2f}' for x in ts)} s"}
    print(json.dumps({
        "metric": "sparse MTTKRP GFLOP/s (algorithmic, 3 x 3*nnz*R per sparse CP-ALS sweep)",
        "value": round(value, 1), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "dims": list(dims), "nnz": nnz, "R": R,
                   "mode0_index": "uniform" if skew is None else f"zipf {skew}"},
        "roofline": roof, "cpu_baseline": cpu,
        "detail": {"mode_us": [round(x * 1e3, 1) for x in mode_ms], "create_s": round(create_s, 4),
                   "sampled_rows_max_err_over_fp32_sum_bound": round(worst, 4),
                   "lambda_finite": bool(torch.isfinite(lam).all().item())}}), flush=True)
    t.close()


NWAY_WORKLOADS = {
    # dims, rank of the CP tensor, R, noise variance
    "nway4_128_r32": ((128, 128, 128, 128), 32, 32, 1e-4),
}


def nway_bench(args):
    """Order-N CP-ALS on one MI355X: a step is one sweep of als_sweep_nway
    (every mode: the merged groups' Khatri-Rao rows, the three-way
    contraction of the view, the update) over a seeded 4-way CP tensor."""
    import torch
    import oracle
    from paper_2411_04785_amd import synth
    from paper_2411_04785_amd.mttkrp import Context
    dims, rank, R, nv = NWAY_WORKLOADS[args.workload]
    prec = args.prec or "bf16x3"
    t0 = time.perf_counter()
    X, init = synth.cp_nway(dims, rank, R, seed=2413, noise_var=nv)
    log(f"[bench] {args.workload}: inputs drawn in {time.perf_counter() - t0:.1f} s")
    ctx = Context(0)
    stream = torch.cuda.current_stream()
    Xd = torch.from_numpy(X).cuda()
    f0 = [torch.from_numpy(f).cuda() for f in init]
    n = len(dims)
    numel = float(np.prod(dims))
    flop_mttkrp = 2.0 * numel * R
    paths = [prec] + [p for p in ("fp32",) if p != prec]
    res = {}
    for p in paths:
        mode_ms, outs = [], []
        for mode in range(n):
            out = ctx.mttkrp_nway(Xd, f0, mode, p)
            if mode == 0:
                gpu_warm(torch, lambda: ctx.mttkrp_nway(Xd, f0, 0, p, out=out))
            mode_ms.append(time_calls(torch, stream, lambda: ctx.mttkrp_nway(Xd, f0, mode, p, out=out),
                                      args.mode_reps))
            outs.append(out.cpu().numpy().astype(np.float64))
        fd = [f.clone() for f in f0]
        lam = torch.ones(R, dtype=torch.float64, device="cuda")
        ctx.als_sweep_nway(Xd, fd, lam, max(1, args.warmup), p)
        torch.cuda.synchronize()
        e0, e1 = _events(torch, stream)
        e0.record(stream)
        ctx.als_sweep_nway(Xd, fd, lam, args.steps, p)
        e1.record(stream)
        torch.cuda.synchronize()
        res[p] = {"mode_ms": mode_ms, "outs": outs, "ms_step": e0.elapsed_time(e1) / args.steps}
        log(f"[bench] {p}: per mode {[round(x * 1e3, 1) for x in mode_ms]} us, sweep {res[p]['ms_step']:.3f} ms")
    refs = [oracle.mttkrp_nway(X, init, mode) for mode in range(n)]
    head = res[prec]
    m = int(np.argmax(head["mode_ms"]))
    others = sum(d for k, d in enumerate(dims) if k != m)
    nbytes = 4 * numel + 4 * R * others + 4 * dims[m] * R
    ach = nbytes / (head["mode_ms"][m] * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": f"mode-{m + 1} N-way MTTKRP (Khatri-Rao rows + contraction of the three-way view)",
            "avg_launch_us": round(head["mode_ms"][m] * 1e3, 2), "algorithmic_bytes": int(nbytes)}
    cpu = None
    if not args.no_cpu_baseline:
        ts = []
        for _ in range(3):
            c0 = time.perf_counter()
            oracle.mttkrp_nway(X, init, 0)
            ts.append(time.perf_counter() - c0)
        med = float(np.median(ts))
        cpu = {"value": round(flop_mttkrp / med / 1e9, 2), "unit": "GFLOP/s", "cores": int(blas_threads()),
               "kind": "oracle", "sample": f"FP64 oracle mode-1 N-way MTTKRP (unfolding x explicit Khatri-Rao "
                                           f"product, BLAS) of the same tensor, median of 3 runs: "
                                           f"{', '.join(f'{x:.2f}' for x in ts)} s"}
    detail = {}
    for p, r in res.items():
        errs = [float(np.linalg.norm(o - ref) / np.linalg.norm(ref)) for o, ref in zip(r["outs"], refs)]
        detail[p] = {"ms_per_sweep": round(r["ms_step"], 4), "mttkrp_us": [round(x * 1e3, 1) for x in r["mode_ms"]],
                     "mttkrp_gbs": [round((4 * numel + 4 * R * (sum(dims) - dims[k]) + 4 * dims[k] * R)
                                          / (t * 1e-3) / 1e9, 1) for k, t in enumerate(r["mode_ms"])],
                     "err_rel_per_mode": [float(f"{e:.3e}") for e in errs]}
    if "fp32" in res and prec != "fp32":
        detail["sweep_speedup_vs_fp32"] = round(res["fp32"]["ms_step"] / head["ms_step"], 3)
    print(json.dumps({
        "metric": "N-way MTTKRP GFLOP/s (algorithmic, N x 2*prod(dims)*R per CP-ALS sweep)",
        "value": round(n * flop_mttkrp / (head["ms_step"] * 1e-3) / 1e9, 1), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(head["ms_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": args.workload, "dims": list(dims), "rank_true": rank, "R": R, "prec": prec},
        "roofline": roof, "cpu_baseline": cpu, "detail": detail}), flush=True)
    ctx.close()


def _events(torch, stream):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    return e0, e1


def gpu_warm(torch, fn, seconds=0.25):
    """Call fn until `seconds` have passed (then synchronise): brings the
    device out of the idle state it sits in while inputs are generated, so
    that the first mode timed is not slower than the others."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(4):
            fn()
        torch.cuda.synchronize()


def time_calls(torch, stream, fn, reps, warm=10):
    """Average ms of fn() over `reps` back-to-back calls, HIP events on the
    library's stream, after `warm` untimed calls (steady clocks, page tables)."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0, e1 = _events(torch, stream)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def run_path(ctx, torch, stream, w, prec, X_run, kw, f0, args):
    """Per-mode MTTKRP times and outputs, then timed CP-ALS sweeps, of one path."""
    R = w.R
    mode_ms, outs = [], []
    for mode in range(3):
        out = ctx.mttkrp(X_run, f0, mode, prec, **kw)
        if mode == 0:
            gpu_warm(torch, lambda: ctx.mttkrp(X_run, f0, 0, prec, out=out, **kw))
        mode_ms.append(time_calls(torch, stream, lambda: ctx.mttkrp(X_run, f0, mode, prec, out=out, **kw),
                                  args.mode_reps))
        outs.append(out.cpu().numpy())
        log(f"[bench] {prec} mode {mode}: {mode_ms[-1] * 1e3:.1f} us per MTTKRP")
    ctx.check()
    fd = [f.clone() for f in f0]
    lam = torch.ones(R, dtype=torch.float64, device=X_run.device)
    ctx.reserve(w.dims, R, prec)
    ctx.als_sweep(X_run, fd, lam, max(1, args.warmup), prec, **kw)
    torch.cuda.synchronize()
    e0, e1 = _events(torch, stream)
    t_wall = time.perf_counter()
    e0.record(stream)
    ctx.als_sweep(X_run, fd, lam, args.steps, prec, **kw)
    e1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_step = e0.elapsed_time(e1) / args.steps
    log(f"[bench] {prec}: {args.steps} sweeps {ms_step:.3f} ms/sweep (wall {t_wall:.3f} s)")
    return {"mode_ms": mode_ms, "outs": outs, "ms_step": ms_step, "factors": fd, "lam": lam}


def dominant_kernel(ctx, torch, stream, w, prec, X_run, kw, f0, mode_ms, reps):
    """The kernel with the largest share of the headline sweep, timed alone
    (HIP events, same stream): with the dimension tree, the Y kernel
    (mttkrp_dimtree mode 0: Y = X x3 C with its partial rows of M1, then a
    reduce of those few rows) or the mode-3 contraction, whichever is longer;
    without it, the slowest mode's contraction.  Returns (name, ms, bytes)."""
    from paper_2411_04785_amd.mttkrp import Context
    cands = []
    if Context.sweep_uses_dimtree(w.dims, w.R, prec):
        out = ctx.mttkrp_dimtree(X_run, f0, 0, prec)
        ms = time_calls(torch, stream, lambda: ctx.mttkrp_dimtree(X_run, f0, 0, prec, out=out), reps)
        cands.append(("ttm_kernel (Y = X x3 C with M1 partial rows) + slice reduce", ms, ytree_bytes(w.dims, w.R)))
        cands.append(("mode-3 contraction (contract_cm_kernel) + split-K reduce", mode_ms[2],
                      algorithmic_bytes(w.dims, w.R, 2, prec)))
    else:
        m = int(np.argmax(mode_ms))
        cands.append((f"mode-{m + 1} contraction + split-K reduce", mode_ms[m], algorithmic_bytes(w.dims, w.R, m, prec)))
    return max(cands, key=lambda c: c[1])


def roofline(name, ms, nbytes, flop, prec):
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    t_cmp = flop / (PEAK_TFLOPS[prec] * 1e12)
    if t_hbm >= t_cmp:
        ach = nbytes / (ms * 1e-3) / 1e9
        r = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(ach / HBM_PEAK_GBS, 4)}
    else:
        ach = flop / (ms * 1e-3) / 1e12
        r = {"bound": "mfma", "achieved": round(ach, 2), "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
             "frac": round(ach / PEAK_TFLOPS[prec], 4)}
    r["kernel"] = name
    r["avg_launch_us"] = round(ms * 1e3, 2)
    r["algorithmic_bytes"] = int(nbytes)
    return r


def err_rows(outs, refs):
    """Per-mode relative Frobenius error over every output row, and the
    worst single row (relative 2-norm over its R values)."""
    e, wr = [], []
    for got, ref in zip(outs, refs):
        d = got.astype(np.float64) - ref
        e.append(float(np.linalg.norm(d) / np.linalg.norm(ref)))
        wr.append(float(np.max(np.linalg.norm(d, axis=1) / np.linalg.norm(ref, axis=1))))
    return [float(f"{v:.3e}") for v in e], [float(f"{v:.3e}") for v in wr]


def fp8_als_vs_oracle(ctx, torch, w, q, kw, Xd, f0):
    """The workload's CP-ALS sweeps on the FP8 tensor against the oracle's
    sweeps on the FP32 tensor (tests/golden/cp768_r128_als.json, written by
    the oracle): fit (direct residual against the unquantised tensor) and the
    model at the recorded sample entries."""
    path = os.path.join(ROOT, "tests", "golden", "cp768_r128_als.json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    fd = [f.clone() for f in f0]
    lam = torch.ones(w.R, dtype=torch.float64, device=Xd.device)
    t0 = time.perf_counter()
    ctx.als_sweep(q, fd, lam, g["sweeps"], "fp8", **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fit = ctx.fit(Xd, fd, lam)
    A, B, C = (f.cpu().numpy().astype(np.float64) for f in fd)
    lv = lam.cpu().numpy()
    got, ref = [], []
    for s, i in enumerate(g["sample_slices"]):
        for (j, k), v in zip(g["sample_jk"][s], g["model_at_samples"][s]):
            got.append(float(np.sum(lv * A[i] * B[j] * C[k])))
            ref.append(v)
    got, ref = np.array(got), np.array(ref)
    return {"sweeps": g["sweeps"], "wall_s_incl_graph_capture": round(dt, 3), "fit_fp8": round(fit, 7),
            "fit_oracle_fp64": round(g["fit"], 7), "fit_abs_diff": float(f"{abs(fit - g['fit']):.3e}"),
            "model_rel_err_at_samples": float(f"{np.linalg.norm(got - ref) / np.linalg.norm(ref):.3e}")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cp1024_r64")
    ap.add_argument("--prec", default=None)
    ap.add_argument("--compare", default=None,
                    help="paths timed beside the headline, comma-separated (default fp32, plus bf16x6 when the "
                         "headline is bf16x3; none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode-reps", type=int, default=20)
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--budget", type=float, default=200e9)
    ap.add_argument("--sat-requests", type=int, default=600)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the multi-GPU sharding is a design "
                                   "note (slabs of mode-1 slices, one all-reduce per mode for modes 2 and 3)"}))
        sys.exit(2)

    if args.workload == "serve":
        serve_bench(args)
        return
    if args.workload == "copy":
        copy_bench(args)
        return
    if args.workload in SPARSE_WORKLOADS:
        sparse_bench(args)
        return
    if args.workload in NWAY_WORKLOADS:
        nway_bench(args)
        return

    import torch
    from paper_2411_04785_amd import synth
    from paper_2411_04785_amd.mttkrp import Context

    w = synth.WORKLOADS[args.workload]
    prec = args.prec or DEFAULT_PREC[w.name]
    if args.compare is None:
        compares = ["fp32", "bf16x6"] if prec == "bf16x3" else ["fp32"]
    else:
        compares = [c for c in args.compare.split(",") if c and c != "none"]
    compares = [c for c in compares if c != prec]
    compare = ",".join(compares) or None
    I, J, K = w.dims
    R = w.R
    log(f"[bench] workload {w.name} dims={w.dims} R={R} prec={prec} compare={compare}: generating input")
    t0 = time.perf_counter()
    X = synth.tensor(w)
    facs = synth.init_factors(w)
    log(f"[bench] generated in {time.perf_counter() - t0:.1f} s; uploading")

    dev = torch.device("cuda:0")
    # All library calls and the timing events go to one dedicated stream (a
    # caller's own stream, as a user of the library would pass it), not the
    # legacy default stream.
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    ctx = Context(0)
    Xd = torch.from_numpy(X).to(dev)
    f0 = [torch.from_numpy(f).to(dev) for f in facs]
    runs = {}
    kw = {}
    X_head = Xd
    if prec == "fp8":
        q, slice_exp, Xt = ctx.quantize_fp8(Xd, transposed=True)
        torch.cuda.synchronize()
        X_head, kw = q, {"slice_exp": slice_exp, "X_t": Xt}
    runs[prec] = run_path(ctx, torch, stream, w, prec, X_head, kw, f0, args)
    name, k_ms, k_bytes = dominant_kernel(ctx, torch, stream, w, prec, X_head, kw, f0, runs[prec]["mode_ms"],
                                          args.mode_reps)
    log(f"[bench] dominant kernel: {name}: {k_ms * 1e3:.1f} us")
    fp8_als = None
    if prec == "fp8" and w.als_sweeps:
        fp8_als = fp8_als_vs_oracle(ctx, torch, w, X_head, kw, Xd, f0)
        log(f"[bench] FP8 CP-ALS vs oracle: {fp8_als}")
    for cp in compares:
        runs[cp] = run_path(ctx, torch, stream, w, cp, Xd, {}, f0, args)
    fit = ctx.fit(X_head, runs[prec]["factors"], runs[prec]["lam"], **kw)

    flop_mttkrp = 2.0 * I * J * K * R
    head = runs[prec]
    value = 3 * flop_mttkrp / (head["ms_step"] * 1e-3) / 1e9
    tree = Context.sweep_uses_dimtree(w.dims, R, prec)
    # Flops a sweep executes: with the tree, the Y contraction (2IJKR), the two
    # sums over Y (2 x 2IJR) and the mode-3 contraction (2IJKR); else 3 x 2IJKR.
    exec_flop = (2 * flop_mttkrp + 2 * 2.0 * I * J * R) if tree else 3 * flop_mttkrp
    roof = roofline(name, k_ms, k_bytes, flop_mttkrp, prec)
    roof["traffic"] = recorded_traffic(w.name, prec, name)

    cpu, refs = None, None
    if not args.no_cpu_baseline:
        log("[bench] FP64 oracle on the host (references for the per-mode errors, then the timed sample)")
        cpu, refs = cpu_baseline(X, facs)

    detail = {"sweep_passes_over_X": 2 if tree else 3,
              "executed_gflop_per_sweep": round(exec_flop / 1e9, 2),
              "executed_gflops": round(exec_flop / (head["ms_step"] * 1e-3) / 1e9, 1),
              "fit_after": round(fit, 7)}
    for p, r in runs.items():
        bytes_modes = [algorithmic_bytes(w.dims, R, m, p) for m in range(3)]
        d = {"ms_per_sweep": round(r["ms_step"], 4),
             "mttkrp_us": [round(t * 1e3, 2) for t in r["mode_ms"]],
             "mttkrp_gflops": [round(flop_mttkrp / (t * 1e-3) / 1e9, 1) for t in r["mode_ms"]],
             "mttkrp_gbs": [round(b / (t * 1e-3) / 1e9, 1) for b, t in zip(bytes_modes, r["mode_ms"])],
             "mttkrp_roofline": [{k: v for k, v in roofline("", t, b, flop_mttkrp, p).items()
                                  if k in ("bound", "frac")} for b, t in zip(bytes_modes, r["mode_ms"])]}
        if refs is not None:
            d["err_rel_per_mode_all_rows"], d["err_rel_worst_row"] = err_rows(r["outs"], refs)
        detail[p] = d
    for cp in compares:
        detail["sweep_speedup_vs_" + cp] = round(runs[cp]["ms_step"] / head["ms_step"], 3)
        detail["mttkrp_speedup_vs_" + cp] = [round(a / b, 3) for a, b in zip(runs[cp]["mode_ms"], head["mode_ms"])]
    if fp8_als is not None:
        detail["fp8_als_vs_oracle"] = fp8_als
    if cpu is not None:
        detail["oracle_full_mode_s"] = cpu.pop("all_modes_s")

    dtype = {"fp32": "f32", "bf16x3": "bf16x3", "bf16x6": "bf16x6", "fp8": "e4m3"}[prec]
    line = {
        "metric": "MTTKRP GFLOP/s (algorithmic, 3 x 2IJKR per CP-ALS sweep) and % roofline vs plain FP32 at stated err",
        "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(head["ms_step"], 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": f"{w.name}: {I}x{J}x{K} rank-{w.rank_true} CP + N(0,{w.noise_var:g}) noise"
                               + (" per-slice magnitudes 10^U(-3,3)" if w.slice_log10 else "")
                               + f", R={R}, {prec}" + (f" timed beside {compare}" if compare else "")
                               + ", step = one CP-ALS sweep",
                   "dims": list(w.dims), "R": R, "prec": prec, "compare": compare},
        "roofline": roof,
        "cpu_baseline": cpu,
        "detail": detail,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
