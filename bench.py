"""Benchmark: time to a 1e-8 relative normal-equation residual on the dense
kernel workload (the largest single-GPU configuration), with the product
kernel against the HBM roofline; the sparse, adjoint and batched workloads
beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
                    [--no-extensions] [--max-rank L] [--products-only]

Headline (value): A = exp(-||p_i - p_j||^2 / 2) on 40000 points uniform in
[0,1]^8, 40000 x 40000 FP32 (6.4 GB), 16 right-hand sides N(0,1), mu = 1e-3,
block 250 (sketch dimension 275).  One step is one whole APLICUR solve
(sketch, adaptive CUR, preconditioner builds, LSQR phases with the 16
columns blocked on FP64-accumulated MFMA products, FP64 eta checks) to eta
<= 1e-8 for every column, with A and B already resident in HBM; step t uses
sketch seed 10 + 100 (t mod 5), and the line reports the median and range
over the steps.  roofline: the blocked product kernel (A X and A^T U, 16
columns), every launch of the timed steps timed by events on its own
dispatch.  Beside it, on the same problem:
FP32 phases, BF16 products, plain LSQR.  Then the sparse workload (CSR
200000 x 20000: product bandwidth warm and cold, APLICUR and plain LSQR), the
adjoint workload (dense FP32 100000 x 2000, 32 RHS: forward, backward, plain
LSQR) and the batched workload (64 uneven problems, 8 RHS: one batched
call, one at a time, plain LSQR on the first 8).  The CPU baseline is the
FP64 oracle on a bounded sample of the headline recipe.  One JSON line on
stdout; progress on stderr.

--products-only runs just the timed sparse A / A^T product loop and a 256
MiB copy of known size (for hardware-counter runs); --blocked-products does
the same for the blocked products of several right-hand sides (dense FP32
A).
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "time to 1e-8 rel. NE residual & A/A^T matvec GB/s; batched+adjoint vs plain"
KERNEL_SRC = os.path.join(ROOT, "paper_2604_05065_amd", "csrc", "kern_gk.hip")
BLK_SRC = os.path.join(ROOT, "paper_2604_05065_amd", "csrc", "kern_blk.hip")
COUNTERS = os.path.join(ROOT, "profiles", "spmv_csr_200000x20000_counters.txt")
BLK_COUNTERS = os.path.join(ROOT, "profiles", "blocked_products_rbf40000_k16_counters.txt")
PRODUCT_REPS = 200
FP64_PEAK_TFS = 78.6
# the dense kernel workload: RBF kernel on 40000 points in [0,1]^8, FP32, 16 RHS
NPTS, NRHS, MU3, BLOCK3, TOL3 = 40000, 16, 1e-3, 250, 1e-8
SEEDS3 = [10 + 100 * t for t in range(5)]  # sketch seeds 7 + 3 + 100 t: five trials


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmv_bytes(rows, cols, nnz, vbytes=8):
    """Algorithmic bytes of one CSR product y = A x - y_prev (the product
    kernel with its epilogue): values and column indices once, row pointers
    once, x once, y read and written."""
    return nnz * (vbytes + 4) + (rows + 1) * 4 + cols * 8 + 2 * rows * 8


def kernel_hash(path=KERNEL_SRC):
    with open(path, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()[:12]


def counter_traffic(path=COUNTERS, src=KERNEL_SRC, key="traffic_bytes_per_launch_A"):
    """HBM bytes per launch of a product kernel from a committed counter
    summary (FETCH_SIZE + WRITE_SIZE scaled by the copy-kernel calibration),
    or None when it is missing or was taken on other kernel source."""
    try:
        txt = open(path).read()
    except OSError:
        return None
    h = re.search(r"^kernel_source_sha1:\s*(\S+)", txt, re.M)
    t = re.search(r"^" + key + r":\s*([0-9.eE+]+)", txt, re.M)
    if not h or not t or h.group(1) != kernel_hash(src):
        return None
    return float(t.group(1))


def cpu_baseline_dense_kernel(npts=5000, budget_s=30.0):
    """The FP64 oracle (NumPy/SciPy APLICUR, Alg. 3) timed to eta <= 1e-8 on
    a bounded sample of the dense kernel workload: the same RBF kernel recipe
    on npts points (CPU generator), one right-hand side, mu = 1e-3, block 250,
    sketch seed 10, on the host cores (BLAS threads as the pool runs them)."""
    import numpy as np
    from oracle.aplicur import Options, aplicur, ne_residual
    from workloads import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(p.get("num_threads", 1)) for p in threadpool_info()] or [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    A = synth.rbf_kernel(np.random.default_rng(3002), npts).astype(np.float64)
    b = np.random.default_rng(3001).standard_normal(npts)
    t0 = time.perf_counter()
    x = aplicur(A, b, MU3, Options(block=BLOCK3, tol_ne=TOL3, seed=SEEDS3[0]))
    ms = (time.perf_counter() - t0) * 1e3
    eta = ne_residual(A, b, x, MU3)
    return {"value": round(ms, 1), "unit": "ms", "cores": threads, "kind": "oracle",
            "sample": (f"oracle APLICUR (FP64, NumPy/SciPy) to eta <= 1e-8 (reached {eta:.1e}) on the RBF kernel "
                       f"recipe at {npts} points (one right-hand side, mu = 1e-3, block 250), not the 40000-point, "
                       f"16-column workload of value; {threads} BLAS threads of "
                       f"{len(os.sched_getaffinity(0))} host cores")}


def _timed(torch, fn):
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) * 1e3, out


def bench_headline(ap, synth, torch, args):
    """The dense kernel workload at full size: A = exp(-||p_i - p_j||^2 / 2) on
    40000 points uniform in [0,1]^8 (FP32, 6.4 GB), 16 right-hand sides N(0,1),
    mu = 1e-3, block 250, every column to eta <= 1e-8; the 16 columns run
    blocked (FP64-accumulated MFMA products).  One step is one whole solve
    (context creation with the sketch, CUR increments, preconditioner builds,
    LSQR phases, FP64 eta checks); step t uses sketch seed SEEDS3[t mod 5].
    The contexts carve their device memory from one caller workspace
    allocated before the warm-up; one more solve with library-allocated
    memory is reported beside them.
    Beside it: the blocked product kernel, timed by events on each of its
    dispatches in the timed steps and alone (20 launches back to back), the
    same solve with FP32 and BF16 phases, and plain LSQR on the same problem
    (iteration budget 2000)."""
    A, B = synth.rbf_kernel_gpu(3003, NPTS, NRHS)
    opts = dict(mu=MU3, block=BLOCK3, tol_ne=TOL3)
    log(f"[bench] dense kernel workload {NPTS}^2 FP32 x {NRHS} generated")
    # the contexts of value's steps take their device memory from one caller
    # workspace, allocated here once (the largest need over the five sketch
    # seeds), as a serving loop would keep it resident
    ws_bytes = max(ap.workspace_bytes(A, NRHS, seed=s, **opts) for s in SEEDS3)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    log(f"[bench] caller workspace {ws_bytes / 2**30:.2f} GiB")

    def solve_ws(seed):
        def run():
            with ap.Context(A, workspace=ws, seed=seed, **opts) as ctx:
                return ctx.solve(B)
        return _timed(torch, run)

    def solve(seed, **kw):
        return _timed(torch, lambda: ap.lstsq(A, B, seed=seed, **opts, **kw))

    # event timing of the product kernel on its own dispatches, on during the
    # warm-up (which creates the events) and the timed steps
    ap.prof_products(True)
    for i in range(args.warmup):
        ms, (_, info) = solve_ws(SEEDS3[0])
        log(f"[bench] warmup {i}: {ms:.1f} ms rank={info.rank} iters={info.iters} eta={info.eta:.2e}")
    ap.prof_read()
    times, infos = [], []
    torch.cuda.synchronize()
    for t in range(args.steps):
        seed = SEEDS3[t % len(SEEDS3)]
        ms, (_, info) = solve_ws(seed)
        times.append(ms)
        infos.append(info)
        log(f"[bench] step {t} (seed {seed}): {ms:.1f} ms rank={info.rank} phases={info.phases} iters={info.iters} "
            f"eta={info.eta:.2e} (sketch {info.t_sketch_ms:.1f}, cur {info.t_cur_ms:.1f}, "
            f"precond {info.t_precond_ms:.1f}, lsqr {info.t_lsqr_ms:.1f} ms)")
        if info.status != 0 or info.eta > TOL3:
            log(f"[bench] WARNING: step {t} did not reach eta <= {TOL3:g} (status {info.status})")
    prof = ap.prof_read()
    ap.prof_products(False)
    # the same solve with library-allocated memory (hipMalloc / hipFree of
    # the context's buffers inside the solve), for reference
    ms_libmem = float("nan")
    if not args.headline_only:
        ms_libmem, (_, info_lm) = solve(SEEDS3[1 % len(SEEDS3)])
        log(f"[bench] seed {SEEDS3[1 % len(SEEDS3)]} with library memory: {ms_libmem:.1f} ms (eta {info_lm.eta:.2e})")
    ms_step = sum(times) / len(times)
    srt = sorted(times)
    med = srt[len(srt) // 2] if len(srt) % 2 else 0.5 * (srt[len(srt) // 2 - 1] + srt[len(srt) // 2])
    info = infos[-1]
    # the product kernel inside the timed steps: A X and A^T U (16 columns, FP64
    # accumulation), each launch timed by events on its own dispatch
    n_ax, us_ax_live, _ = prof.get("AX_f64", (0, float("nan"), 0))
    n_atu, us_atu_live, _ = prof.get("ATX_f64", (0, float("nan"), 0))
    untimed = sum(v[2] for v in prof.values())
    us_live = (n_ax * us_ax_live + n_atu * us_atu_live) / max(1, n_ax + n_atu)
    bytes_prod = 4 * NPTS * NPTS + 2 * NPTS * NRHS * 8  # A (or its transposed copy) once in FP32, X read, Y written
    flops_prod = 2.0 * NPTS * NPTS * NRHS
    gbs = bytes_prod / (us_live * 1e-6) / 1e9
    log(f"[bench] product kernel in the timed steps: {n_ax} A X launches {us_ax_live:.0f} us, {n_atu} A^T U "
        f"launches {us_atu_live:.0f} us (untimed {untimed}); mean {us_live:.0f} us = {gbs:.0f} GB/s, "
        f"{flops_prod / us_live / 1e6:.1f} TFLOP/s")
    # the same kernel alone, 20 launches back to back
    us_ax = us_atu = float("nan")
    if not args.headline_only:
        with ap.Context(A, precond=False, **opts) as ctx:
            X = torch.randn(NPTS, NRHS, device="cuda", dtype=torch.float64)
            us_ax = ctx.time_matmat(X, trans=False, reps=20)
            us_atu = ctx.time_matmat(X, trans=True, reps=20)
        log(f"[bench] product kernel alone (20 back to back): A X {us_ax:.0f} us, A^T U {us_atu:.0f} us")
    compare = {}
    for name, kw in (() if args.headline_only else
                     (("aplicur_fp32_phases", dict(precision=1)), ("aplicur_bf16_products", dict(precision=2)),
                      ("plain_lsqr", dict(precond=False, max_iter=2000)))):
        if name != "plain_lsqr":
            solve(SEEDS3[0], **kw)  # warm-up of the mode (its copies of A)
        ms, (_, inf) = solve(SEEDS3[0], **kw)
        compare[name] = {"ms": round(ms, 1), "iters": inf.iters, "phases": inf.phases, "eta": inf.eta,
                         "status": inf.status, "rank": inf.rank,
                         "reached": bool(inf.status == 0 and inf.eta <= TOL3)}
        log(f"[bench] {name}: {ms:.0f} ms iters={inf.iters} phases={inf.phases} eta={inf.eta:.2e} "
            f"status={inf.status}")
    del A, B
    traffic = counter_traffic(BLK_COUNTERS, BLK_SRC, "traffic_bytes_per_launch_AX")
    return {
        "ms_per_step": round(ms_step, 3),
        "config": {"workload": (f"APLICUR solve of the dense RBF kernel workload to eta<=1e-8 per column: "
                                f"A = exp(-|p_i-p_j|^2/2), {NPTS} points in [0,1]^8, {NPTS}x{NPTS} FP32, "
                                f"{NRHS} right-hand sides, mu={MU3:g}, block {BLOCK3}, columns blocked on "
                                f"FP64-accumulated MFMA products"),
                   "npts": NPTS, "nrhs": NRHS, "mu": MU3, "block": BLOCK3, "tol_ne": TOL3,
                   "sketch_seeds": SEEDS3},
        "seeds": {"median_ms": round(med, 1), "min_ms": round(srt[0], 1), "max_ms": round(srt[-1], 1),
                  "per_step_ms": [round(t, 1) for t in times]},
        "memory": {"caller_workspace_bytes": int(ws_bytes),
                   "library_memory_ms": None if args.headline_only else
                   {"seed": SEEDS3[1 % len(SEEDS3)], "ms": round(ms_libmem, 1)}},
        "aplicur": {"rank": info.rank, "phases": info.phases, "iters": info.iters, "outer": info.outer,
                    "rebuilds": info.rebuilds, "eta": max(i.eta for i in infos),
                    "all_reached": all(i.status == 0 and i.eta <= TOL3 for i in infos),
                    "t_sketch_ms": round(info.t_sketch_ms, 2), "t_cur_ms": round(info.t_cur_ms, 2),
                    "t_precond_ms": round(info.t_precond_ms, 2), "t_lsqr_ms": round(info.t_lsqr_ms, 2)},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": ("k_rows_gemm_xl (A X and A^T U for 16 columns, FP32 A widened, FP64 16x16x4 "
                                "MFMA, X staged in LDS per workgroup), launches of the timed steps"),
                     "launches": n_ax + n_atu, "bytes_per_launch": int(bytes_prod),
                     "us_per_launch": round(us_live, 3),
                     "mfma_tflops": round(flops_prod / us_live / 1e6, 2),
                     "mfma_frac_fp64": round(flops_prod / us_live / 1e6 / FP64_PEAK_TFS, 4)},
        "products": {"timed_steps": {"AX_launches": n_ax, "AX_us": round(us_ax_live, 1), "ATU_launches": n_atu,
                                     "ATU_us": round(us_atu_live, 1), "untimed": untimed},
                     "alone_back_to_back": None if args.headline_only else {
                         "AX_us": round(us_ax, 1), "ATU_us": round(us_atu, 1),
                         "AX_GBs": round(bytes_prod / (us_ax * 1e-6) / 1e9, 1),
                         "ATU_GBs": round(bytes_prod / (us_atu * 1e-6) / 1e9, 1)}},
        "compare": compare,
    }


def bench_c2(ap, synth, torch, args):
    """The sparse workload (CSR 200000 x 20000, 10 random columns per row,
    column scaling 1e-6, mu = 1e-4, block 100, rank cap args.max_rank): the A
    and A^T product kernels (warm, and cold with 1 GiB read and written before
    each timed launch), a measured device copy, and APLICUR against plain
    LSQR to eta <= 1e-8 (FP64)."""
    t0 = time.time()
    w = synth.workload(2, 1.0)
    A, b, mu, block, tol = w.A, w.B, w.mu, w.block, w.tol
    m, n = A.shape
    nnz = int(A.nnz)
    log(f"[bench] sparse workload {m}x{n} nnz={nnz} generated in {time.time() - t0:.1f}s")
    Ag = ap.CSRMatrix.from_scipy(A, device="cuda", dtype=torch.float64)
    bg = torch.as_tensor(b, device="cuda")
    with ap.Context(Ag, precond=False, mu=mu) as ctx:
        xv = torch.randn(n, device="cuda", dtype=torch.float64)
        ctx.time_product(xv, trans=False, reps=10)
        us_a = ctx.time_product(xv, trans=False, reps=PRODUCT_REPS)
        us_at = ctx.time_product(xv, trans=True, reps=PRODUCT_REPS)
        us_a_cold = us_at_cold = float("nan")
        if not args.products_only:
            flush = torch.zeros(1 << 28, dtype=torch.int32, device="cuda")
            us_a_cold = ctx.time_product(xv, trans=False, reps=20, flush=flush)
            us_at_cold = ctx.time_product(xv, trans=True, reps=20, flush=flush)
            del flush
    bytes_a = spmv_bytes(m, n, nnz)
    bytes_at = spmv_bytes(n, m, nnz) - n * 8  # the A^T kernel stores its output without reading it
    if args.products_only:
        big = torch.empty(32 << 20, dtype=torch.float64, device="cuda")  # 256 MiB
        dst = torch.empty_like(big)
        for _ in range(3):
            dst.copy_(big)
        torch.cuda.synchronize()
        print(json.dumps({"us_A": us_a, "us_AT": us_at, "bytes_A": bytes_a, "bytes_AT": bytes_at,
                          "copy_bytes_each_way": big.numel() * 8}), flush=True)
        return None
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    gbs = lambda b_, us: b_ / (us * 1e-6) / 1e9  # noqa: E731
    log(f"[bench] CSR A x: {us_a:.2f} us ({gbs(bytes_a, us_a):.0f} GB/s), cold {us_a_cold:.2f} us "
        f"({gbs(bytes_a, us_a_cold):.0f} GB/s); A^T u: {us_at:.2f} us ({gbs(bytes_at, us_at):.0f} GB/s), cold "
        f"{us_at_cold:.2f} us ({gbs(bytes_at, us_at_cold):.0f} GB/s); device copy {copy_gbs:.0f} GB/s")
    res = {}
    for name, pc, prec in (("aplicur_f64", True, 0), ("plain_lsqr_f64", False, 0), ("aplicur_f32_phases", True, 1),
                           ("plain_lsqr_f32_phases", False, 1)):
        o = dict(mu=mu, block=block, tol_ne=tol, seed=7, max_rank=args.max_rank, precond=pc, precision=prec)
        ap.lstsq(Ag, bg, **o)  # warm-up
        ms, (_, inf) = _timed(torch, lambda: ap.lstsq(Ag, bg, **o))
        res[name] = {"ms": round(ms, 1), "iters": inf.iters, "phases": inf.phases, "eta": inf.eta,
                     "rank": inf.rank, "us_per_iter": round(inf.t_lsqr_ms * 1e3 / max(inf.iters, 1), 2)}
        log(f"[bench] CSR {name}: {ms:.0f} ms iters={inf.iters} eta={inf.eta:.2e} rank={inf.rank}")
    return {"m": m, "n": n, "nnz": nnz, "mu": mu, "block": block, "max_rank": args.max_rank,
            "A_us": round(us_a, 3), "A_GBs": round(gbs(bytes_a, us_a), 1),
            "AT_us": round(us_at, 3), "AT_GBs": round(gbs(bytes_at, us_at), 1),
            "A_us_cold": round(us_a_cold, 3), "A_GBs_cold": round(gbs(bytes_a, us_a_cold), 1),
            "A_frac_cold": round(gbs(bytes_a, us_a_cold) / HBM_PEAK_GBS, 4),
            "AT_us_cold": round(us_at_cold, 3), "AT_GBs_cold": round(gbs(bytes_at, us_at_cold), 1),
            "AT_frac_cold": round(gbs(bytes_at, us_at_cold) / HBM_PEAK_GBS, 4),
            "A_bytes": int(bytes_a), "AT_bytes": int(bytes_at), "A_traffic": counter_traffic(),
            "copy_GBs": round(copy_gbs, 1), "solves": res}


def bench_batched(ap, synth, torch, count=16, scale=0.25, nrhs=2, plain_subset=None):
    """The batched workload (count problems, m ~ U{5000..100000} scale, n ~
    U{500..min(5000, m/4)} scale, sigma_i = 10^(-k i/n), k ~ U[2,8], FP32,
    nrhs RHS, mu = 1e-6, block 50): one batched call (worker streams, graph
    replay, tuned tiles) against one-at-a-time APLICUR and one-at-a-time
    plain LSQR (on the first plain_subset problems when given)."""
    shapes = synth.batch_shapes(count, m_range=(int(5000 * scale), int(100000 * scale)),
                                n_range=(int(500 * scale), int(5000 * scale)))
    probs = []
    for i, (m, n, k) in enumerate(shapes):
        probs.append(synth.dense_svd_gpu(4000 + i, m, n, k, nrhs))
        if (i + 1) % 16 == 0:
            log(f"[bench] batched: {i + 1} of {count} problems generated")
    opts = dict(mu=1e-6, block=50, tol_ne=1e-8)
    As, Bs = [p[0] for p in probs], [p[1] for p in probs]

    def one_at_a_time(limit=None, **kw):
        out = []
        for i, (A, B) in enumerate(zip(As[:limit], Bs[:limit])):
            out.append(ap.lstsq(A, B, **opts, **kw)[1])
            if (i + 1) % 8 == 0:
                log(f"[bench] batched: {i + 1} one-at-a-time solves ({kw or 'APLICUR'})")
        return out
    ap.solve_batched(As[:2], Bs[:2], workers=2, **opts)  # warm-up
    ms_b, (_, infos) = _timed(torch, lambda: ap.solve_batched(As, Bs, workers=8, **opts))
    log(f"[bench] batched: one call {ms_b:.0f} ms")
    ms_s, inf_s = _timed(torch, lambda: one_at_a_time())
    sub = plain_subset or count
    ms_p, inf_p = _timed(torch, lambda: one_at_a_time(limit=sub, precond=False))
    ms_ps, inf_ps = _timed(torch, lambda: one_at_a_time(limit=sub))  # APLICUR on the same subset
    ok = all(i.status == 0 for i in list(infos) + inf_s + inf_p)
    log(f"[bench] batched {count} problems: batched {ms_b:.0f} ms, one-at-a-time APLICUR {ms_s:.0f} ms; "
        f"first {sub}: plain LSQR {ms_p:.0f} ms, APLICUR {ms_ps:.0f} ms (all converged: {ok})")
    return {"problems": count, "nrhs": nrhs, "sum_mn": int(sum(m * n for m, n, _ in shapes)),
            "batched_ms": round(ms_b, 1), "sequential_aplicur_ms": round(ms_s, 1),
            "plain_subset": sub, "sequential_plain_subset_ms": round(ms_p, 1),
            "sequential_aplicur_subset_ms": round(ms_ps, 1), "workers": 8, "all_converged": ok,
            "max_eta": max(i.eta for i in list(infos) + inf_s + inf_p),
            "max_iters_aplicur": max(i.iters for i in inf_s), "max_iters_plain": max(i.iters for i in inf_p)}


def bench_adjoint(ap, synth, torch, m=25000, n=500, nrhs=4):
    """The adjoint workload at 1/4 of its sizes (dense FP32 25000 x 500,
    sigma_i = 10^(-5 i/n), 4 RHS, mu = 1e-5, block 100; L = sum X^2): forward
    APLICUR, backward with the final preconditioner, and the same backward
    with plain LSQR (no preconditioner)."""
    A, B = synth.dense_svd_gpu(5000, m, n, 5.0, nrhs)
    opts = dict(mu=1e-5, block=100, tol_ne=1e-8)
    with ap.Context(A, **opts) as ctx:
        ms_f, (X, info) = _timed(torch, lambda: ctx.solve(B))
        ms_b, (Z, dB, dA, binfo) = _timed(torch, lambda: ctx.solve_backward(X, B, 2.0 * X))
    with ap.Context(A, precond=False, **opts) as ctx:
        ms_pf, (X0, pfinfo) = _timed(torch, lambda: ctx.solve(B))
        ms_p, (_, _, _, pinfo) = _timed(torch, lambda: ctx.solve_backward(X0, B, 2.0 * X0))
    log(f"[bench] adjoint {m}x{n}: forward {ms_f:.0f} ms (eta {info.eta:.1e}), backward {ms_b:.0f} ms "
        f"(eta {binfo.eta:.1e}, {binfo.iters} it); plain LSQR forward {ms_pf:.0f} ms ({pfinfo.iters} it), "
        f"plain backward {ms_p:.0f} ms ({pinfo.iters} it)")
    return {"m": m, "n": n, "nrhs": nrhs, "forward_ms": round(ms_f, 1), "forward_eta": info.eta,
            "backward_ms": round(ms_b, 1), "backward_eta": binfo.eta, "backward_iters": binfo.iters,
            "plain_forward_ms": round(ms_pf, 1), "plain_forward_iters": pfinfo.iters,
            "plain_forward_eta": pfinfo.eta, "plain_backward_ms": round(ms_p, 1),
            "plain_backward_iters": pinfo.iters, "rank": info.rank}


def bench_multi_rhs(ap, synth, torch, npts=20000, nrhs=16):
    """The dense kernel workload at half its size (Gaussian RBF kernel, h = 1,
    on 20000 points in [0,1]^8, FP32 A, 16 RHS, mu = 1e-3, block 250): APLICUR
    with the 16 columns blocked (one pass over A per iteration for all; FP64,
    FP32 phases with FP64 refinement, and those with BF16 products) against
    the same solve one column at a time, and the blocked product bandwidth (A X
    and A^T U with 16 columns, event-timed whole matmat calls, bytes of the
    matrix read: FP32 A for the FP64 and FP32 products, its BF16 copy for the
    BF16 ones)."""
    A, B = synth.rbf_kernel_gpu(3003, npts, nrhs)
    opts = dict(mu=1e-3, block=250, tol_ne=1e-8)
    out = {"npts": npts, "nrhs": nrhs}
    for name, cols, prec in (("columns", 1, 0), ("blocked", 0, 0), ("blocked_fp32_ir", 0, 1),
                             ("blocked_bf16_ir", 0, 2)):
        ms, (X, info) = _timed(torch, lambda: ap.lstsq(A, B, columns=cols, precision=prec, **opts))
        out[name] = {"ms": round(ms, 1), "lsqr_ms": round(info.t_lsqr_ms, 1), "iters": info.iters,
                     "phases": info.phases, "rank": info.rank, "eta": info.eta}
        if prec == 2:
            out[name]["phases_bf16"] = info.phases_bf16
        log(f"[bench] multi-RHS rbf {npts} x {nrhs} ({name}): {ms:.0f} ms (LSQR {info.t_lsqr_ms:.0f} ms, "
            f"rank {info.rank}, {info.iters} it, eta {info.eta:.1e})")
    with ap.Context(A, precond=False, precision=2, **opts) as ctx:
        X = torch.randn(npts, nrhs, device="cuda", dtype=torch.float64)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for prec, tag, esize in ((0, "", 4), (1, "_fp32", 4), (2, "_bf16", 2)):
            for trans, key in ((False, "AX"), (True, "ATU")):
                ctx.matmat(X, trans=trans, prec=prec)
                best = 1e30
                for _ in range(5):
                    e0.record()
                    ctx.matmat(X, trans=trans, prec=prec)
                    e1.record()
                    torch.cuda.synchronize()
                    best = min(best, e0.elapsed_time(e1))
                gbs = A.numel() * esize / best / 1e6
                out[key + tag + "_ms"], out[key + tag + "_GBs"] = round(best, 3), round(gbs, 1)
                log(f"[bench] blocked product {key} prec {prec} ({nrhs} columns, RBF {npts}^2): {best:.3f} ms, "
                    f"{gbs:.0f} GB/s")
    return out


def blocked_products(ap, synth, torch, npts=20000, nrhs=16, rounds=20, prec=0):
    """The blocked products alone (A X and A^T U, 16 columns, FP32 RBF kernel
    on npts points; prec 0: FP64 accumulation, 1: FP32 products, 2: BF16
    products) alternating for `rounds` rounds after a warm-up, event timed,
    then three copies of 256 MiB used to calibrate the hardware counters.
    One JSON line; bytes_A is the matrix as the kernel reads it (FP32, or the
    padded BF16 copy)."""
    A, _ = synth.rbf_kernel_gpu(3003, npts, nrhs)
    with ap.Context(A, precond=False, mu=1e-3, precision=prec) as ctx:
        X = torch.randn(npts, nrhs, device="cuda", dtype=torch.float64)
        ctx.matmat(X, prec=prec)
        ctx.matmat(X, trans=True, prec=prec)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ta = tt = 0.0
        for _ in range(rounds):
            e[0].record()
            ctx.matmat(X, prec=prec)
            e[1].record()
            ctx.matmat(X, trans=True, prec=prec)
            e[2].record()
            torch.cuda.synchronize()
            ta += e[0].elapsed_time(e[1])
            tt += e[1].elapsed_time(e[2])
    big = torch.empty(32 << 20, dtype=torch.float64, device="cuda")  # 256 MiB
    dst = torch.empty_like(big)
    for _ in range(3):
        dst.copy_(big)
    torch.cuda.synchronize()
    bytes_a = A.numel() * A.element_size()
    if prec == 2:
        bytes_a = ((npts + 31) // 32 * 32) * ((npts + 63) // 64 * 64) * 2
    print(json.dumps({"ms_AX": ta / rounds, "ms_ATU": tt / rounds, "bytes_A": bytes_a, "nrhs": nrhs, "prec": prec,
                      "GBs_AX": bytes_a / (ta / rounds) / 1e6, "GBs_ATU": bytes_a / (tt / rounds) / 1e6,
                      "copy_bytes_each_way": big.numel() * 8}), flush=True)


def sketch_study(ap, synth, torch):
    """Sparse sign against Gaussian sketch: set-up time of the sketch and the
    whole solve with each, on the dense kernel workload at half size (FP32 A,
    16 RHS) and on the sparse workload (CSR 200000 x 20000, rank cap 256);
    and the error of the Gaussian sketch of FP32 A (FP32 GEMM) against the
    same sketch of the values widened to FP64 (FP64 GEMM).  One JSON line."""
    out = {}
    A, B = synth.rbf_kernel_gpu(3003, 20000, 16)
    opts = dict(mu=1e-3, block=250, tol_ne=1e-8)
    dense = {}
    for kind in ("sparse", "gaussian"):
        ap.lstsq(A, B, sketch=kind, **opts)  # warm-up (library and rocBLAS initialisation)
        ms, (X, info) = _timed(torch, lambda: ap.lstsq(A, B, sketch=kind, **opts))
        dense[kind] = {"ms": round(ms, 1), "t_sketch_ms": round(info.t_sketch_ms, 2), "rank": info.rank,
                       "iters": info.iters, "eta": info.eta}
        log(f"[bench] sketch study rbf 20000 ({kind}): {ms:.0f} ms (sketch {info.t_sketch_ms:.1f} ms), "
            f"rank {info.rank}, {info.iters} it")
    with ap.Context(A, sketch="gaussian", max_outer=1, **opts) as c32:
        s = c32.sizes()["s"]
        y32 = torch.as_tensor(c32.query(1)).reshape(s, -1)
    A64 = A.to(torch.float64)
    with ap.Context(A64, sketch="gaussian", max_outer=1, **opts) as c64:
        y64 = torch.as_tensor(c64.query(1)).reshape(s, -1)
    del A64
    err = (y32 - y64).abs()
    dense["gaussian_fp32_vs_fp64"] = {"max_abs_err_over_max_abs": float(err.max() / y64.abs().max()),
                                      "rel_frobenius": float(err.norm() / y64.norm())}
    log(f"[bench] Gaussian sketch of FP32 A, FP32 GEMM vs FP64 GEMM: {dense['gaussian_fp32_vs_fp64']}")
    out["rbf20000"] = dense
    del A, B
    torch.cuda.empty_cache()
    w = synth.workload(2, 1.0)
    Ag = ap.CSRMatrix.from_scipy(w.A, device="cuda", dtype=torch.float64)
    bg = torch.as_tensor(w.B, device="cuda")
    sparse = {}
    for kind in ("sparse", "gaussian"):
        ap.lstsq(Ag, bg, mu=w.mu, block=w.block, tol_ne=w.tol, max_rank=256, sketch=kind)  # warm-up
        ms, (x, info) = _timed(torch, lambda: ap.lstsq(Ag, bg, mu=w.mu, block=w.block, tol_ne=w.tol, max_rank=256,
                                                      sketch=kind))
        sparse[kind] = {"ms": round(ms, 1), "t_sketch_ms": round(info.t_sketch_ms, 2), "rank": info.rank,
                        "iters": info.iters, "eta": info.eta}
        log(f"[bench] sketch study CSR 200000x20000 ({kind}): {ms:.0f} ms (sketch {info.t_sketch_ms:.1f} ms), "
            f"{info.iters} it")
    out["csr200000"] = sparse
    print(json.dumps({"sketch_study": out}), flush=True)


def paper_workloads(ap, synth, torch, tol=1e-8, budget=30000):
    """The paper's own test sets (Sec. 6.3, the experiments of Secs. 7-8 without
    the comparison systems): APLICUR against plain LSQR, both FP64 on the GPU,
    time to eta <= tol (iteration budget `budget` each), block b = n/50.  Dense
    incoherent / coherent U Sigma V^T with sharp (kappa 1e7, 1e15) or smooth
    (kappa 1e15) decay and consistent-x right-hand sides (noise 0, 1e-12 or
    1e-2 of ||A x*||), the mu sweep {1e-4, 1e-6, 1e-8, 0} on the incoherent
    sharp and smooth sets; sparse 1% density 12000 x 10000 and 30000 x 4000,
    incoherent / coherent, sharp / smooth.  One JSON line."""
    # (name, kind, (m, n, decay, coherent), [(mu, noise), ...]); dense right-hand
    # sides are consistent-x with the given relative noise, sparse ones N(0, I)
    sweep = [(1e-4, 1e-2), (1e-6, 1e-2), (1e-8, 1e-2), (0.0, 1e-2)]
    noises = [(1e-4, 1e-2), (1e-4, 0.0), (1e-4, 1e-12)]
    cases = [
        ("dense 6000x5000 incoherent sharp 1e7", "dense", (6000, 5000, "sharp7", False), sweep + noises[1:]),
        ("dense 6000x5000 incoherent sharp 1e15", "dense", (6000, 5000, "sharp15", False), sweep),
        ("dense 6000x5000 coherent sharp 1e7", "dense", (6000, 5000, "sharp7", True), noises),
        ("dense 15000x2000 incoherent sharp 1e7", "dense", (15000, 2000, "sharp7", False), noises),
        ("dense 6000x5000 incoherent smooth 1e15", "dense", (6000, 5000, "smooth", False), sweep + noises[1:]),
        ("sparse 12000x10000 1% incoherent sharp 1e7", "sparse", (12000, 10000, "sharp7", False), [(1e-4, None)]),
        ("sparse 12000x10000 1% coherent sharp 1e7", "sparse", (12000, 10000, "sharp7", True), [(1e-4, None)]),
        ("sparse 30000x4000 1% incoherent sharp 1e7", "sparse", (30000, 4000, "sharp7", False), [(1e-4, None)]),
        ("sparse 30000x4000 1% coherent sharp 1e7", "sparse", (30000, 4000, "sharp7", True), [(1e-4, None)]),
        ("sparse 30000x4000 1% incoherent smooth 1e15", "sparse", (30000, 4000, "smooth", False), [(1e-4, None)]),
        ("sparse 30000x4000 1% coherent smooth 1e15", "sparse", (30000, 4000, "smooth", True), [(1e-4, None)]),
    ]
    out = []
    Aw, bw = synth.paper_dense_gpu(1, 300, 60, "sharp7")
    ap.lstsq(Aw, bw, mu=1e-4, block=6)  # warm-up (library initialisation)
    for ci, (name, kind, (m, n, decay, coh), runs) in enumerate(cases):
        As = bh = None
        if kind == "sparse":
            As, bh = synth.paper_sparse(6000 + ci, m, n, decay, coherent=coh)
        for mu, noise in runs:
            if kind == "dense":
                A, b = synth.paper_dense_gpu(6000 + ci, m, n, decay, coherent=coh, noise=noise)
            else:
                A = ap.CSRMatrix.from_scipy(As, device="cuda", dtype=torch.float64)
                b = torch.as_tensor(bh, device="cuda")
            row = {"workload": name, "mu": mu, "noise": noise}
            for label, pc in (("aplicur", True), ("plain_lsqr", False)):
                o = dict(mu=mu, block=max(1, n // 50), tol_ne=tol, max_iter=budget, precond=pc)
                try:
                    ms, (x, info) = _timed(torch, lambda: ap.lstsq(A, b, **o))
                except RuntimeError as e:  # a breakdown the method reports (e.g. CholQR of C)
                    row[label] = {"error": str(e)}
                    log(f"[bench] paper workload {name} mu={mu:g} noise={noise} {label}: {e}")
                    continue
                row[label] = {"ms": round(ms, 1), "iters": info.iters, "eta": info.eta, "status": info.status,
                              "rank": info.rank}
                log(f"[bench] paper workload {name} mu={mu:g} noise={noise} {label}: {ms:.0f} ms, "
                    f"{info.iters} it, eta {info.eta:.1e}, rank {info.rank}, status {info.status}")
            out.append(row)
            del A, b
            torch.cuda.empty_cache()
    print(json.dumps({"paper_workloads": out}), flush=True)


def svdfree_study(ap, synth, torch, tol=1e-8, budget=30000):
    """SVD-based (Alg. 2) against SVD-free (Alg. 8) preconditioner builds at
    mu = 0, FP64 on the GPU, time to eta <= tol: the small dense workload
    (2000 x 200, tol 1e-10) and the paper's test sets at mu = 0 (b = n/50).
    Per variant: total time, P-build time and count, CUR time, iterations,
    rank.  One JSON line."""
    cases = [("dense 2000x200 (sigma 10^(-6i/200))", None, 1e-10),
             ("dense 6000x5000 incoherent sharp 1e15", ("dense", 6000, 5000, "sharp15"), tol),
             ("dense 6000x5000 incoherent smooth 1e15", ("dense", 6000, 5000, "smooth"), tol),
             ("dense 15000x2000 incoherent sharp 1e15", ("dense", 15000, 2000, "sharp15"), tol),
             ("sparse 12000x10000 1% incoherent sharp 1e15", ("sparse", 12000, 10000, "sharp15"), tol)]
    out = []
    Aw, bw = synth.paper_dense_gpu(1, 300, 60, "sharp7")
    for pc in (1, 2):
        ap.lstsq(Aw, bw, mu=0.0, block=6, precond=pc)  # warm-up
    for ci, (name, spec, t) in enumerate(cases):
        if spec is None:
            w = synth.workload(1, 1.0)
            A, b, block = torch.as_tensor(w.A, device="cuda"), torch.as_tensor(w.B, device="cuda"), w.block
        elif spec[0] == "dense":
            A, b = synth.paper_dense_gpu(7000 + ci, spec[1], spec[2], spec[3], noise=1e-2)
            block = spec[2] // 50
        else:
            As, bh = synth.paper_sparse(7000 + ci, spec[1], spec[2], spec[3])
            A = ap.CSRMatrix.from_scipy(As, device="cuda", dtype=torch.float64)
            b, block = torch.as_tensor(bh, device="cuda"), spec[2] // 50
        row = {"workload": name, "mu": 0.0, "tol": t}
        for label, pc in (("svd", 1), ("svd_free", 2)):
            o = dict(mu=0.0, block=block, tol_ne=t, max_iter=budget, precond=pc)
            ap.lstsq(A, b, **o)  # warm-up at this shape (rocBLAS kernels, allocator)
            ms, (x, info) = _timed(torch, lambda: ap.lstsq(A, b, **o))
            row[label] = {"ms": round(ms, 1), "t_precond_ms": round(info.t_precond_ms, 1),
                          "builds": info.rebuilds, "t_cur_ms": round(info.t_cur_ms, 1),
                          "t_lsqr_ms": round(info.t_lsqr_ms, 1), "iters": info.iters, "rank": info.rank,
                          "eta": info.eta, "status": info.status}
            log(f"[bench] svd-free study {name} {label}: {ms:.0f} ms (P builds {info.t_precond_ms:.0f} ms / "
                f"{info.rebuilds}, CUR {info.t_cur_ms:.0f} ms, LSQR {info.t_lsqr_ms:.0f} ms), {info.iters} it, "
                f"rank {info.rank}, eta {info.eta:.1e}, status {info.status}")
        out.append(row)
        del A, b
        torch.cuda.empty_cache()
    print(json.dumps({"svdfree_study": out}), flush=True)


def schedule_study(ap, synth, torch):
    """Sec. 7.1 variants on the dense kernel workload at half size (FP32 A,
    16 RHS, mu = 1e-3, block 250) and on the sparse workload (rank cap 256):
    fully adaptive (schedule 0), rank-adaptive single shot (1), fixed-rank
    single shot at the rank the adaptive run reached (2).  One JSON line."""
    out = {}
    A, B = synth.rbf_kernel_gpu(3003, 20000, 16)
    w = synth.workload(2, 1.0)
    Ag = ap.CSRMatrix.from_scipy(w.A, device="cuda", dtype=torch.float64)
    bg = torch.as_tensor(w.B, device="cuda")
    cases = (("rbf20000", A, B, dict(mu=1e-3, block=250, tol_ne=1e-8)),
             ("csr200000", Ag, bg, dict(mu=w.mu, block=w.block, tol_ne=w.tol, max_rank=256)))
    for name, M, R, opts in cases:
        res, rank0 = {}, None
        for sched in (0, 1, 2):
            o = dict(opts)
            if sched == 2:
                o["max_rank"] = rank0
            ap.lstsq(M, R, schedule=sched, **o)  # warm-up
            ms, (X, info) = _timed(torch, lambda: ap.lstsq(M, R, schedule=sched, **o))
            if sched == 0:
                rank0 = info.rank
            res[f"schedule{sched}"] = {"ms": round(ms, 1), "rank": info.rank, "iters": info.iters,
                                       "phases": info.phases, "rebuilds": info.rebuilds, "eta": info.eta,
                                       "t_cur_ms": round(info.t_cur_ms, 1), "t_precond_ms": round(info.t_precond_ms, 1),
                                       "t_lsqr_ms": round(info.t_lsqr_ms, 1)}
            log(f"[bench] schedule study {name} schedule {sched}: {ms:.0f} ms rank {info.rank} "
                f"{info.iters} it {info.rebuilds} builds")
        out[name] = res
    print(json.dumps({"schedule_study": out}), flush=True)


def main():
    ap_ = argparse.ArgumentParser()
    ap_.add_argument("--gpus", type=int, default=1)
    ap_.add_argument("--steps", type=int, default=5)
    ap_.add_argument("--warmup", type=int, default=1)
    ap_.add_argument("--max-rank", type=int, default=256)
    ap_.add_argument("--no-cpu", action="store_true")
    ap_.add_argument("--products-only", action="store_true")
    ap_.add_argument("--blocked-products", action="store_true",
                     help="only the blocked products (FP32 RBF kernel 20000^2, 16 columns) and the calibration copy")
    ap_.add_argument("--npts", type=int, default=40000, help="points of the kernel matrix for --blocked-products")
    ap_.add_argument("--blocked-prec", type=int, default=0, choices=(0, 1, 2),
                     help="arithmetic of --blocked-products: 0 FP64 accumulation, 1 FP32, 2 BF16")
    ap_.add_argument("--no-extensions", action="store_true", help="skip the batched and adjoint comparisons")
    ap_.add_argument("--sparse-only", action="store_true",
                     help="only the sparse workload (CSR 200000 x 20000): its product loop and its APLICUR and "
                          "plain LSQR solves, one JSON line")
    ap_.add_argument("--headline-only", action="store_true",
                     help="only the warm-up and timed solves of the dense kernel workload (no comparisons, no "
                          "other workloads): the run that profiles the product kernel of value's steps")
    ap_.add_argument("--paper-workloads", action="store_true",
                     help="only the paper's test sets, APLICUR against plain LSQR, one JSON line")
    ap_.add_argument("--schedule-study", action="store_true",
                     help="only the adaptive against single-shot schedules comparison, one JSON line")
    ap_.add_argument("--svdfree-study", action="store_true",
                     help="only the SVD-based against SVD-free preconditioner comparison at mu = 0, one JSON line")
    ap_.add_argument("--sketch-study", action="store_true",
                     help="only the sparse sign against Gaussian sketch comparison, one JSON line")
    ap_.add_argument("--full-configs", action="store_true",
                     help="only the batched, dense-kernel and adjoint workloads at their full sizes (64 problems "
                          "x 8 RHS; RBF 40000^2 x 16 RHS; 100000 x 2000 x 32 RHS), one JSON line")
    args = ap_.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (got --gpus {args.gpus}): every problem here fits one MI355X and "
              "the multi-GPU layout is a design note, not a measured configuration.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2604_05065_amd as ap
    from workloads import synth

    if args.blocked_products:
        blocked_products(ap, synth, torch, npts=args.npts, prec=args.blocked_prec)
        return
    if args.paper_workloads:
        paper_workloads(ap, synth, torch)
        return
    if args.schedule_study:
        schedule_study(ap, synth, torch)
        return
    if args.sketch_study:
        sketch_study(ap, synth, torch)
        return
    if args.svdfree_study:
        svdfree_study(ap, synth, torch)
        return
    if args.full_configs:
        full = {"adjoint": bench_adjoint(ap, synth, torch, m=100000, n=2000, nrhs=32)}
        torch.cuda.empty_cache()
        full["multi_rhs"] = bench_multi_rhs(ap, synth, torch, npts=40000, nrhs=16)
        torch.cuda.empty_cache()
        full["batched"] = bench_batched(ap, synth, torch, count=64, scale=1.0, nrhs=8)
        print(json.dumps({"full_configs": full}), flush=True)
        return

    if args.products_only:
        bench_c2(ap, synth, torch, args)
        return
    if args.sparse_only:
        print(json.dumps({"csr_200000x20000": bench_c2(ap, synth, torch, args)}), flush=True)
        return

    head = bench_headline(ap, synth, torch, args)
    if args.headline_only:
        print(json.dumps({"value": head["ms_per_step"], "unit": "ms", "steps": args.steps, "warmup": args.warmup,
                          "roofline": head["roofline"], "seeds": head["seeds"], "memory": head["memory"],
                          "aplicur": head["aplicur"],
                          "products": head["products"]}), flush=True)
        return
    torch.cuda.empty_cache()
    c2 = bench_c2(ap, synth, torch, args)
    torch.cuda.empty_cache()
    adjoint = batched = None
    if not args.no_extensions:
        adjoint = bench_adjoint(ap, synth, torch, m=100000, n=2000, nrhs=32)
        torch.cuda.empty_cache()
        batched = bench_batched(ap, synth, torch, count=64, scale=1.0, nrhs=8, plain_subset=8)
        torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline_dense_kernel()
        log(f"[bench] cpu baseline: {cpu['value']:.0f} ms ({cpu['sample']})")

    out = {
        "metric": METRIC, "value": head["ms_per_step"], "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "seeds": head["seeds"],
        "memory": head["memory"],
        "aplicur": head["aplicur"],
        "compare": head["compare"],
        "products": head["products"],
        "csr_200000x20000": c2,
        "adjoint": adjoint,
        "batched": batched,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
