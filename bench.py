"""Benchmark of the blockwise inversion library on one GPU.

--workload plain (default): plain FP64 blockwise inversion of one n = 8192
  matrix A = Q diag(s) Q^T (Q Haar-orthogonal, s log-uniform in [1, 1e4] with
  s_0 = 1 and s_1 = 1e4, so cond_2(A) = 1e4), split into a 16 x 16 grid of
  512 x 512 blocks.  One step = one full inversion (A -> X, out of place) with
  A already resident in HBM.
--workload batched: one batch of 100000 SPD 5 x 5 matrices plus 20000 SPD
  matrices of order uniform in [8, 256] (B B^T + 0.1 I, B Gaussian), each split
  into k in {2, 3, 4} near-equal diagonal blocks.  One step = the whole batch.
--workload mixed: n = 16384, 32 x 32 grid of 512-blocks, A = U diag(s) V^T
  (U, V Haar, s geometric with cond in {1e2, 1e4, 1e6}); the FP32 sweep with
  FP64 pivots and FP64 Newton-Schulz refinement to rho <= 1e-10, next to the
  plain FP64 sweep (refined from FP64 when it misses the target).
--workload serve: a Poisson stream of 5000 requests, orders log-uniform in
  [5, 8192], cond 10^U[1, 6], tagged fp64 or mixed (target 1e-10), through
  the continuous-batching server, at the arrival rate equal to the measured
  serial checked capacity, and at saturation (all at t = 0).
--workload levels: the paper's own parallel algorithm (section 5) on the
  batched workload's small matrices, next to the blockwise sweep's tiers.
--workload small: n = 256, 4 x 4 grid of 64-blocks; latency per inversion,
  eager and replayed from a HIP graph.
--workload host: out of core, n = 16384 in pinned host memory with a device
  budget of a quarter of the matrix; bitwise equal to the in-core result.
--workload mfma: the sustained rates of the FP64 instructions the trailing
  update can be built on (the 4x4x4 and 16x16x4 MFMAs and the vector FMA),
  from the standalone program paper_2305_11103_amd/mfma_rate.

Throughput counts 2 n^3 flops per inverse and is only reported as valid when
the oracle's compensated residual rho = ||AX - I||_F / sqrt(n) (sampled rows,
or sampled matrices) is within the workload's bound.  Prints one JSON line
with the throughput, a roofline entry for the dominant kernel (timed with HIP
events on the stream it runs on, during the timed region) and the CPU
oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "inverse TFLOP/s (2n³) at ‖AX−I‖≤bound vs plain FP64; solves/s + p50/p99 ms"
PEAK_FP64 = 78.6  # TFLOP/s, MI355X dense FP64 (matrix and vector)
PEAK_FP32 = 157.3  # TFLOP/s, MI355X dense FP32
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "schur_f64_n8192_b512_traffic.json")
BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "batched_swept_step_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2305_11103_amd", "csrc", "kernels.hip")
BATCH_SRC = os.path.join(ROOT, "paper_2305_11103_amd", "csrc", "batched_api.hip")
PEAK_HBM = 8000.0  # GB/s, MI355X HBM3E


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def sources_hash(*paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_batch_traffic():
    """Calibrated HBM bytes per swept-step launch of the batched workload from
    committed rocprofv3 counter runs, or None when the kernel or the plan's job
    formation changed since they were taken."""
    try:
        with open(BATCH_TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("sources_sha256_16") != sources_hash(KERNEL_SRC, BATCH_SRC):
        return None
    return t.get("bytes_per_launch")


def load_traffic():
    """HBM bytes per Schur launch from committed rocprofv3 counter runs, or None
    when the kernel source changed since they were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256_16") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(A: np.ndarray, budget_s: float, what: str = "the n=8192 matrix") -> dict:
    """The oracle's Gauss-Jordan inverse timed on host cores on the leading
    m x m principal block of the same matrix (a matrix of the same family),
    with m chosen so the run takes a bounded time."""
    import oracle

    oracle.build(force=False)
    m = 256
    t = 0.0
    # grow m until one run takes a meaningful slice of the budget
    while True:
        sub = np.ascontiguousarray(A[:m, :m])
        t0 = time.perf_counter()
        oracle.gj_inverse(sub)
        t = time.perf_counter() - t0
        if t > budget_s / 8 or 2 * m > A.shape[0]:
            break
        m *= 2
    rate = 2.0 * m ** 3 / t / 1e12
    return {"value": rate, "unit": "TFLOP/s", "cores": cores_used(), "kind": "oracle",
            "sample": f"Gauss-Jordan with partial pivoting (oracle) on the leading {m}x{m} block "
                      f"of {what}, one run of {t:.2f} s, rate 2m^3/t"}


def cores_used() -> int:
    cores = os.cpu_count() or 1
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    return min(int(os.environ.get("OMP_NUM_THREADS", cores)), cores)


def bench_plain(args):
    import torch

    from paper_2305_11103_amd import binv, workloads

    n, blk = args.n, args.block
    log(f"bench: generating SPD Haar matrix n={n} cond={args.cond:g} ({args.gen} QR)")
    t0 = time.perf_counter()
    dev = torch.device("cuda:0")
    if args.gen == "device":
        A = workloads.spd_haar_device(n, workloads.stream_seed(2, 0), args.cond, dev).contiguous()
        A_np = A.cpu().numpy()
    else:  # host QR (numpy): used where device QR cannot run, e.g. under counter collection
        A_np = workloads.spd_haar(n, workloads.stream_seed(2, 0), cond=args.cond)
        A = torch.from_numpy(A_np).to(dev)
    torch.cuda.empty_cache()
    log(f"bench: generated in {time.perf_counter() - t0:.1f} s")
    X = torch.empty_like(A)
    ctx = binv.default_context(0)
    part = workloads.uniform_partition(n, blk)

    def step():
        binv.invert(A, part=part, out=X, sync=False, ctx=ctx)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"bench: warmup {i + 1}/{args.warmup} done")

    # Only the trailing-update launches (on their own stream) carry timing
    # events in the timed region: event pairs on the caller's stream would add
    # their own gaps to the step being measured.
    ctx.set_timing(["schur"])
    ctx.get_timing()  # discard anything pending
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record()
        step()
        ends[i].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timing = ctx.get_timing()
    per = sorted(s.elapsed_time(e) for s, e in zip(starts, ends))
    ms_step = wall * 1e3 / args.steps
    log(f"bench: {args.steps} steps in {wall:.3f} s ({ms_step:.3f} ms/step)")
    # phase breakdown from one more step, outside the timed region, with every
    # phase's launches bracketed by events
    ctx.set_timing(["schur", "band", "pivot", "row", "tail"])
    ctx.get_timing()
    step()
    torch.cuda.synchronize()
    phases = ctx.get_timing()
    ctx.set_timing([])

    flops = 2.0 * n ** 3
    tflops = flops / (ms_step * 1e-3) / 1e12

    # parity gate: oracle residual on sampled rows
    import oracle
    Xh = X.cpu().numpy()
    rng = np.random.default_rng(1234)
    rows = np.sort(rng.choice(n, size=min(args.check_rows, n), replace=False))
    st = oracle.residual_stats(A_np, Xh, rows)
    ok = bool(st["rho"] <= 1e-10 and np.isfinite(Xh).all())
    log(f"bench: sampled rho={st['rho']:.3e} rho_max={st['rho_max']:.3e} ok={ok}")

    # roofline for the Schur trailing-update kernel: the library reports the
    # algorithmic flops of every timed launch (2 b per contracted element)
    s_ms, s_cnt, s_fl = timing["schur"]
    avg_ms = s_ms / max(s_cnt, 1)
    nb = len(part)
    schur_flops = s_fl / max(s_cnt, 1)
    achieved = schur_flops / (avg_ms * 1e-3) / 1e12
    traffic = load_traffic()

    cpu = None
    if not args.no_cpu:
        log("bench: timing the CPU oracle")
        cpu = cpu_baseline(A_np, args.cpu_budget)

    out = {
        "metric": METRIC,
        "value": round(tflops if ok else 0.0, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"plain FP64 blockwise inversion, n={n}, {nb}x{nb} grid of {blk}-blocks, "
                               f"SPD Q diag(s) Q^T cond {args.cond:g}",
                   "n": n, "block": blk, "k": nb, "cond": args.cond},
        "valid": ok,
        "rho_sampled": st["rho"],
        "rho_max_sampled": st["rho_max"],
        "rho_bound": 1e-10,
        "solves_per_s": round(1e3 / ms_step, 3),
        "p50_ms": round(per[len(per) // 2], 4),
        "p99_ms": round(per[min(len(per) - 1, int(0.99 * len(per)))], 4),
        "roofline": {"bound": "mfma", "kernel": "k_gemm_step<SCHUR,128,128>",
                     "achieved": round(achieved, 3), "peak": PEAK_FP64, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP64, 4), "traffic": traffic,
                     "avg_launch_ms": round(avg_ms, 4), "launches": s_cnt,
                     "flops_per_launch": schur_flops},
        "phase_ms_one_step_untimed": {ph: round(phases[ph][0], 4) for ph in ("schur", "band", "pivot", "row", "tail")},
        "lookahead_reserved_cus": ctx.lookahead_cus(),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_batched(args):
    import torch

    import oracle
    from paper_2305_11103_amd import binv, workloads

    log("bench: generating the uneven SPD batch (100000 x 5^2 + 20000 x U{8..256}^2)")
    t0 = time.perf_counter()
    sizes, parts = workloads.batch_spec(workloads.stream_seed(4, 0))
    mats = workloads.spd_gram_batch(sizes, workloads.stream_seed(4, 1))
    log(f"bench: generated in {time.perf_counter() - t0:.1f} s")
    ctx = binv.default_context(0)
    plan = binv.Batch(sizes, parts=parts, ctx=ctx)
    A = torch.from_numpy(plan.pack(mats)).to("cuda:0")
    X = torch.empty_like(A)
    info = torch.empty(plan.count, dtype=torch.int32, device="cuda:0")
    t0 = time.perf_counter()
    chosen, tune_ms, shapes = plan.tune(A, X, info=info, reps=3)
    tuned = {f"tier{t}": {"shape": list(shapes[t][c]), "ms": [round(v, 4) for v in tune_ms[t]]}
             for t, c in enumerate(chosen) if c >= 0}
    log(f"bench: autotuned tier shapes in {time.perf_counter() - t0:.2f} s: "
        + ", ".join(f"{k} {v['shape']}" for k, v in tuned.items()))
    for i in range(args.warmup):
        plan.invert(A, out=X, info=info, graph=True)
        log(f"bench: warmup {i + 1}/{args.warmup} done")

    # timed region: eager launches with per-phase events
    phases = ["small", "pivot", "row", "schur", "other"]
    ctx.set_timing(phases)
    ctx.get_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.invert(A, out=X, info=info, graph=False, sync=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timing = ctx.get_timing()
    ctx.set_timing([])
    ms_step = wall * 1e3 / args.steps
    # the same batch replayed as one HIP graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.invert(A, out=X, info=info, graph=True, sync=False)
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t0) * 1e3 / args.steps
    log(f"bench: {ms_step:.3f} ms/batch eager, {ms_graph:.3f} ms/batch graph")

    # parity gate on sampled matrices (all sizes represented)
    Xs = plan.unpack(X.cpu().numpy())
    inf = info.cpu().numpy()
    rng = np.random.default_rng(5)
    big = np.argsort(sizes)[-20:]
    pick = np.unique(np.concatenate([rng.choice(len(sizes), 300, replace=False), big]))
    rho = max(oracle.residual_stats(mats[i], Xs[i])["rho"] for i in pick)
    # every matrix's rho on the device (FP64, one workgroup per matrix)
    rho_dev = plan.residual(A, X).cpu().numpy()
    rho_dev_max = float(rho_dev.max())
    ok = bool((inf == 0).all() and rho <= 1e-12 and rho_dev_max <= 1e-12)
    log(f"bench: sampled max rho {rho:.3e} (oracle), all-matrix max rho {rho_dev_max:.3e} (device) ok={ok}")

    # a loop of single-matrix calls (plain FP64 path) on a sample, scaled up
    small_idx = [i for i in range(len(sizes)) if sizes[i] == 5][:200]
    large_idx = [i for i in range(len(sizes)) if sizes[i] > 5][:100]
    Ag = [torch.from_numpy(mats[i]).to("cuda:0") for i in small_idx + large_idx]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for M, i in zip(Ag, small_idx + large_idx):
        binv.invert(M, part=parts[i], sync=False, ctx=ctx)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    n_small, n_large = sum(1 for m in sizes if m == 5), sum(1 for m in sizes if m > 5)
    per_small = None
    t0 = time.perf_counter()
    for M, i in zip(Ag[:len(small_idx)], small_idx):
        binv.invert(M, part=parts[i], sync=False, ctx=ctx)
    torch.cuda.synchronize()
    per_small = (time.perf_counter() - t0) / max(len(small_idx), 1)
    per_large = (t_loop - per_small * len(small_idx)) / max(len(large_idx), 1)
    loop_s = per_small * n_small + per_large * n_large

    # roofline: the phase with the most time is the dominant kernel.  The
    # swept step (orders above the register tiers') is bound by HBM: its algorithmic traffic is
    # reading and writing each matrix once per step, 16 m^2 bytes per matrix
    # and step (one step per diagonal block, blocks over 128 split in two).
    dom = max(phases, key=lambda p: timing[p][0])
    d_ms, d_cnt, d_fl = timing[dom]
    kernel = {"small": "k_small_inverse (register tiers)",
              "schur": "k_swept_step (leaf + row panel + Schur update, one workgroup per matrix)",
              "row": "row panel", "pivot": "leaf", "other": "other"}[dom]
    avg_ms = d_ms / max(d_cnt, 1)
    if dom == "schur":
        steps_bytes = sum(16.0 * m * m * sum((b + 127) // 128 for b in pb)
                          for m, pb in zip(sizes, parts) if m > binv.TIER_LIMITS[-1])
        bytes_per_launch = steps_bytes * args.steps / max(d_cnt, 1)
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if d_ms > 0 else 0.0
        roof = {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1), "peak": PEAK_HBM, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM, 4), "traffic": load_batch_traffic(),
                "algorithmic_bytes_per_launch": bytes_per_launch,
                "launch": "one step of the swept tier (its shape-class dispatches, back to back)",
                "avg_launch_ms": round(avg_ms, 4),
                "launches": d_cnt, "tflops_per_launch": round(d_fl / max(d_cnt, 1) / (avg_ms * 1e-3) / 1e12, 3)}
    else:
        achieved = d_fl / max(d_cnt, 1) / (avg_ms * 1e-3) / 1e12 if d_ms > 0 else 0.0
        roof = {"bound": "alu", "kernel": kernel, "achieved": round(achieved, 3), "peak": PEAK_FP64,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64, 4), "traffic": None,
                "avg_launch_ms": round(avg_ms, 4), "launches": d_cnt, "flops_per_launch": d_fl / max(d_cnt, 1)}

    cpu = None
    if not args.no_cpu:
        log("bench: timing the CPU oracle on a sample of the batch")
        # matrices in a seeded random order (the batch's own size mix) until
        # the time budget is spent; rate = 2 sum m^3 / time
        order = np.random.default_rng(17).permutation(len(sizes))
        t0 = time.perf_counter()
        done = 0
        fl = 0.0
        n_large = 0
        while time.perf_counter() - t0 < args.cpu_budget and done < len(order):
            i = int(order[done])
            oracle.gj_inverse(mats[i])
            fl += 2.0 * sizes[i] ** 3
            n_large += sizes[i] > 5
            done += 1
        tc = time.perf_counter() - t0
        cpu = {"value": fl / tc / 1e12, "unit": "TFLOP/s", "cores": cores_used(), "kind": "oracle",
               "sample": f"Gauss-Jordan (oracle) on {done} matrices of the batch drawn in random order "
                         f"({n_large} of order 8..256, the rest of order 5), {tc:.1f} s; the whole batch at this "
                         f"rate would take {plan.flops / (fl / tc):.1f} s"}

    tflops = plan.flops / (ms_step * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": round(tflops if ok else 0.0, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batched uneven SPD: 100000 x 5^2 + 20000 x U{8..256}^2, k in {2,3,4} blocks",
                   "matrices": plan.count, "flops_per_batch": plan.flops},
        "valid": ok, "rho_max_sampled": rho, "rho_max_all_device": rho_dev_max, "rho_bound": 1e-12,
        "solves_per_s": round(plan.count / (ms_step * 1e-3), 1),
        "ms_per_batch_graph": round(ms_graph, 4),
        "loop_of_single_calls_ms_estimate": round(loop_s * 1e3, 1),
        "speedup_vs_loop": round(loop_s * 1e3 / ms_step, 1),
        "roofline": roof,
        "phase_ms_per_step": {p: round(timing[p][0] / args.steps, 4) for p in phases},
        "autotuned_tiers": tuned,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_small(args):
    """Config 1: one FP64 256 x 256 matrix (U[-1, 1] + 256 I), a 4 x 4 grid of
    64-blocks.  Latency-bound: reported in microseconds per inversion, eager
    (every launch enqueued by the host) and replayed from a HIP graph, each
    as the latency of one synchronized call (p50 / p99) and as the back-to-back
    rate."""
    import torch

    import oracle
    from paper_2305_11103_amd import binv, workloads

    n, part = 256, [64] * 4
    A_np = workloads.diag_dominant(n, workloads.stream_seed(1, 0))
    A = torch.from_numpy(A_np).to("cuda:0")
    X = torch.empty_like(A)
    ctx = binv.default_context(0)
    reps = max(args.steps, 200)
    res = {}
    # eager with and without the lookahead's side streams; the graph records
    # the one-stream schedule (the library captures only that one)
    for mode in ("eager_lookahead", "eager", "graph"):
        g = mode == "graph"
        look = mode == "eager_lookahead"
        for _ in range(max(args.warmup, 3)):
            binv.invert(A, part=part, out=X, ctx=ctx, sync=False, graph=g, lookahead=look)
        torch.cuda.synchronize()
        lat = []
        for _ in range(reps):
            t0 = time.perf_counter()
            binv.invert(A, part=part, out=X, ctx=ctx, sync=False, graph=g, lookahead=look)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t0) * 1e6)
        lat.sort()
        t0 = time.perf_counter()
        for _ in range(reps):
            binv.invert(A, part=part, out=X, ctx=ctx, sync=False, graph=g, lookahead=look)
        torch.cuda.synchronize()
        per = (time.perf_counter() - t0) * 1e6 / reps
        res[mode] = {"p50_us": round(lat[len(lat) // 2], 2), "p99_us": round(lat[int(0.99 * (len(lat) - 1))], 2),
                     "back_to_back_us": round(per, 2)}
        log(f"bench: {mode}: p50 {res[mode]['p50_us']} us, p99 {res[mode]['p99_us']} us, "
            f"back to back {res[mode]['back_to_back_us']} us per inversion")
    Xh = X.cpu().numpy()
    Xo = oracle.gj_inverse(A_np)
    err = float(np.max(np.abs(Xh - Xo)) / np.max(np.abs(Xo)))
    rho = oracle.residual_stats(A_np, Xh)["rho"]
    ok = bool(err <= 64 * n * 2.0 ** -53 * np.linalg.cond(A_np) and rho <= 1e-10)
    cpu = None
    if not args.no_cpu:
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < min(args.cpu_budget, 5.0):
            oracle.gj_inverse(A_np)
            k += 1
        t_gj = (time.perf_counter() - t0) / k
        t0 = time.perf_counter()
        oracle.blockwise_inverse(A_np, part)
        t_bw = time.perf_counter() - t0
        cpu = {"value": 2.0 * n ** 3 / t_gj / 1e12, "unit": "TFLOP/s", "cores": cores_used(), "kind": "oracle",
               "sample": f"Gauss-Jordan with partial pivoting (oracle) on the same matrix, {k} runs, "
                         f"{t_gj * 1e6:.0f} us each; the oracle's blockwise inversion {t_bw * 1e6:.0f} us"}
    flops = 2.0 * n ** 3
    best = res["graph"]["back_to_back_us"]
    out = {
        "metric": METRIC,
        "value": round(flops / (best * 1e-6) / 1e12 if ok else 0.0, 5),
        "unit": "TFLOP/s",
        "n_gpus": 1, "steps": reps, "warmup": max(args.warmup, 3),
        "ms_per_step": round(best / 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "plain FP64 blockwise inversion, n=256, 4x4 grid of 64-blocks, U[-1,1] + 256 I",
                   "n": n, "block": 64, "k": 4},
        "valid": ok, "max_rel_err_vs_oracle": err, "rho": rho,
        "latency_us": res,
        "solves_per_s": round(1e6 / best, 1),
        "p50_ms": round(res["graph"]["p50_us"] / 1e3, 5), "p99_ms": round(res["graph"]["p99_us"] / 1e3, 5),
        "roofline": {"bound": "latency", "kernel": "whole inversion (about 17 launches, replayed as one graph)",
                     "achieved": round(flops / (best * 1e-6) / 1e12, 5), "peak": PEAK_FP64, "unit": "TFLOP/s",
                     "frac": round(flops / (best * 1e-6) / 1e12 / PEAK_FP64, 6), "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_host(args):
    """Out of core (binv_invert_host): the n = 16384 SPD matrix (cond 1e4,
    32 x 32 grid of 512-blocks) stays in pinned host memory and the device
    may hold a quarter of it; every step streams all rows through the device
    in row slabs.  The result must equal the in-core inversion bit for bit.
    Bound by the host link: each step moves the whole matrix to the device
    and back (16 n^2 bytes) plus the pivot rows and the column panel."""
    import torch

    import oracle
    from paper_2305_11103_amd import binv, workloads

    dev = torch.device("cuda:0")
    n, blk = 16384, 512
    part = workloads.uniform_partition(n, blk)
    k = len(part)
    A = workloads.spd_haar_device(n, workloads.stream_seed(2, 1), args.cond, dev).contiguous()
    ctx = binv.default_context(0)
    ref = binv.invert(A, part=part, ctx=ctx)  # in core, the reference bits
    torch.cuda.synchronize()
    ref_h = ref.cpu()
    del ref
    Ah = A.cpu().pin_memory()
    del A
    torch.cuda.empty_cache()
    W = torch.empty_like(Ah).pin_memory()
    budget = 8 * n * n // 4
    for _ in range(max(args.warmup, 1)):
        W.copy_(Ah)
        binv.invert_host(W, budget, part=part, ctx=ctx)
    times = []
    steps = max(args.steps // 5, 2)
    for _ in range(steps):
        W.copy_(Ah)  # untimed: the input back in place (the call inverts in place)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        binv.invert_host(W, budget, part=part, ctx=ctx)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    t = min(times)
    ok = bool(torch.equal(W, ref_h))
    log(f"bench: out of core n={n}, device budget {budget / 2**30:.2f} GiB: {t * 1e3:.1f} ms per inversion "
        f"(best of {steps}), bitwise equal to in core: {ok}")
    flops = 2.0 * n ** 3
    link_bytes = k * (16.0 * n * n + 16.0 * blk * n)  # rows in and out per step, plus the pivot rows and column panel
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(Ah.numpy(), args.cpu_budget, f"the n={n} SPD matrix")
    out = {
        "metric": METRIC,
        "value": round(flops / t / 1e12 if ok else 0.0, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1, "steps": steps, "warmup": max(args.warmup, 1),
        "ms_per_step": round(t * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"out of core, n={n}, {k}x{k} grid of {blk}-blocks, SPD Q diag(s) Q^T cond "
                               f"{args.cond:g}, matrix in pinned host memory, device budget n^2 doubles / 4",
                   "n": n, "block": blk, "device_budget_bytes": budget},
        "valid": ok,
        "bitwise_equal_in_core": ok,
        "host_link_bytes_per_inversion": link_bytes,
        "roofline": {"bound": "host link", "kernel": "whole out-of-core inversion (row slabs over PCIe, both ways)",
                     "achieved": round(link_bytes / t / 1e9, 2), "peak": 128.0, "unit": "GB/s",
                     "frac": round(link_bytes / t / 1e9 / 128.0, 4), "traffic": None,
                     "peak_note": "PCIe 5.0 x16, 64 GB/s each way"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_levels(args):
    """The paper's own parallel algorithm (§5, binv_invert_batched_levels) on
    the batched workload's small matrices: 100000 SPD 5 x 5 (Table 2 gives
    blocks [2, 3]) plus 20000 SPD of order uniform in [8, 64], each split by
    Table 2's scheme, against the blockwise sweep's register tiers on the same
    plan (the same partitions)."""
    import torch

    import oracle
    from oracle import level_scheme as ls
    from paper_2305_11103_amd import binv, workloads

    rng = np.random.default_rng(workloads.stream_seed(4, 9))
    sizes = [5] * 100000 + [int(x) for x in rng.integers(8, 65, 20000)]
    parts = [binv.level_partition(m) for m in sizes]
    log("bench: generating the level-scheme batch (100000 x 5^2 + 20000 x U{8..64}^2 SPD)")
    mats = workloads.spd_gram_batch(sizes, workloads.stream_seed(4, 10))
    ctx = binv.default_context(0)
    plan = binv.Batch(sizes, parts=parts, ctx=ctx)
    A = torch.from_numpy(plan.pack(mats)).to("cuda:0")
    X = torch.empty_like(A)
    Xs = torch.empty_like(A)
    info = torch.empty(plan.count, dtype=torch.int32, device="cuda:0")
    # the scheme's own flop count, per distinct partition times its multiplicity
    from collections import Counter
    cnt = Counter(tuple(p) for p in parts)
    lvl_flops = sum(ls.level_scheme_flops(list(p)) * c for p, c in cnt.items())
    for i in range(args.warmup):
        plan.invert_levels(A, out=X, info=info)
        plan.invert(A, out=Xs, info=info, graph=True)
        log(f"bench: warmup {i + 1}/{args.warmup} done")
    ctx.set_timing(["small"])
    ctx.get_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.invert_levels(A, out=X, info=info, sync=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timing = ctx.get_timing()
    ctx.set_timing([])
    ms_step = wall * 1e3 / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.invert(A, out=Xs, info=info, graph=True, sync=False)
    torch.cuda.synchronize()
    ms_sweep = (time.perf_counter() - t0) * 1e3 / args.steps
    log(f"bench: level scheme {ms_step:.3f} ms/batch, blockwise sweep tiers {ms_sweep:.3f} ms/batch")
    plan.invert_levels(A, out=X, info=info)
    inf = info.cpu().numpy()
    rho_dev = plan.residual(A, X).cpu().numpy()
    Xh = plan.unpack(X.cpu().numpy())
    pick = np.unique(np.concatenate([np.random.default_rng(5).choice(len(sizes), 200, replace=False),
                                     np.argsort(sizes)[-20:]]))
    err = 0.0
    for i in pick:
        Xo = ls.level_scheme_inverse(mats[i], parts[i])
        tol = 64 * sizes[i] * 2.0 ** -53 * np.linalg.cond(mats[i]) * np.max(np.abs(Xo))
        err = max(err, float(np.max(np.abs(Xh[i] - Xo)) / tol))
    rho = max(oracle.residual_stats(mats[i], Xh[i])["rho"] for i in pick)
    ok = bool((inf == 0).all() and float(rho_dev.max()) <= 1e-12 and rho <= 1e-12 and err <= 1.0)
    log(f"bench: device max rho {rho_dev.max():.3e}, sampled oracle rho {rho:.3e}, "
        f"max error / tolerance {err:.3f}, ok={ok}")
    d_ms, d_cnt, d_fl = timing["small"]
    avg_ms = d_ms / max(d_cnt, 1)
    cpu = None
    if not args.no_cpu:
        log("bench: timing the oracle's level scheme on a sample of the batch")
        order = np.random.default_rng(17).permutation(len(sizes))
        t0 = time.perf_counter()
        fl, done = 0.0, 0
        while time.perf_counter() - t0 < args.cpu_budget and done < len(order):
            i = int(order[done])
            ls.level_scheme_inverse(mats[i], parts[i])
            fl += 2.0 * sizes[i] ** 3
            done += 1
        tc = time.perf_counter() - t0
        cpu = {"value": fl / tc / 1e12, "unit": "TFLOP/s", "cores": 1, "kind": "oracle",
               "sample": f"the oracle's level scheme (numpy, one thread) on {done} matrices of the batch in "
                         f"random order, {tc:.1f} s, rate 2 m^3 per matrix / time"}
    out = {
        "metric": METRIC,
        "value": round(plan.flops / (ms_step * 1e-3) / 1e12 if ok else 0.0, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "paper's level scheme (section 5) on 100000 x 5^2 + 20000 x U{8..64}^2 SPD, "
                               "Table 2 partitions", "matrices": plan.count, "flops_2m3": plan.flops,
                   "flops_level_scheme": lvl_flops},
        "valid": ok, "rho_max_all_device": float(rho_dev.max()), "rho_max_sampled": rho,
        "max_error_over_tolerance_sampled": err,
        "solves_per_s": round(plan.count / (ms_step * 1e-3), 1),
        "blockwise_sweep_ms_per_batch": round(ms_sweep, 4),
        "speedup_vs_blockwise_sweep": round(ms_sweep / ms_step, 3),
        "roofline": {"bound": "alu", "kernel": "k_level_scheme (one workgroup per matrix, one launch per order class)",
                     "achieved": round(d_fl / max(d_cnt, 1) / (avg_ms * 1e-3) / 1e12, 4) if d_ms > 0 else 0.0,
                     "peak": PEAK_FP64, "unit": "TFLOP/s",
                     "frac": round(d_fl / max(d_cnt, 1) / (avg_ms * 1e-3) / 1e12 / PEAK_FP64, 5) if d_ms > 0 else 0.0,
                     "traffic": None, "avg_launch_ms": round(avg_ms, 4), "launches": d_cnt,
                     "flops_counted": "the scheme's own flops (n^3 (3 - 1/N_k) for uniform blocks)"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_mixed(args):
    """Config 3 at each cond: the paper's unpivoted FP64 sweep, the FP64 sweep
    with block-row pivoting, and the two paths that end at the target: FP64
    (pivoted) + Newton-Schulz where needed, and the FP32 sweep + Newton-Schulz
    (falling back to the FP64 sweep when the FP32 start is beyond its reach).
    Both of those end with the device's compensated FP64 residual check, which
    is timed in both.  A result is valid only if the device reports it
    converged (rho <= 1e-10 by its full compensated residual) AND the oracle's
    compensated residual over sampled rows agrees with it."""
    import torch

    import oracle
    from paper_2305_11103_amd import binv, workloads

    n, blk = args.n if args.n != 8192 else 16384, args.block
    dev = torch.device("cuda:0")
    ctx = binv.default_context(0)
    part = workloads.uniform_partition(n, blk)
    rows = np.sort(np.random.default_rng(7).choice(n, size=min(args.check_rows, n), replace=False))
    target = 1e-10
    results = []
    t_plain_all, t_mixed_all = 0.0, 0.0
    ideal_all, fl_all = [], []
    cpu = None

    def timed(fn, reps=1):
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            best = t if best is None else min(best, t)
        return best, r

    for ci, cond in enumerate((1e2, 1e4, 1e6)):
        log(f"bench: generating U diag(s) V^T, n={n}, cond={cond:g} (device QR)")
        A = workloads.general_haar_device(n, workloads.stream_seed(3, ci), cond, dev).contiguous()
        torch.cuda.synchronize()
        X = torch.empty_like(A)
        Xm = torch.empty_like(A)
        # the two plain sweeps, warm then timed (best of 3), each with the
        # residual of its result (not timed)
        sweeps = {}
        for piv in (False, True):
            binv.invert(A, part=part, out=X, ctx=ctx, pivot=piv)
            t, _ = timed(lambda: binv.invert(A, part=part, out=X, ctx=ctx, pivot=piv), 3)
            sweeps[piv] = (t, binv.residual(A, X, ctx=ctx, compensated=True))
            log(f"bench: cond {cond:g}: FP64 sweep pivot={piv}: {t * 1e3:.1f} ms, rho {sweeps[piv][1]:.3e}")
        # FP64 (pivoted) sweep + compensated check + Newton-Schulz where needed
        binv.invert_mixed(A, part=part, out=X, ctx=ctx, from_fp64=True, pivot=True, target=target)
        t_ref, (X64, inf64) = timed(lambda: binv.invert_mixed(A, part=part, out=X, ctx=ctx, from_fp64=True,
                                                              pivot=True, target=target))
        # FP32 sweep + FP64 Newton-Schulz (FP64 pivoted sweep if it falls back)
        binv.invert_mixed(A, part=part, out=Xm, ctx=ctx, pivot=True, target=target)
        t_mixed, (Xm, infm) = timed(lambda: binv.invert_mixed(A, part=part, out=Xm, ctx=ctx, pivot=True,
                                                              target=target))
        Ah = A.cpu().numpy()
        rho_m = oracle.residual_stats(Ah, Xm.cpu().numpy(), rows)["rho"]
        rho_p = oracle.residual_stats(Ah, X64.cpu().numpy(), rows)["rho"]
        if cpu is None and not args.no_cpu:
            log("bench: timing the CPU oracle")
            cpu = cpu_baseline(Ah, args.cpu_budget, f"the n={n} cond={cond:g} U diag(s) V^T matrix")
        del Ah
        log(f"bench: cond {cond:g}: FP64+check/refine {t_ref * 1e3:.1f} ms (rho {inf64['rho']:.2e}, steps "
            f"{inf64['refine_steps']}, converged {inf64['converged']}), mixed {t_mixed * 1e3:.1f} ms "
            f"(rho {infm['rho']:.2e}, steps {infm['refine_steps']}, fell back {infm['fell_back']}, "
            f"converged {infm['converged']}); oracle sampled rho {rho_p:.2e} / {rho_m:.2e}")
        t_plain_all += t_ref
        t_mixed_all += t_mixed
        # roofline of each path: the flops its phases do, each at its MFMA
        # peak (FP32 sweep at the FP32 rate; the FP64 sweep, every compensated
        # residual (three FP64 products of 2 n^3) and every correction X R at
        # the FP64 rate).  Residuals: the start's, the FP64 sweep's after a
        # fallback, and one per Newton-Schulz step formed (accepted or not).
        g = 2.0 * n ** 3

        def path_flops(inf, fp32_start):
            formed = max(len(inf["rho_steps"]) - 1 - int(inf["fell_back"]), 0)  # Newton-Schulz steps formed
            resid = 1 + int(inf["fell_back"]) + formed
            f32 = g if fp32_start else 0.0
            f64 = (g if (inf["fell_back"] or not fp32_start) else 0.0) + 3 * resid * g + formed * g
            return f32, f64
        m32, m64 = path_flops(infm, True)
        _, p64 = path_flops(inf64, False)
        ideal_m = m32 / (PEAK_FP32 * 1e12) + m64 / (PEAK_FP64 * 1e12)
        ideal_p = p64 / (PEAK_FP64 * 1e12)
        ideal_all.append(ideal_m)
        fl_all.append(m32 + m64)
        results.append({
            "cond": cond,
            "fp64_sweep_unpivoted_ms": round(sweeps[False][0] * 1e3, 2), "fp64_sweep_unpivoted_rho": sweeps[False][1],
            "fp64_sweep_unpivoted_tflops": round(g / sweeps[False][0] / 1e12, 3),
            "fp64_sweep_pivoted_ms": round(sweeps[True][0] * 1e3, 2), "fp64_sweep_pivoted_rho": sweeps[True][1],
            "fp64_sweep_pivoted_tflops": round(g / sweeps[True][0] / 1e12, 3),
            "fp64_checked_ms": round(t_ref * 1e3, 2), "fp64_checked_rho": inf64["rho"],
            "fp64_checked_steps": inf64["refine_steps"], "fp64_checked_converged": inf64["converged"],
            "fp64_checked_rho_oracle_sampled": rho_p,
            "mixed_ms": round(t_mixed * 1e3, 2), "mixed_rho": infm["rho"], "mixed_rho_steps": infm["rho_steps"],
            "mixed_steps": infm["refine_steps"], "mixed_fell_back": infm["fell_back"],
            "mixed_converged": infm["converged"], "mixed_rho_oracle_sampled": rho_m,
            "mixed_flops_done": m32 + m64, "mixed_ideal_ms": round(ideal_m * 1e3, 2),
            "mixed_roofline_frac": round(ideal_m / t_mixed, 4),
            "fp64_checked_ideal_ms": round(ideal_p * 1e3, 2),
            "fp64_checked_roofline_frac": round(ideal_p / t_ref, 4),
            "speedup_mixed_vs_fp64_at_equal_accuracy": round(t_ref / t_mixed, 3)})
        del A, X, Xm, X64
        torch.cuda.empty_cache()
    # valid: the device's own convergence flag (full compensated residual)
    # and the oracle's compensated residual on sampled rows, for every matrix
    ok = all(r["mixed_converged"] and r["mixed_rho_oracle_sampled"] <= target for r in results)
    ok_p = all(r["fp64_checked_converged"] and r["fp64_checked_rho_oracle_sampled"] <= target for r in results)
    flops = 3 * 2.0 * n ** 3
    out = {
        "metric": METRIC,
        "value": round(flops / t_mixed_all / 1e12 if ok else 0.0, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(t_mixed_all / 3 * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"mixed precision, n={n}, {len(part)}x{len(part)} grid of {blk}-blocks, "
                               f"U diag(s) V^T Haar, cond 1e2/1e4/1e6, target rho 1e-10", "n": n, "block": blk},
        "valid": ok,
        "fp64_checked_valid": ok_p,
        "fp64_checked_tflops_equal_accuracy": round(flops / t_plain_all / 1e12 if ok_p else 0.0, 4),
        "per_cond": results,
        # the mixed path over the three matrices: achieved = the flops its
        # phases did / its time; peak = those flops / their ideal time (each
        # phase at its own MFMA peak), so frac = ideal time / measured time
        "roofline": {"bound": "mfma",
                     "kernel": "mixed path (FP32 sweep, FP64 pivoted sweep on fallback, compensated FP64 residuals, "
                               "FP64 corrections)",
                     "achieved": round(sum(fl_all) / t_mixed_all / 1e12, 3),
                     "peak": round(sum(fl_all) / sum(ideal_all) / 1e12, 3), "unit": "TFLOP/s",
                     "frac": round(sum(ideal_all) / t_mixed_all, 4), "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_serve(args):
    import torch

    import oracle
    from paper_2305_11103_amd import binv, workloads

    dev = torch.device("cuda:0")
    N = args.requests
    sizes, conds, tags = workloads.request_stream(N, workloads.stream_seed(5, 0))
    seeds = [workloads.stream_seed(5, 1 + i) for i in range(N)]
    flops = float(np.sum(2.0 * sizes.astype(np.float64) ** 3))
    # the serial baselines get a context of their own, closed before the
    # server starts: a context that has run the lookahead holds a CU-masked
    # stream, i.e. a hardware queue of its own, which the server's streams
    # would otherwise have to do without
    ctx = binv.Context(0)
    cur = torch.cuda.current_stream(dev)
    budget = args.budget_gib << 30

    # Every request's matrix is formed up front and stays resident, so no timed
    # region includes input preparation (about 153 GiB for the 5000 requests).
    log(f"bench: forming the {N} request matrices on the device")
    t0 = time.perf_counter()
    inputs = [workloads.householder_conditioned_device(int(sizes[i]), seeds[i], float(conds[i]), dev).contiguous()
              for i in range(N)]
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    log(f"bench: formed in {t_gen:.1f} s, {sum(a.numel() for a in inputs) * 8 / 2**30:.1f} GiB")

    def gen(i):
        return inputs[i]

    def blk(n):
        return 512 if n >= 2048 else (256 if n >= 512 else 128)

    def need(n, prec):  # device bytes the server charges (client-side back-pressure)
        b = 16 * n * n
        if n > 128:
            bl = min(512, n)
            b += 32 * bl * n + 16 * bl * bl + (20 * n * n if prec == "mixed" else 0)
        return b

    # Serial FIFO capacity, one request at a time: the plain FP64 sweep alone,
    # and the same sweep followed by the server's residual check (the random-
    # probe estimate; refinement when it fails), i.e. at the accuracy the server
    # gives.
    log(f"bench: serial plain-FP64 baseline over {N} requests")
    t_plain = t_checked = 0.0
    X_full = torch.empty(int(sizes.max()) ** 2, dtype=torch.float64, device=dev)
    for i in range(N):
        n = int(sizes[i])
        A = gen(i)
        X = X_full[: n * n].view(n, n)
        t0 = time.perf_counter()
        binv.invert(A, block=blk(n), out=X, ctx=ctx, lookahead=n >= 4096)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        # the same sweep with the server's check at every order (the full
        # residual below the probe estimate's minimum order)
        t0 = time.perf_counter()
        binv.invert_mixed(A, block=blk(n), out=X, ctx=ctx, lookahead=n >= 4096, from_fp64=True,
                          sampled_check=True)
        torch.cuda.synchronize()
        t_checked += time.perf_counter() - t0
        if (i + 1) % 500 == 0:
            log(f"bench: serial {i + 1}/{N}: plain {t_plain:.1f} s, checked {t_checked:.1f} s")
    mu_plain = N / t_plain
    mu = N / t_checked
    log(f"bench: serial capacity {mu_plain:.1f}/s plain, {mu:.1f}/s checked")
    del X_full
    torch.cuda.synchronize()
    ctx.close()
    torch.cuda.empty_cache()

    def run(rate, label, strict=False):
        srv = binv.Server(hbm_budget=budget, strict_precision=strict)
        rng = np.random.default_rng(11)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, N)) if rate > 0 else np.zeros(N)
        small = [i for i in range(N) if sizes[i] <= 1024]
        check = set(rng.choice(small, size=min(args.check_requests, len(small)), replace=False).tolist())
        tickets, t_sub, lat = {}, {}, np.zeros(N)
        not_conv = {"fp64": 0, "mixed": 0}
        # host copies and result buffers of the checked requests, made before the clock starts
        keep = {i: (inputs[i].cpu().numpy(),
                    torch.empty((int(sizes[i]), int(sizes[i])), dtype=torch.float64, device=dev)) for i in check}
        torch.cuda.synchronize()
        start = time.perf_counter()
        nxt, done_n, held = 0, 0, 0

        def collect(wait_us=0):
            nonlocal done_n, held
            got = 0
            while True:  # drain the server's completion queue
                t = srv.next_done(wait_us if got == 0 else 0)
                if t is None:
                    break
                i = tickets[t]
                out = keep[i][1] if i in keep else None
                r = srv.poll(t, out=out, copy=out is not None)
                _, info, tm = r
                lat[i] = (t_sub[i] - start - arrivals[i]) * 1e3 + tm["total_ms"]
                if not info["converged"]:
                    not_conv[str(tags[i])] += 1
                if i in keep:
                    keep[i] = (keep[i][0], keep[i][1].cpu().numpy(), info)
                held -= need(int(sizes[i]), str(tags[i]))
                del tickets[t]
                done_n += 1
                got += 1
            return got

        while done_n < N:
            progressed = collect() > 0
            now = time.perf_counter() - start
            while nxt < N and arrivals[nxt] <= now and held + need(int(sizes[nxt]), str(tags[nxt])) <= budget:
                n = int(sizes[nxt])
                A = gen(nxt)
                t_sub[nxt] = time.perf_counter()
                tickets[srv.submit(A, prec=str(tags[nxt]), target=1e-10)] = nxt
                held += need(n, str(tags[nxt]))
                nxt += 1
                progressed = True
                now = time.perf_counter() - start
            if not progressed:
                wait = 500 if nxt >= N or arrivals[nxt] > time.perf_counter() - start else 0
                collect(wait)
        makespan = time.perf_counter() - start
        peak = srv.stats()["peak"]
        srv.close()
        # accuracy on the oracle-checked requests: the gate is the target, or
        # twice the oracle Gauss-Jordan inverse's own rho where that is larger
        rhos = {"fp64": [], "mixed": []}
        worst, worst_req = 0.0, None
        for i, v in keep.items():
            A, X, info = v
            r = oracle.residual_stats(A, X)["rho"]
            r_o1 = oracle.residual_stats(A, oracle.gj_inverse(A))["rho"]
            rhos[str(tags[i])].append(r)
            q = r / max(1e-10, 2.0 * r_o1)
            if q >= worst:
                worst = q
                worst_req = {"request": int(i), "n": int(sizes[i]), "cond": float(conds[i]), "tag": str(tags[i]),
                             "rho_oracle": r, "rho_oracle_gj": r_o1, "rho_device": info["rho"],
                             "estimated": bool(info["sampled"]), "refine_steps": int(info["refine_steps"])}
        p50, p99 = float(np.percentile(lat, 50)), float(np.percentile(lat, 99))
        log(f"bench: {label}: {N / makespan:.1f} solves/s, {flops / makespan / 1e12:.2f} TFLOP/s, "
            f"p50 {p50:.2f} ms, p99 {p99:.2f} ms, peak {peak / 2**30:.1f} GiB")
        return {"solves_per_s": round(N / makespan, 2), "makespan_s": round(makespan, 3),
                "tflops": round(flops / makespan / 1e12, 4), "p50_ms": round(p50, 3), "p99_ms": round(p99, 3),
                "peak_charged_bytes": int(peak), "oracle_checked": len(keep),
                "rho_max_fp64_sampled": max(rhos["fp64"]) if rhos["fp64"] else None,
                "rho_max_mixed_sampled": max(rhos["mixed"]) if rhos["mixed"] else None,
                "worst_rho_over_gate": worst, "worst_request": worst_req, "not_converged": not_conv}

    served = run(mu, f"served at lambda={mu:.1f}/s")
    sat = run(0, "saturation")
    strict = run(0, "saturation, mixed tags honoured strictly", strict=True)
    ok = all(r["worst_rho_over_gate"] <= 1.0 for r in (served, sat, strict))

    cpu = None
    if not args.no_cpu:
        # the oracle on requests of the stream drawn in a seeded random order
        # until the time budget is spent (the last one may overrun it); rate =
        # 2 sum n^3 / time, and requests per second
        log("bench: timing the CPU oracle on a sample of the requests")
        oracle.build(force=False)
        order = np.random.default_rng(23).permutation(N)
        t0 = time.perf_counter()
        done, fl, nmax = 0, 0.0, 0
        while time.perf_counter() - t0 < args.cpu_budget and done < N:
            i = int(order[done])
            oracle.gj_inverse(inputs[i].cpu().numpy())
            fl += 2.0 * float(sizes[i]) ** 3
            nmax = max(nmax, int(sizes[i]))
            done += 1
        tc = time.perf_counter() - t0
        cpu = {"value": fl / tc / 1e12, "unit": "TFLOP/s", "cores": cores_used(), "kind": "oracle",
               "solves_per_s": round(done / tc, 2),
               "sample": f"Gauss-Jordan with partial pivoting (oracle) on {done} requests of the stream drawn in "
                         f"random order (largest order {nmax}), {tc:.1f} s including each input's copy to the host"}
    out = {
        "metric": METRIC,
        "value": round(sat["tflops"] if ok else 0.0, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(sat["makespan_s"] * 1e3, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"serving: {N} Poisson requests, n log-uniform [5, 8192], cond 10^U[1,6], "
                               f"fp64/mixed tags, target 1e-10, HBM budget {args.budget_gib} GiB"},
        "valid": ok,
        "solves_per_s": sat["solves_per_s"],
        "serial_fp64_solves_per_s": round(mu_plain, 2),
        "serial_fp64_checked_solves_per_s": round(mu, 2),
        "input_formation_s_untimed": round(t_gen, 3),
        "speedup_vs_serial_checked_at_saturation": round(sat["solves_per_s"] / mu, 3),
        "speedup_vs_serial_plain_at_saturation": round(sat["solves_per_s"] / mu_plain, 3),
        "served_at_serial_rate": served,
        "saturation": sat,
        "saturation_strict_precision": strict,
        # whole job: only each request's 2n^3 at the FP64 peak is counted (the
        # residual checks and refinement GEMMs are not), so frac is a floor
        "roofline": {"bound": "mfma", "kernel": "whole server at saturation (every request's 2n^3)",
                     "achieved": sat["tflops"], "peak": PEAK_FP64, "unit": "TFLOP/s",
                     "frac": round(sat["tflops"] / PEAK_FP64, 4), "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_mfma(args):
    """The FP64 instruction rates behind the GEMM core's design: runs the
    standalone measurement program (a child process; this process touches no
    GPU) and reports the 4x4x4 MFMA's sustained rate as the line's value."""
    import subprocess
    exe = os.path.join(ROOT, "paper_2305_11103_amd", "mfma_rate")
    if not os.path.exists(exe):
        raise SystemExit("paper_2305_11103_amd/mfma_rate is not built (run __graft_entry__.build())")
    reps = max(args.steps, 1)
    log(f"bench: running {exe} ({reps} timed launches per instruction)")
    r = subprocess.run([exe, str(reps)], capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        raise SystemExit(f"mfma_rate failed ({r.returncode}): {r.stderr.strip()}")
    lines = [json.loads(x) for x in r.stdout.splitlines() if x.strip().startswith("{")]
    dev = lines[0]
    rates = {x["instruction"]: x for x in lines[1:]}
    for x in lines[1:]:
        log(f"bench: {x['instruction']}: {x['tflops_best']:.2f} TFLOP/s best, {x['tflops_median']:.2f} median "
            f"({x['waves_per_simd']} waves per SIMD)")
    m4 = rates["v_mfma_f64_4x4x4_4b_f64"]
    out = {
        "metric": "sustained FP64 TFLOP/s of v_mfma_f64_4x4x4_4b_f64 (independent chains, every CU)",
        "value": round(m4["tflops_median"], 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": reps, "warmup": 1,
        "ms_per_step": round(m4["ms_median"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "FP64 instruction-rate microbenchmark: 4x4x4 and 16x16x4 MFMA, vector FMA, "
                               f"{dev['accumulators_per_wave']} independent chains per wave",
                   "compute_units": dev["compute_units"], "device": dev["device"]},
        "rates": {k: {"tflops_best": v["tflops_best"], "tflops_median": v["tflops_median"],
                      "waves_per_simd": v["waves_per_simd"], "flops_per_wave_instruction":
                      v["flops_per_wave_instruction"]} for k, v in rates.items()},
        "roofline": {"bound": "mfma", "kernel": "k_rate_mfma4 (v_mfma_f64_4x4x4_4b_f64 chains)",
                     "achieved": round(m4["tflops_median"], 3), "peak": PEAK_FP64, "unit": "TFLOP/s",
                     "frac": round(m4["tflops_median"] / PEAK_FP64, 4), "traffic": None},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["plain", "batched", "mixed", "serve", "levels", "small", "host", "mfma"],
                    default="plain")
    ap.add_argument("--gen", choices=["device", "host"], default="device",
                    help="where the plain workload's Haar factor is formed")
    ap.add_argument("--requests", type=int, default=5000)
    ap.add_argument("--check-requests", type=int, default=60)
    ap.add_argument("--budget-gib", type=int, default=64)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--block", type=int, default=512)
    ap.add_argument("--cond", type=float, default=1e4)
    ap.add_argument("--check-rows", type=int, default=64)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the batched and served forms shard with no communication; see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    {"plain": bench_plain, "batched": bench_batched, "mixed": bench_mixed, "serve": bench_serve,
     "levels": bench_levels, "small": bench_small, "host": bench_host, "mfma": bench_mfma}[args.workload](args)


if __name__ == "__main__":
    main()
