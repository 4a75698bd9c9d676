"""Benchmark of the blockwise inversion library on one GPU.

--workload plain (default): plain FP64 blockwise inversion of one n = 8192
  matrix A = Q diag(s) Q^T (Q Haar-orthogonal, s log-uniform in [1, 1e4] with
  s_0 = 1 and s_1 = 1e4, so cond_2(A) = 1e4), split into a 16 x 16 grid of
  512 x 512 blocks.  One step = one full inversion (A -> X, out of place) with
  A already resident in HBM.
--workload batched: one batch of 100000 SPD 5 x 5 matrices plus 20000 SPD
  matrices of order uniform in [8, 256] (B B^T + 0.1 I, B Gaussian), each split
  into k in {2, 3, 4} near-equal diagonal blocks.  One step = the whole batch.

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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "schur_f64_n8192_b512_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2305_11103_amd", "csrc", "kernels.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


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


def cpu_baseline(A: np.ndarray, budget_s: float) -> dict:
    """The oracle's Gauss-Jordan inverse timed on host cores on the leading
    m x m principal block of the same matrix (an SPD matrix of the same
    family), with m chosen so the run takes a bounded time."""
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
                      f"of the n=8192 matrix, one run of {t:.2f} s, rate 2m^3/t"}


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
    log(f"bench: generating SPD Haar matrix n={n} cond={args.cond:g}")
    t0 = time.perf_counter()
    A_np = workloads.spd_haar(n, workloads.stream_seed(2, 0), cond=args.cond)
    log(f"bench: generated in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    A = torch.from_numpy(A_np).to(dev)
    X = torch.empty_like(A)
    ctx = binv.default_context(0)
    part = workloads.uniform_partition(n, blk)

    def step():
        binv.invert(A, part=part, out=X, sync=False, ctx=ctx)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"bench: warmup {i + 1}/{args.warmup} done")

    ctx.set_timing(["schur", "band", "pivot", "row"])
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
    ctx.set_timing([])
    per = sorted(s.elapsed_time(e) for s, e in zip(starts, ends))
    ms_step = wall * 1e3 / args.steps
    log(f"bench: {args.steps} steps in {wall:.3f} s ({ms_step:.3f} ms/step)")

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
        "phase_ms_per_step": {ph: round(timing[ph][0] / args.steps, 4) for ph in ("schur", "band", "pivot", "row")},
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
    ok = bool((inf == 0).all() and rho <= 1e-12)
    log(f"bench: sampled max rho {rho:.3e} ok={ok}")

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

    # roofline: the phase with the most time is the dominant kernel
    dom = max(phases, key=lambda p: timing[p][0])
    d_ms, d_cnt, d_fl = timing[dom]
    kernel = {"small": "k_small_inverse (register tiers)", "schur": "k_gemm_step_batched<SCHUR,64x64>",
              "row": "k_gemm_step_batched<ROW,64x64>", "pivot": "k_leaf_inverse_batched",
              "other": "k_col_save_batched"}[dom]
    bound = "mfma" if dom in ("schur", "row") else "alu"
    achieved = d_fl / (d_ms / max(d_cnt, 1) * 1e-3) / max(d_cnt, 1) / 1e12 if d_ms > 0 else 0.0

    cpu = None
    if not args.no_cpu:
        log("bench: timing the CPU oracle on a sample of the batch")
        sample = small_idx + large_idx
        t0 = time.perf_counter()
        done = 0
        fl = 0.0
        while time.perf_counter() - t0 < args.cpu_budget / 4 and done < len(sample):
            i = sample[done]
            oracle.gj_inverse(mats[i])
            fl += 2.0 * sizes[i] ** 3
            done += 1
        tc = time.perf_counter() - t0
        cpu = {"value": fl / tc / 1e12, "unit": "TFLOP/s", "cores": cores_used(), "kind": "oracle",
               "sample": f"Gauss-Jordan (oracle) on {done} matrices of the batch (200 of order 5 then orders 8..256), "
                         f"{tc:.2f} s"}

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
        "valid": ok, "rho_max_sampled": rho, "rho_bound": 1e-12,
        "solves_per_s": round(plan.count / (ms_step * 1e-3), 1),
        "ms_per_batch_graph": round(ms_graph, 4),
        "loop_of_single_calls_ms_estimate": round(loop_s * 1e3, 1),
        "speedup_vs_loop": round(loop_s * 1e3 / ms_step, 1),
        "roofline": {"bound": bound, "kernel": kernel, "achieved": round(achieved, 3), "peak": PEAK_FP64,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64, 4), "traffic": None,
                     "avg_launch_ms": round(d_ms / max(d_cnt, 1), 4), "launches": d_cnt,
                     "flops_per_launch": d_fl / max(d_cnt, 1)},
        "phase_ms_per_step": {p: round(timing[p][0] / args.steps, 4) for p in phases},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["plain", "batched"], default="plain")
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
    {"plain": bench_plain, "batched": bench_batched}[args.workload](args)


if __name__ == "__main__":
    main()
