"""Continuous-batching server (GPU): every result is the same alone and in the
mix, meets its accuracy target (oracle residual), and admission never holds
more device memory than the budget."""
import time

import numpy as np
import pytest

import oracle
from paper_2305_11103_amd import workloads as wl

pytestmark = pytest.mark.gpu


def wait_all(srv, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t in out:
                continue
            try:
                r = srv.poll(t)
            except Exception as e:  # failed request: keep the exception
                out[t] = e
                continue
            if r is not None:
                out[t] = r
        if time.time() - t0 > timeout:
            raise TimeoutError("requests did not finish")
        time.sleep(0.002)
    return out


def in_round(n, prec, strict):
    """Does the server run this request in a shared round?  Orders up to 192
    always; 193..256 unless it is a mixed request honoured strictly (which
    starts from the FP32 sweep on a worker; its target 1e-10 is below that
    sweep's reach)."""
    return n <= 192 or (n <= 256 and not (prec == "mixed" and strict))


def alone(A, n, prec, strict=True, full_check=True):
    """The same request through the single-matrix entry points, under the
    server's policy: a round's request through the batched API (register
    tiers up to 192, swept steps of blocks of at most 128 above: the same
    kernels and blocks), a worker's through invert_mixed with an FP64 start
    unless a mixed request is honoured strictly."""
    import torch
    from paper_2305_11103_amd import binv
    At = torch.from_numpy(A).cuda()
    if in_round(n, prec, strict):
        b = binv.Batch([n])
        X, _ = b.invert(At.reshape(-1).contiguous(), graph=False)
        return X.reshape(n, n).cpu().numpy()
    blk = 512 if n >= 2048 else (256 if n >= 512 else 128)
    X, _ = binv.invert_mixed(At, block=blk, lookahead=n >= 4096, from_fp64=prec == "fp64" or not strict,
                             sampled_check=not full_check)
    return X.cpu().numpy()


@pytest.mark.parametrize("strict,full_check", [(True, True), (False, False)])
def test_mix_matches_alone_bitwise_and_meets_target(gpu, strict, full_check):
    import torch
    from paper_2305_11103_amd import binv
    srv = binv.Server(hbm_budget=8 << 30, strict_precision=strict, full_check=full_check)
    sizes = [5, 7, 16, 33, 64, 100, 128, 129, 200, 513, 700, 1100, 2048]
    reqs = []
    for i, n in enumerate(sizes * 2):
        prec = "mixed" if (i % 2 and n > 128) else "fp64"
        A = wl.spd_gram(n, 1000 + i) if n <= 256 else wl.general_haar(n, 2000 + i, 1e3) if prec == "mixed" \
            else wl.spd_haar(n, 2000 + i, 1e3)
        # every third request comes from device memory (copied at once)
        src = torch.from_numpy(A).cuda() if i % 3 == 0 else A
        torch.cuda.synchronize()
        reqs.append((A, n, prec, srv.submit(src, prec=prec)))
        del src
    res = wait_all(srv, [r[3] for r in reqs])
    for A, n, prec, t in reqs:
        if isinstance(res[t], Exception):
            raise AssertionError(f"request n={n} prec={prec} failed: {res[t]}") from res[t]
        X, info, times = res[t]
        assert info["converged"]
        assert times["total_ms"] >= times["queue_ms"] >= 0
        assert np.array_equal(X, alone(A, n, prec, strict, full_check)), (n, prec)
        assert info["sampled"] == (0 if (in_round(n, prec, strict) or full_check) else info["sampled"])
        if in_round(n, prec, strict):  # full residual measured on the device, no refinement needed here
            assert info["refine_steps"] == 0
            assert info["rho"] == pytest.approx(oracle.residual_stats(A, X)["rho"], rel=0.5, abs=1e-15)
        assert oracle.residual_stats(A, X)["rho"] <= 1e-10
    st = srv.stats()
    # what stays held once every result is collected: the blocks kept for
    # reuse and the workspace of the worker contexts and round buffers
    assert st["completed"] == len(reqs) and st["used"] <= st["peak"] <= 8 << 30
    srv.close()


def test_admission_holds_at_most_the_budget(gpu):
    from paper_2305_11103_amd import binv
    n = 1024
    budget = 3 * (16 * n * n + 4 * 8 * 512 * n + 8 * 512 * 512 * 2)  # room for three requests
    srv = binv.Server(hbm_budget=budget)
    mats = [wl.spd_haar(n, 70 + i, 1e2) for i in range(8)]
    tickets = [srv.submit(A) for A in mats]
    res = wait_all(srv, tickets)
    assert srv.stats()["peak"] <= budget
    for A, t in zip(mats, tickets):
        assert oracle.residual_stats(A, res[t][0])["rho"] <= 1e-10
    srv.close()


def test_singular_request_fails_alone(gpu):
    from paper_2305_11103_amd import binv
    srv = binv.Server(hbm_budget=1 << 30)
    good = wl.spd_gram(50, 3)
    bad = np.eye(300)[::-1].copy()
    tg, tb = srv.submit(good), srv.submit(bad)
    res = wait_all(srv, [tg, tb])
    assert isinstance(res[tb], binv.SingularError)
    assert oracle.residual_stats(good, res[tg][0])["rho"] <= 1e-12
    srv.close()


def test_budget_and_ticket_errors(gpu):
    from paper_2305_11103_amd import binv
    srv = binv.Server(hbm_budget=1 << 20)
    with pytest.raises(binv.BinvError):
        srv.submit(np.eye(1000))
    with pytest.raises(binv.BinvError):
        srv.poll(12345)
    srv.close()


def test_completion_queue_returns_every_ticket_once(gpu):
    """binv_next_done hands out each finished ticket exactly once, in
    completion order, and skips tickets collected directly."""
    from paper_2305_11103_amd import binv
    srv = binv.Server(hbm_budget=2 << 30)
    mats = [wl.spd_gram(m, 60 + i) for i, m in enumerate([5, 40, 130, 300, 8, 600])]
    tickets = [srv.submit(A) for A in mats]
    first = wait_all(srv, tickets[:1])  # collected directly: never handed out
    seen = []
    t0 = time.time()
    while len(seen) < len(tickets) - 1 and time.time() - t0 < 60:
        t = srv.next_done(wait_us=20000)
        if t is not None:
            seen.append(t)
            X, info, _ = srv.poll(t)
            A = mats[tickets.index(t)]
            assert oracle.residual_stats(A, X)["rho"] <= 1e-12
    assert sorted(seen) == sorted(tickets[1:])
    assert srv.next_done() is None
    assert isinstance(first[tickets[0]], tuple)
    srv.close()


def test_order_one_and_edge_orders(gpu):
    """Orders 1, 128, 129 (the small/large boundary) and 4096 (the large lane)
    through the server, against the oracle."""
    from paper_2305_11103_amd import binv
    srv = binv.Server(hbm_budget=4 << 30)
    mats = [np.array([[8.0]]), wl.spd_gram(128, 1), wl.spd_gram(129, 2), wl.diag_dominant(4096, 3)]
    tickets = [srv.submit(A) for A in mats]
    res = wait_all(srv, tickets, timeout=300)
    for A, t in zip(mats, tickets):
        X = res[t][0]
        if A.shape[0] == 1:
            assert X[0, 0] == 0.125
        else:
            rows = np.arange(0, A.shape[0], max(1, A.shape[0] // 64))
            assert oracle.residual_stats(A, X, rows)["rho"] <= 1e-10
    srv.close()


def test_device_memory_stays_within_budget(gpu):
    """The device memory the server really holds (hipMemGetInfo, sampled while
    requests run) stays within its budget: request blocks, the blocks it
    keeps for reuse, the workspace its worker contexts grow (residual, next
    iterate, compensated residual splits, panels) and its round buffers are
    all charged.  A budget of 1 GiB admits one order-3000 request at a time."""
    import torch
    from paper_2305_11103_amd import binv
    binv.invert(torch.eye(300, dtype=torch.float64, device="cuda"), block=128)  # library loaded
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    budget = 1 << 30
    srv = binv.Server(hbm_budget=budget)
    free0, _ = torch.cuda.mem_get_info()
    sizes = [3000, 2100, 1500, 40, 700, 90, 2500, 1200, 64, 3000, 900, 5, 2048]
    mats = [wl.spd_haar(n, 900 + i, 1e3) if n > 128 else wl.spd_gram(n, 900 + i) for i, n in enumerate(sizes)]
    tickets = [srv.submit(A, prec="mixed" if i % 3 == 1 else "fp64") for i, A in enumerate(mats)]
    out, worst = {}, 0
    t0 = time.time()
    while len(out) < len(tickets):
        free, _ = torch.cuda.mem_get_info()
        worst = max(worst, free0 - free)
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < 120
        time.sleep(0.001)
    st = srv.stats()
    print(f"budget {budget >> 20} MiB: ledger peak {st['peak'] >> 20} MiB, device peak {worst >> 20} MiB", flush=True)
    assert st["peak"] <= budget
    assert worst <= budget + (64 << 20)  # the runtime's own allocations
    for A, t in zip(mats, tickets):
        assert oracle.residual_stats(A, out[t][0])["rho"] <= 1e-10
    srv.close()


def test_swept_round_groups_steps_and_isolates_failures(gpu):
    """Orders 129..256 run in the server's rounds: up to 192 in the register
    tier, above that block step by block step in shared launches (one
    workgroup per request per step).  Every result is bitwise the batched
    API's for the same order (same kernels, same blocks),
    matches the oracle element by element and by residual, and a singular
    request in the round fails alone with its row."""
    from paper_2305_11103_amd import binv
    srv = binv.Server(hbm_budget=2 << 30)
    sizes = [129, 256, 150, 200, 131, 255, 192, 64, 230]
    mats = [wl.spd_gram(n, 3300 + i) for i, n in enumerate(sizes)]
    bad = wl.spd_gram(200, 3399)
    bad[:, 150] = 0.0
    tickets = [srv.submit(A) for A in mats]
    tb = srv.submit(bad)
    res = wait_all(srv, tickets + [tb])
    assert isinstance(res[tb], binv.SingularError) and "row 151" in str(res[tb])
    for A, n, t in zip(mats, sizes, tickets):
        X, info, _ = res[t]
        assert np.array_equal(X, alone(A, n, "fp64")), n
        assert info["refine_steps"] == 0 and info["converged"]
        ref = oracle.gj_inverse(A)
        tol = 64 * n * np.finfo(float).eps * np.linalg.cond(A) * np.abs(ref).max()
        assert np.abs(X - ref).max() <= tol, n
        assert oracle.residual_stats(A, X)["rho"] <= 1e-12
    srv.close()
