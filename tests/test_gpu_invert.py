"""Parity of the HIP blockwise inversion with the CPU oracle (needs a GPU).

Tolerances: the gate is the normalized residual rho = ||AX - I||_F / sqrt(n)
<= 1e-10 (measured by the oracle's compensated residual), and elementwise
|X_gpu - X_oracle| <= 64 n u kappa max|X_oracle| with u = 2^-53.
"""
import numpy as np
import pytest

import oracle
from paper_2305_11103_amd import workloads as wl

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def _inv(A_np, part=None, block=None, **kw):
    import torch
    from paper_2305_11103_amd import binv
    A = torch.from_numpy(np.ascontiguousarray(A_np)).cuda()
    X = binv.invert(A, part=part, block=block, **kw)
    torch.cuda.synchronize()
    return X.cpu().numpy()


def _check(A, X, kappa=None, rho_bound=1e-10):
    n = A.shape[0]
    Xo = oracle.gj_inverse(A)
    if kappa is None:
        kappa = np.linalg.cond(A)
    tol = 64 * n * U * kappa * np.max(np.abs(Xo))
    err = np.max(np.abs(X - Xo))
    assert err <= tol, (err, tol)
    st = oracle.residual_stats(A, X)
    assert st["rho"] <= rho_bound, st
    return err, st


def test_diag_dominant_256_4x4_blocks(gpu):
    A = wl.diag_dominant(256, wl.stream_seed(1, 0))
    X = _inv(A, part=[64] * 4)
    _check(A, X)
    X2 = oracle.blockwise_inverse(A, [64] * 4)
    assert np.max(np.abs(X - X2)) <= 64 * 256 * U * 2 * np.max(np.abs(X2))


@pytest.mark.parametrize("n,part", [
    (1, None), (2, [1, 1]), (5, [2, 3]), (63, [63]), (65, [64, 1]), (130, [128, 2]),
    (300, [64, 64, 64, 64, 44]), (517, None), (1000, [200, 300, 500]), (777, [7] * 111),
    # pivot blocks at the fused nested sweep's bounds: 129 (sub-blocks 64, 64,
    # 1), 2047 (the largest it takes) and 2048 (the copy-and-sweep path)
    (131, [129, 2]), (2100, [2047, 53]), (2100, [2048, 52]),
    # full 128 x 128 trailing-update tiles (operands staged straight into LDS)
    # with 1, 2, 3, 13 and 109 K-chunks of 16: odd counts end on the
    # single-chunk tail of the two-buffer loop
    (2048, [16, 32, 48, 208, 1744]),
])
def test_ragged_partitions(gpu, n, part):
    A = wl.diag_dominant(n, 1000 + n)
    X = _inv(A, part=part, block=128 if part is None else None)
    _check(A, X)


def test_spd_conditioned_1024(gpu):
    A = wl.spd_haar(1024, 21, cond=1e4)
    X = _inv(A, block=256)
    _check(A, X, kappa=1e4)


def test_inplace_equals_out_of_place_bitwise(gpu):
    import torch
    from paper_2305_11103_amd import binv
    A = torch.from_numpy(wl.diag_dominant(384, 5)).cuda()
    X = binv.invert(A, block=128)
    B = A.clone()
    binv.invert(B, block=128, inplace=True)
    torch.cuda.synchronize()
    assert torch.equal(X, B)


def test_run_to_run_bitwise(gpu):
    A = wl.spd_haar(640, 3, cond=1e3)
    assert np.array_equal(_inv(A, block=192), _inv(A, block=192))


def test_padded_leading_dimension(gpu):
    import torch
    from paper_2305_11103_amd import binv
    n = 200
    A_np = wl.diag_dominant(n, 8)
    big = torch.zeros((n, n + 13), dtype=torch.float64, device="cuda")
    big[:, :n] = torch.from_numpy(A_np).cuda()
    outbig = torch.full((n, n + 7), 7.0, dtype=torch.float64, device="cuda")
    binv.invert(big[:, :n], block=64, out=outbig[:, :n])
    torch.cuda.synchronize()
    X = outbig[:, :n].cpu().numpy()
    _check(A_np, X)
    assert torch.all(outbig[:, n:] == 7.0)


def test_block_diagonal_gives_exact_zero_off_blocks(gpu):
    rng = np.random.default_rng(5)
    part = [64, 100, 37, 128, 71]
    n = sum(part)
    M = np.zeros((n, n))
    off = 0
    mask = np.zeros((n, n), dtype=bool)
    for b in part:
        M[off:off + b, off:off + b] = rng.uniform(-1, 1, (b, b)) + b * np.eye(b)
        mask[off:off + b, off:off + b] = True
        off += b
    X = _inv(M, part=part)
    assert np.all(X[~mask] == 0.0)
    _check(M, X)


def test_unit_bidiagonal_exact(gpu):
    n = 300
    L = np.eye(n) - np.eye(n, k=-1)
    X = _inv(L, part=[64, 64, 100, 72])
    assert np.array_equal(X, np.tril(np.ones((n, n))))


def test_reversal_permutation_is_singular(gpu):
    from paper_2305_11103_amd import binv
    n = 128
    J = np.eye(n)[::-1].copy()
    with pytest.raises(binv.SingularError):
        _inv(J, part=[64, 64])


def test_singular_row_reported(gpu):
    import torch
    from paper_2305_11103_amd import binv
    n = 96
    A = wl.diag_dominant(n, 2)
    A[:, 40] = 0.0  # column 40 stays zero through step 0, so block 1 meets a zero pivot there
    info = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(binv.SingularError):
        binv.invert(torch.from_numpy(A).cuda(), part=[32, 32, 32], info=info)
    assert int(info.item()) == 41
    with pytest.raises(oracle.SingularError) as e:
        oracle.gj_inverse(A)
    assert e.value.row == 41


@pytest.mark.parametrize("inplace", [False, True])
def test_singular_row_in_a_nested_first_block(gpu, inplace):
    """A zero column inside block 0 of order 200 (inverted by the nested sweep;
    out of place with the lookahead, beside the copy of A into X): the call is
    singular and reports the 1-based row of the first zero pivot, as the oracle."""
    import torch
    from paper_2305_11103_amd import binv
    n = 300
    A = wl.diag_dominant(n, 3)
    A[:, 137] = 0.0
    info = torch.zeros(1, dtype=torch.int64, device="cuda")
    At = torch.from_numpy(A).cuda()
    with pytest.raises(binv.SingularError):
        binv.invert(At, part=[200, 100], info=info, inplace=inplace)
    with pytest.raises(oracle.SingularError) as e:
        oracle.gj_inverse(A)
    assert int(info.item()) == e.value.row == 138


def test_empty_matrix(gpu):
    import torch
    from paper_2305_11103_amd import binv
    X = binv.invert(torch.zeros((0, 0), dtype=torch.float64, device="cuda"))
    assert X.shape == (0, 0)


def test_invalid_partition_rejected(gpu):
    import torch
    from paper_2305_11103_amd import binv
    A = torch.eye(10, dtype=torch.float64, device="cuda")
    with pytest.raises(binv.BinvError):
        binv.invert(A, part=[3, 3])


@pytest.mark.parametrize("n,part", [(1000, [200, 300, 500]), (1536, [512, 512, 512]), (700, None), (2304, None)])
def test_lookahead_is_bitwise_identical(gpu, n, part):
    A = wl.diag_dominant(n, 77 + n)
    X1 = _inv(A, part=part, block=None if part else 256, lookahead=True)
    X2 = _inv(A, part=part, block=None if part else 256, lookahead=False)
    X3 = _inv(A, part=part, block=None if part else 256)  # the library's choice by order
    assert np.array_equal(X1, X3)
    assert np.array_equal(X1, X2)
    _check(A, X1)


_MASK_CHECK = """
import numpy as np, torch
from paper_2305_11103_amd import binv, workloads as wl
ctx = binv.Context(0)
print("reserved", ctx.lookahead_cus())
A = torch.from_numpy(wl.diag_dominant(1536, 5)).cuda()
X1 = binv.invert(A, block=256, ctx=ctx, lookahead=True)
X2 = binv.invert(A, block=256, ctx=ctx, lookahead=False)
torch.cuda.synchronize()
print("bitwise", bool(torch.equal(X1, X2)))
"""


@pytest.mark.parametrize("env,reserved", [({"BINV_SIDE_NCU": "8"}, 8), ({"BINV_REST_SPLIT": "0.6"}, 0)])
def test_lookahead_modes_in_a_fresh_process(gpu, env, reserved):
    """The lookahead's stream settings are read once per process, so each mode
    runs in a child process (one at a time): with BINV_SIDE_NCU = 8 the device
    must accept the trailing update's CU mask (one CU left out per XCD; the
    mask's bits go to the XCDs in turn), and with or without it, with the
    trailing update split around the pivot chain, the result must be bitwise
    equal to the serial schedule."""
    import os
    import subprocess
    import sys
    import torch
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    e = dict(os.environ, **env)
    out = subprocess.run([sys.executable, "-c", _MASK_CHECK], cwd=root, env=e, capture_output=True, text=True,
                         timeout=240)
    assert out.returncode == 0, out.stderr[-2000:]
    lines = dict(l.split(" ", 1) for l in out.stdout.strip().splitlines() if " " in l)
    assert int(lines["reserved"]) == (reserved if ncu > 16 else 0)
    assert lines["bitwise"] == "True"


def test_lookahead_has_no_mask_by_default(gpu):
    from paper_2305_11103_amd import binv
    assert binv.Context(0).lookahead_cus() == 0


def test_timing_reports_flops(gpu):
    import torch
    from paper_2305_11103_amd import binv
    n, blk = 2048, 512
    A = torch.from_numpy(wl.diag_dominant(n, 3)).cuda()
    ctx = binv.default_context(0)
    ctx.set_timing(["schur", "band", "tail", "row", "pivot"])
    ctx.get_timing()
    binv.invert(A, block=blk, ctx=ctx)
    t = ctx.get_timing()
    ctx.set_timing([])
    # every contracted element of the trailing update costs 2 b flops: the
    # trailing update, the lookahead's diagonal-block update and the part that
    # follows the pivot chain cover 2 b (n - b) n per block
    k = n // blk
    assert t["schur"][2] + t["band"][2] + t["tail"][2] == pytest.approx(k * 2.0 * blk * (n - blk) * n)
    assert t["row"][2] == pytest.approx(k * 2.0 * blk * blk * (n - blk))
    assert t["schur"][1] == k and t["band"][1] == k - 1


def test_full_size_bench_configuration(gpu):
    """The benchmark's own configuration (n = 8192, 16 x 16 grid of 512-blocks,
    SPD Q diag(s) Q^T with cond 1e4, lookahead schedule): the oracle's
    compensated residual on 48 sampled rows, the symmetry of the inverse of a
    symmetric matrix on the sampled rows and columns, and every element
    against the oracle's Gauss-Jordan inverse within 64 n u cond max|X|."""
    import torch
    from paper_2305_11103_amd import binv
    n = 8192
    A = wl.spd_haar_device(n, wl.stream_seed(2, 0), 1e4, "cuda").contiguous()
    X = binv.invert(A, block=512, lookahead=True)
    torch.cuda.synchronize()
    An, Xn = A.cpu().numpy(), X.cpu().numpy()
    rows = np.sort(np.random.default_rng(21).choice(n, 48, replace=False))
    st = oracle.residual_stats(An, Xn, rows)
    assert st["rho"] <= 1e-10, st
    assert np.isfinite(Xn).all()
    # the inverse of a symmetric matrix is symmetric: rounding-level asymmetry only
    asym = np.max(np.abs(Xn[rows][:, rows] - Xn[rows][:, rows].T)) / np.max(np.abs(Xn))
    assert asym <= 1e-9
    # element by element against Gauss-Jordan with partial pivoting on the
    # whole matrix (the oracle on the host's cores, about half a minute)
    print("full-size elementwise check against the oracle", flush=True)
    Xo = oracle.gj_inverse(An)
    assert np.max(np.abs(Xn - Xo)) <= 64 * n * U * 1e4 * np.max(np.abs(Xo))


@pytest.mark.parametrize("inplace,where", [(False, (0, 0)), (False, (699, 3)), (True, (5, 698)), (True, (699, 699))])
@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_non_finite_input_is_invalid(gpu, inplace, where, bad):
    """A NaN or an infinity anywhere in A: d_info = -1 and, synchronously,
    BINV_E_INVALID (in place and out of place, with and without lookahead)."""
    import torch
    from paper_2305_11103_amd import binv
    A_np = wl.diag_dominant(700, wl.stream_seed(1, 77))
    A_np[where] = bad
    for look in (True, False):
        A = torch.from_numpy(A_np).cuda()
        info = torch.full((1,), 5, dtype=torch.int64, device="cuda")
        binv.invert(A, part=[256, 256, 188], inplace=inplace, sync=False, info=info, lookahead=look)
        torch.cuda.synchronize()
        assert int(info.item()) == -1
        A = torch.from_numpy(A_np).cuda()
        with pytest.raises(binv.BinvError) as e:
            binv.invert(A, part=[256, 256, 188], inplace=inplace, lookahead=look)
        assert e.value.status == binv.BINV_E_INVALID and not isinstance(e.value, binv.SingularError)


def test_non_finite_with_a_zero_pivot_reports_invalid(gpu):
    """Both a NaN and an exactly-zero pivot column: the non-finite input wins."""
    import torch
    from paper_2305_11103_amd import binv
    A_np = wl.diag_dominant(256, wl.stream_seed(1, 78))
    A_np[:, 3] = 0.0
    A_np[200, 200] = np.nan
    info = torch.zeros(1, dtype=torch.int64, device="cuda")
    binv.invert(torch.from_numpy(A_np).cuda(), part=[64] * 4, sync=False, info=info)
    torch.cuda.synchronize()
    assert int(info.item()) == -1


_LOOKAHEAD_CAPTURE_OFF = ("capture of the two-stream lookahead schedule ended the test process with a host "
                          "segmentation fault on its first run (no GPU fault); the cause is not found, so that "
                          "path is switched off (BINV_F_GRAPH needs the one-stream schedule)")


@pytest.mark.parametrize("n,part,look", [
    pytest.param(256, [64] * 4, True, marks=pytest.mark.skip(reason=_LOOKAHEAD_CAPTURE_OFF)),
    pytest.param(1536, [512, 512, 512], True, marks=pytest.mark.skip(reason=_LOOKAHEAD_CAPTURE_OFF)),
    (700, [300, 400], False), (256, [64] * 4, False), (1536, [512, 512, 512], False),
    (256, [64] * 4, None), (1000, [200, 300, 500], None),  # below n = 2048 the default is the serial schedule
    pytest.param(1000, [200, 300, 500], True, marks=pytest.mark.skip(reason=_LOOKAHEAD_CAPTURE_OFF))])
def test_graph_replays_match_eager_every_time(gpu, n, part, look):
    """BINV_F_GRAPH: the first call runs eagerly and captures; every later
    call replays.  Each replay, with other eager work and synchronizations in
    between, equals the eager result bitwise, also after A's contents change
    under the same pointer (the replay reads A afresh)."""
    import torch
    from paper_2305_11103_amd import binv
    A1 = wl.diag_dominant(n, wl.stream_seed(1, 120 + n))
    A2 = wl.spd_haar(n, wl.stream_seed(2, 121 + n), 1e2)
    A = torch.from_numpy(A1).cuda()
    X = torch.empty_like(A)
    other = torch.from_numpy(wl.diag_dominant(300, 5)).cuda()
    ref1 = binv.invert(A, part=part, lookahead=look)
    for i in range(4):
        binv.invert(A, part=part, out=X, lookahead=look, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(X, ref1), i
        binv.invert(other, block=128)  # eager work between replays
        torch.cuda.synchronize()
    A.copy_(torch.from_numpy(A2).cuda())
    ref2 = binv.invert(A, part=part, lookahead=look)
    for i in range(3):
        X.fill_(7.0)
        binv.invert(A, part=part, out=X, lookahead=look, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(X, ref2), i
    _check(A2, X.cpu().numpy(), kappa=1e2)


def test_graph_singular_and_non_finite_through_replays(gpu):
    import torch
    from paper_2305_11103_amd import binv
    n, part = 256, [64] * 4
    A_np = wl.diag_dominant(n, 33)
    A = torch.from_numpy(A_np).cuda()
    X = torch.empty_like(A)
    # graph capture needs the one-stream schedule (rejected before any launch):
    # the lookahead asked for, or the library's default from n = 2048
    with pytest.raises(binv.BinvError) as e:
        binv.invert(A, part=part, out=X, graph=True, lookahead=True)
    assert e.value.status == binv.BINV_E_INVALID
    big = torch.eye(2048, dtype=torch.float64, device="cuda")
    with pytest.raises(binv.BinvError) as e:
        binv.invert(big, block=512, graph=True)
    assert e.value.status == binv.BINV_E_INVALID
    del big
    kw = dict(part=part, out=X, graph=True, lookahead=False)
    binv.invert(A, **kw)
    binv.invert(A, **kw)
    bad = A_np.copy()
    bad[:, 70] = 0.0
    A.copy_(torch.from_numpy(bad).cuda())
    with pytest.raises(binv.SingularError):
        binv.invert(A, **kw)
    bad[3, 3] = np.nan
    A.copy_(torch.from_numpy(bad).cuda())
    with pytest.raises(binv.BinvError) as e:
        binv.invert(A, **kw)
    assert e.value.status == binv.BINV_E_INVALID
    A.copy_(torch.from_numpy(A_np).cuda())
    binv.invert(A, **kw)
    torch.cuda.synchronize()
    _check(A_np, X.cpu().numpy())
