"""The residual norm check on its own (binv_residual): the full FP64 residual
against the oracle's compensated one, and the random-probe estimate against
the full value, including an error that sits in a single row, where a sample
of evenly spaced rows would see nothing (GPU).

The estimate is the mean of ||(AX - I) z||^2 over 64 random sign vectors z;
for a rank-one residual e_r v^T its ratio to ||AX - I||_F^2 is distributed
like chi-square(64) / 64, inside [0.36, 2.25] with probability above
1 - 1e-6, so rho's ratio is inside [0.6, 1.5].  The probes are a fixed
function of n, so each case below is deterministic."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2305_11103_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _dev(*mats):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(M)).cuda() for M in mats]


def test_full_residual_matches_the_oracle(gpu):
    from paper_2305_11103_amd import binv
    n = 700
    A = wl.general_haar(n, 90, 1e2)
    X = oracle.gj_inverse(A) + 1e-7 * np.random.default_rng(4).standard_normal((n, n))
    ro = oracle.residual_stats(A, X)["rho"]
    At, Xt = _dev(A, X)
    assert abs(binv.residual(At, Xt) - ro) <= 1e-6 * ro


def test_estimate_sees_an_error_in_one_row(gpu):
    """AX - I = e_r v^T (X = A^-1 + A^-1 e_r v^T): the whole error is row r,
    which is not one of rows 0, 15, 30, ... of a 64-row sample at n = 1000."""
    from paper_2305_11103_amd import binv
    n, r = 1000, 517
    A = wl.general_haar(n, 91, 1e2)
    Xo = oracle.gj_inverse(A)
    v = 1e-6 * np.random.default_rng(5).standard_normal(n)
    X = Xo + np.outer(Xo[:, r], v)
    rows = oracle.residual_rows(A, X)
    other = np.delete(np.arange(n), r)
    assert np.sqrt(np.sum(rows[other] ** 2)) <= 1e-3 * np.linalg.norm(rows[r])
    ro = oracle.residual_stats(A, X)["rho"]
    At, Xt = _dev(A, X)
    full = binv.residual(At, Xt)
    est = binv.residual(At, Xt, estimate=True)
    assert abs(full - ro) <= 1e-6 * ro
    assert 0.6 * ro <= est <= 1.5 * ro


def test_estimate_of_a_spread_error(gpu):
    """An error spread over every row: the estimate's spread is far smaller."""
    from paper_2305_11103_amd import binv
    n = 1000
    A = wl.general_haar(n, 92, 1e3)
    X = oracle.gj_inverse(A) + 1e-8 * np.random.default_rng(6).standard_normal((n, n))
    ro = oracle.residual_stats(A, X)["rho"]
    At, Xt = _dev(A, X)
    est = binv.residual(At, Xt, estimate=True)
    assert 0.8 * ro <= est <= 1.25 * ro


@pytest.mark.parametrize("n", [1, 64, 150, 191])
def test_small_orders_take_the_full_residual(gpu, n):
    from paper_2305_11103_amd import binv
    A = wl.general_haar(n, 93 + n, 10.0)
    X = oracle.gj_inverse(A) + 1e-9 * np.random.default_rng(n).standard_normal((n, n))
    At, Xt = _dev(A, X)
    assert binv.residual(At, Xt, estimate=True) == binv.residual(At, Xt)


@pytest.mark.parametrize("n", [192, 333])
def test_estimate_edge_orders_and_padded_rows(gpu, n):
    """n = 192 is the smallest order estimated (its probe workspace fills the
    n^2 buffer exactly); A and X are views with leading dimension n + 7."""
    import torch
    from paper_2305_11103_amd import binv
    A = wl.general_haar(n, 94 + n, 1e2)
    X = oracle.gj_inverse(A) + 1e-8 * np.random.default_rng(n).standard_normal((n, n))
    ro = oracle.residual_stats(A, X)["rho"]
    Ab = torch.zeros((n, n + 7), dtype=torch.float64, device="cuda")
    Xb = torch.full((n, n + 7), 7.0, dtype=torch.float64, device="cuda")
    Ab[:, :n] = torch.from_numpy(A).cuda()
    Xb[:, :n] = torch.from_numpy(X).cuda()
    At, Xt = Ab[:, :n], Xb[:, :n]
    assert abs(binv.residual(At, Xt) - ro) <= 1e-6 * ro
    est = binv.residual(At, Xt, estimate=True)
    assert 0.6 * ro <= est <= 1.5 * ro


def test_estimate_at_order_4096_tracks_the_full_residual(gpu):
    import torch
    from paper_2305_11103_amd import binv
    n = 4096
    A = wl.general_haar_device(n, wl.stream_seed(3, 9), 1e2, "cuda").contiguous()
    X = binv.invert(A, block=512)
    g = torch.Generator(device="cuda").manual_seed(3)
    X += 1e-9 * torch.randn((n, n), dtype=torch.float64, device="cuda", generator=g)
    full = binv.residual(A, X)
    est = binv.residual(A, X, estimate=True)
    assert full > 1e-9
    assert 0.8 * full <= est <= 1.25 * full


def test_argument_errors(gpu):
    import torch
    from paper_2305_11103_amd import binv
    lib = binv.load_library()
    ctx = binv.default_context(0)
    A = torch.eye(8, dtype=torch.float64, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rho = ctypes.c_double(-1.0)
    p = ctypes.c_void_p(A.data_ptr())
    assert lib.binv_residual(ctx.handle, 8, p, 8, p, 8, 4, s, ctypes.byref(rho)) == binv.BINV_E_INVALID
    both = binv.BINV_RESID_ESTIMATE | binv.BINV_RESID_COMPENSATED
    assert lib.binv_residual(ctx.handle, 8, p, 8, p, 8, both, s, ctypes.byref(rho)) == binv.BINV_E_INVALID
    assert lib.binv_residual(ctx.handle, 8, p, 7, p, 8, 0, s, ctypes.byref(rho)) == binv.BINV_E_INVALID
    assert lib.binv_residual(ctx.handle, -1, p, 8, p, 8, 0, s, ctypes.byref(rho)) == binv.BINV_E_INVALID
    assert lib.binv_residual(ctx.handle, 8, None, 8, p, 8, 0, s, ctypes.byref(rho)) == binv.BINV_E_INVALID
    assert lib.binv_residual(ctx.handle, 8, p, 8, p, 8, 0, s, None) == binv.BINV_E_INVALID
    assert lib.binv_residual(ctx.handle, 0, None, 0, None, 0, 0, s, ctypes.byref(rho)) == binv.BINV_OK
    assert rho.value == 0.0
    assert lib.binv_residual(ctx.handle, 8, p, 8, p, 8, 0, s, ctypes.byref(rho)) == binv.BINV_OK
    assert rho.value == 0.0  # I I - I = 0 exactly


@pytest.mark.parametrize("cond", [1e4, 1e6])
def test_compensated_residual_matrix_elementwise(gpu, cond):
    """binv_residual_matrix (the error-free split of A by rows and X by
    columns) against the oracle's compensated dot products, element by
    element on sampled rows: agreement to 1e-3 of the residual's own size,
    where a plain FP64 residual is off by about u |A| |X|, as large as the
    residual itself at cond 1e6."""
    import torch
    from paper_2305_11103_amd import binv
    n = 1024
    A_np = wl.general_haar(n, wl.stream_seed(3, 800 + int(np.log10(cond))), cond)
    X_np = oracle.gj_inverse(A_np)
    A = torch.from_numpy(A_np).cuda()
    X = torch.from_numpy(X_np).cuda()
    R, rho = binv.residual_matrix(A, X)
    torch.cuda.synchronize()
    rows = np.sort(np.random.default_rng(3).choice(n, 48, replace=False))
    Ro = -oracle.residual_rows(A_np, X_np, rows)  # oracle: A X - I; device: I - A X
    Rd = R.cpu().numpy()[rows]
    scale = np.max(np.abs(Ro))
    assert np.max(np.abs(Rd - Ro)) <= 1e-3 * scale
    st = oracle.residual_stats(A_np, X_np)
    assert abs(rho - st["rho"]) <= 1e-3 * st["rho"]
