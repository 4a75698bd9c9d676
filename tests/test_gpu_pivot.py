"""Block-row pivoting on the GPU (BINV_F_PIVOT) against the oracle (needs a GPU).

The oracle's orc_block_gj computes the same readings in plain loops: without
pivoting across blocks (the paper's method) and with tournament block-row
pivoting.  Tolerances: elementwise |X - X_ref| <= 64 n u kappa max|X_ref|
(u = 2^-53, kappa the exact condition number of the generated matrix); the
residual gate is rho = ||AX - I||_F / sqrt(n) <= max(1e-10, 2 rho_GJ), where
rho_GJ is that of Gauss-Jordan with partial pivoting on the same matrix (its
own rho exceeds 1e-10 at kappa = 1e6, so the bound is the one it reaches).
"""
import numpy as np
import pytest

import oracle
from paper_2305_11103_amd import workloads as wl

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def _inv(A_np, part, **kw):
    import torch
    from paper_2305_11103_amd import binv
    A = torch.from_numpy(np.ascontiguousarray(A_np)).cuda()
    X = binv.invert(A, part=part, **kw)
    torch.cuda.synchronize()
    return X.cpu().numpy()


def _rho(A, X):
    return oracle.residual_stats(A, X)["rho"]


@pytest.mark.parametrize("n,cond", [(1024, 1e2), (1024, 1e4), (1024, 1e6), (2048, 1e4)])
def test_pivoted_general_matches_oracle_and_gauss_jordan(gpu, n, cond):
    A = wl.general_haar(n, wl.stream_seed(3, 100 + n + int(np.log10(cond))), cond)
    part = wl.uniform_partition(n, 512)
    print(f"pivoted n={n} cond={cond:g}", flush=True)
    X = _inv(A, part, pivot=True)
    Xr = oracle.block_gj_inverse(A, part, pivot=True)
    Xo = oracle.gj_inverse(A)
    tol = 64 * n * U * cond * np.abs(Xo).max()
    assert np.abs(X - Xr).max() <= tol
    assert np.abs(X - Xo).max() <= tol
    r, ro = _rho(A, X), _rho(A, Xo)
    assert r <= max(1e-10, 2 * ro), (r, ro)


@pytest.mark.parametrize("cond", [1e4, 1e6])
def test_unpivoted_growth_is_the_method_not_the_kernel(gpu, cond):
    """General input, no pivoting across blocks: the GPU sweep and the
    oracle's reading of it lose accuracy alike (the same growth), so their
    difference is no larger than the oracle's own error."""
    n = 1024
    A = wl.general_haar(n, wl.stream_seed(3, 200 + int(np.log10(cond))), cond)
    part = wl.uniform_partition(n, 512)
    X = _inv(A, part)
    Xr = oracle.block_gj_inverse(A, part, pivot=False)
    Xo = oracle.gj_inverse(A)
    own = np.abs(Xr - Xo).max()
    assert np.abs(X - Xr).max() <= 10 * own + 64 * n * U * cond * np.abs(Xo).max()
    r, rr = _rho(A, X), _rho(A, Xr)
    assert rr / 30 <= r <= 30 * rr, (r, rr)


@pytest.mark.parametrize("n,part", [
    (1, [1]), (5, [2, 3]), (64, [64]), (100, [37, 63]), (130, [65, 65]), (300, [129, 171]),
    (700, [100, 300, 300]), (1000, [512, 488]), (2100, [2047, 53]), (333, [1] * 333),
])
def test_pivoted_ragged_partitions(gpu, n, part):
    A = wl.general_haar(n, wl.stream_seed(3, 300 + n), 1e3) if n > 1 else np.array([[3.0]])
    print(f"ragged n={n} k={len(part)}", flush=True)
    X = _inv(A, part, pivot=True)
    Xo = oracle.gj_inverse(A)
    assert np.abs(X - Xo).max() <= 64 * n * U * 1e3 * np.abs(Xo).max()
    assert _rho(A, X) <= max(1e-10, 2 * _rho(A, Xo))


@pytest.mark.parametrize("n,b", [(1024, 512), (600, 128), (200, 64)])
def test_reversal_permutation_is_inverted_exactly(gpu, n, b):
    """§3's counter-example: every leading block of the reversal permutation
    is singular; with block-row pivoting the inverse is exact (J^-1 = J)."""
    J = np.eye(n)[::-1].copy()
    X = _inv(J, wl.uniform_partition(n, b), pivot=True)
    assert np.array_equal(X, J)


def test_scaled_permutation_exact_over_many_tournament_leaves(gpu):
    """A = P D (one nonzero per row and column, powers of two): every
    tournament node keeps the rows with nonzeros in its columns, across
    4 leaves per strip; the inverse D^-1 P^T is exact."""
    n = 1100
    rng = np.random.default_rng(4)
    pi = rng.permutation(n)
    d = 2.0 ** rng.integers(-3, 4, n) * rng.choice([-1.0, 1.0], n)
    A = np.zeros((n, n))
    A[np.arange(n), pi] = d
    Xe = np.zeros((n, n))
    Xe[pi, np.arange(n)] = 1.0 / d
    X = _inv(A, [512, 300, 288], pivot=True)
    assert np.array_equal(X, Xe)


def test_pivoted_exact_on_dyadic_plu_single_leaf(gpu):
    from tests import exact
    rng = np.random.default_rng(12)
    for trial in range(3):
        A, Ai, _ = exact.dyadic_plu(12, rng)
        X = _inv(A, [5, 4, 3], pivot=True)
        assert np.array_equal(X, Ai), trial


def test_pivoted_lookahead_inplace_bitwise(gpu):
    import torch
    from paper_2305_11103_amd import binv
    n = 1536
    A_np = wl.general_haar(n, wl.stream_seed(3, 400), 1e4)
    part = [512, 384, 640]
    A = torch.from_numpy(A_np).cuda()
    X1 = binv.invert(A, part=part, pivot=True, lookahead=True)
    X2 = binv.invert(A, part=part, pivot=True, lookahead=False)
    X3 = A.clone()
    binv.invert(X3, part=part, pivot=True, inplace=True)
    torch.cuda.synchronize()
    assert torch.equal(X1, X2) and torch.equal(X1, X3)
    X4 = binv.invert(A, part=part, pivot=True)
    torch.cuda.synchronize()
    assert torch.equal(X1, X4)  # run to run


def test_pivoted_zero_column_reports_row(gpu):
    import torch
    from paper_2305_11103_amd import binv
    n = 700
    A_np = wl.general_haar(n, wl.stream_seed(3, 401), 1e2)
    A_np[:, 300] = 0.0
    A = torch.from_numpy(A_np).cuda()
    info = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(binv.SingularError):
        binv.invert(A, part=[256, 256, 188], pivot=True, info=info)
    assert int(info.item()) == 301
    with pytest.raises(oracle.SingularError) as e:
        oracle.gj_inverse(A_np)
    assert e.value.row == 301


def test_pivot_rejects_blocks_above_its_limit(gpu):
    import torch
    from paper_2305_11103_amd import binv
    A = torch.eye(2100, dtype=torch.float64, device="cuda")
    with pytest.raises(binv.BinvError) as e:
        binv.invert(A, part=[2048, 52], pivot=True)
    assert e.value.status == binv.BINV_E_INVALID
