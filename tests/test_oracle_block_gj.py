"""Pins for the oracle's block Gauss-Jordan (no GPU).

orc_block_gj implements the two readings the GPU path computes: block
Gauss-Jordan over the partition (Eq. (a) of §3 unrolled one diagonal block at
a time, the in-place procedure of §4.2) without pivoting across blocks, and
with block-row pivoting by tournament selection.  Each test checks it against
something fixed outside it: exact rational inverses of dyadic P L U matrices
(where elimination in the pivot order is exact, so the result must be
bitwise the exact inverse), the paper's permutation counter-example (§3),
exact zero blocks, Gauss-Jordan with partial pivoting on one leaf, and the
residual of the plain definition on general inputs.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2305_11103_amd import workloads as wl
from tests import exact

U = np.finfo(np.float64).eps / 2


@pytest.mark.parametrize("n", [1, 7, 64, 128])
def test_one_small_block_is_gauss_jordan_bitwise(n):
    A = wl.diag_dominant(n, 11 + n) - 0.9 * n * np.eye(n)
    X = oracle.block_gj_inverse(A, [n], pivot=False)
    assert np.array_equal(X, oracle.gj_inverse(A))


@pytest.mark.parametrize("n,part,sub", [(9, [9], 3), (10, [4, 6], 2), (12, [5, 4, 3], 3), (12, [3] * 4, 4)])
def test_pivoted_exact_on_dyadic_plu(n, part, sub):
    """One tournament leaf covering every row: the selection is partial
    pivoting itself, which recovers Pi, L and U, so every operation is exact
    and the result must equal the exact inverse bit for bit; the final row
    order must be Pi's."""
    rng = np.random.default_rng(1000 + n + sub)
    for trial in range(3):
        A, Ai, pi = exact.dyadic_plu(n, rng)
        X, perm = oracle.block_gj_inverse(A, part, pivot=True, sub=sub, leaf_rows=4 * n, arity=2,
                                          return_perm=True)
        assert np.array_equal(X, Ai), f"trial {trial}"
        # position i holds the original row of A whose pivot is (L U) row i
        assert np.array_equal(np.argsort(pi), perm)


@pytest.mark.parametrize("n,part,sub,leaf,arity", [(20, [7, 6, 7], 3, 4, 2), (24, [8, 8, 8], 4, 5, 3),
                                                   (17, [17], 4, 3, 2), (26, [13, 13], 5, 4, 4)])
def test_pivoted_multi_leaf_tournament_exact_on_permuted_triangular(n, part, sub, leaf, arity):
    """A = Pi U (U upper triangular, dyadic): every tournament node meets one
    nonzero candidate per column among the rows it must keep, so the root
    picks U's rows in order across many leaves and merges; elimination in
    that order is exact."""
    rng = np.random.default_rng(2000 + n)
    for trial in range(3):
        A, Ai, pi = exact.dyadic_plu(n, rng, lower=False)
        X, perm = oracle.block_gj_inverse(A, part, pivot=True, sub=sub, leaf_rows=leaf, arity=arity,
                                          return_perm=True)
        assert np.array_equal(X, Ai), f"trial {trial}"
        assert np.array_equal(np.argsort(pi), perm)


@pytest.mark.parametrize("n,b", [(8, 4), (12, 4), (600, 128)])
def test_reversal_permutation_counter_example(n, b):
    """§3: for the reversal permutation every leading block is singular, so the
    unpivoted blockwise method fails; block-row pivoting inverts it exactly."""
    J = np.eye(n)[::-1].copy()
    part = wl.uniform_partition(n, b)
    with pytest.raises(oracle.SingularError):
        oracle.block_gj_inverse(J, part, pivot=False)
    X = oracle.block_gj_inverse(J, part, pivot=True, sub=min(b, 64), leaf_rows=256 if n > 64 else 3)
    assert np.array_equal(X, J)


@pytest.mark.parametrize("pivot", [False, True])
def test_block_diagonal_gives_exact_zero_blocks(pivot):
    rng = np.random.default_rng(5)
    part = [40, 30, 50]
    n = sum(part)
    A = np.zeros((n, n))
    o = 0
    for b in part:
        A[o:o + b, o:o + b] = rng.standard_normal((b, b)) + b * np.eye(b)
        o += b
    X = oracle.block_gj_inverse(A, part, pivot=pivot, sub=16, leaf_rows=32)
    o = 0
    for b in part:
        blk = X[o:o + b, o:o + b]
        assert np.abs(X[o:o + b, :o]).max(initial=0) == 0 and np.abs(X[o:o + b, o + b:]).max(initial=0) == 0
        Xi = np.linalg.inv(A[o:o + b, o:o + b])
        assert np.abs(blk - Xi).max() <= 1e-12 * np.abs(Xi).max()
        o += b


@pytest.mark.parametrize("part", [[64, 64, 64, 64], [200, 56], [100, 156]])
def test_unpivoted_agrees_with_gj_when_no_row_crosses_a_block(part):
    """Column diagonally dominant: partial pivoting never swaps, so pivoting
    only inside blocks loses nothing; the two differ by rounding only."""
    n = sum(part)
    rng = np.random.default_rng(9)
    A = rng.uniform(-1, 1, (n, n))
    A += np.diag(np.abs(A).sum(axis=0) + 1.0)
    Xo = oracle.gj_inverse(A)
    kappa = np.linalg.cond(A)
    for pivot in (False, True):
        X = oracle.block_gj_inverse(A, part, pivot=pivot)
        assert np.abs(X - Xo).max() <= 16 * n * U * kappa * np.abs(Xo).max()


@pytest.mark.parametrize("cond", [1e2, 1e4, 1e6])
def test_pivoted_residual_matches_plain_definition_on_general_inputs(cond):
    """U diag(s) V^T with Haar U, V: tournament block-row pivoting keeps the
    residual of Gauss-Jordan with partial pivoting (within a small factor),
    across many leaves (leaf_rows 32 over 256 rows) and sub-blocks."""
    n = 256
    A = wl.general_haar(n, wl.stream_seed(9, int(np.log10(cond))), cond)
    part = [64, 64, 64, 64]
    Xo = oracle.gj_inverse(A)
    X = oracle.block_gj_inverse(A, part, pivot=True, sub=16, leaf_rows=32, arity=4)
    ro = oracle.residual_stats(A, Xo)["rho"]
    r = oracle.residual_stats(A, X)["rho"]
    assert r <= 4 * ro + 4 * U
    assert np.abs(X - Xo).max() <= 64 * n * U * cond * np.abs(Xo).max()


def test_zero_column_reports_the_same_row_as_gauss_jordan():
    rng = np.random.default_rng(3)
    n = 40
    A = rng.standard_normal((n, n))
    A[:, 23] = 0.0
    with pytest.raises(oracle.SingularError) as e1:
        oracle.gj_inverse(A)
    with pytest.raises(oracle.SingularError) as e2:
        oracle.block_gj_inverse(A, [16, 16, 8], pivot=True, sub=8, leaf_rows=8)
    assert e1.value.row == e2.value.row == 24


def test_two_blocks_unpivoted_is_eq_a_within_rounding():
    """k = 2 without pivoting is Eq. (a) itself (A^-1, the Schur complement and
    its inverse, assembled); on a diagonally dominant input it agrees with
    Gauss-Jordan with partial pivoting to rounding."""
    n, h = 96, 40
    A = wl.diag_dominant(n, 4) - 50 * np.eye(n)
    X = oracle.block_gj_inverse(A, [h, n - h], pivot=False)
    Xo = oracle.gj_inverse(A)
    assert np.abs(X - Xo).max() <= 1e-11 * np.abs(Xo).max()
