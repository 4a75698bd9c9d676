"""Pins for the CPU oracle (no GPU).

Each test checks the oracle against something fixed outside it: exact rational
inverses (Leibniz adjugate), integer matrices whose inverse is known in closed
form, the Hilbert inverse formula, the paper's permutation counter-example
(§3), the alternative block formulas Eq. (d) and Eq. (ad) of §3, power-of-two
scaling, and exact Newton-Schulz algebra.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2305_11103_amd import workloads as wl
from tests import exact

U = np.finfo(np.float64).eps / 2  # unit roundoff


def rel_err(X, Y):
    return float(np.linalg.norm(X - Y) / np.linalg.norm(Y))


# --------------------------------------------------------------------------
# O1: Gauss-Jordan with partial pivoting
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_gj_matches_exact_rational_inverse(n):
    rng = np.random.default_rng(100 + n)
    for trial in range(4):
        A = rng.integers(-9, 10, size=(n, n)).astype(np.float64)
        Af = exact.to_frac(A)
        if exact.det_leibniz(Af) == 0:
            continue
        Xe = exact.to_float(exact.inverse_adjugate(Af))
        X = oracle.gj_inverse(A)
        kappa = np.linalg.cond(A, 1)
        assert np.max(np.abs(X - Xe)) <= 8 * n * U * kappa * np.max(np.abs(Xe)) + 1e-300


def test_gj_unit_bidiagonal_gives_all_ones_triangle_exactly():
    n = 37
    L = np.eye(n) - np.eye(n, k=-1)
    X = oracle.gj_inverse(L)
    assert np.array_equal(X, np.tril(np.ones((n, n))))


def test_gj_permutation_gives_transpose_exactly():
    rng = np.random.default_rng(7)
    n = 23
    P = np.eye(n)[rng.permutation(n)]
    assert np.array_equal(oracle.gj_inverse(P), P.T)


def test_gj_diagonal_gives_correctly_rounded_reciprocals():
    d = np.array([3.0, -7.0, 0.1, 1e-3, 12345.678, -2.5])
    X = oracle.gj_inverse(np.diag(d))
    assert np.array_equal(np.diag(X), 1.0 / d)
    assert np.count_nonzero(X - np.diag(np.diag(X))) == 0


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_gj_hilbert_against_closed_form(n):
    H = exact.hilbert(n)
    Hi = exact.hilbert_inverse(n)
    X = oracle.gj_inverse(H)
    kappa = np.linalg.cond(H)
    assert rel_err(X, Hi) <= 20 * n * U * kappa


def test_gj_matches_lapack_on_random():
    A = wl.diag_dominant(120, 5) - 100 * np.eye(120)  # weakly dominant, pivots swap
    X = oracle.gj_inverse(A)
    assert rel_err(X, np.linalg.inv(A)) < 1e-12


def test_gj_power_of_two_scaling_is_bitwise():
    A = wl.spd_gram(40, 11)
    X = oracle.gj_inverse(A)
    for e in (-7, 3, 20):
        Xs = oracle.gj_inverse(np.ldexp(A, e))
        assert np.array_equal(Xs, np.ldexp(X, -e))


def test_gj_involution():
    A = wl.diag_dominant(50, 3)
    assert rel_err(oracle.gj_inverse(oracle.gj_inverse(A)), A) < 1e-14


def test_gj_singular_reports_row():
    A = np.ones((4, 4))
    with pytest.raises(oracle.SingularError) as e:
        oracle.gj_inverse(A)
    assert e.value.row == 2
    with pytest.raises(oracle.SingularError) as e:
        oracle.gj_inverse(np.zeros((3, 3)))
    assert e.value.row == 1


# --------------------------------------------------------------------------
# O2: recursive blockwise inversion by Eq. (a)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 3, 4])
def test_leaf_closed_forms_exact_on_unimodular(n):
    rng = np.random.default_rng(30 + n)
    for _ in range(20):
        A, Ai, _ = exact.unit_lower_times_upper(n, rng, mag=3)
        # permute rows and columns so the leaf sees a general unimodular matrix
        p = rng.permutation(n)
        q = rng.permutation(n)
        B = A[p][:, q]
        Bi = exact.to_float(exact.inverse_adjugate(exact.to_frac(B)))
        assert np.array_equal(oracle.blockwise_inverse(B, [n]), Bi)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_leaf_closed_forms_against_adjugate_on_random(n):
    rng = np.random.default_rng(40 + n)
    for _ in range(20):
        A = rng.uniform(-1, 1, size=(n, n))
        Xe = exact.to_float(exact.inverse_adjugate(exact.to_frac(A)))
        X = oracle.blockwise_inverse(A, [n])
        kappa = np.linalg.cond(A)
        assert np.max(np.abs(X - Xe)) <= 50 * U * kappa * np.max(np.abs(Xe))


@pytest.mark.parametrize("n,part", [(8, [4, 4]), (12, [3, 4, 5]), (16, [2, 2, 3, 4, 5]), (9, None)])
def test_blockwise_exact_on_unit_lu_integer(n, part):
    """All leading blocks and Schur complements are unimodular integer matrices,
    so Eq. (a) applied exactly in FP64 returns the exact integer inverse."""
    rng = np.random.default_rng(n)
    A, Ai, _ = exact.unit_lower_times_upper(n, rng, mag=1)
    assert np.max(np.abs(Ai)) < 2 ** 40
    X = oracle.blockwise_inverse(A, part)
    assert np.array_equal(X, Ai)


@pytest.mark.parametrize("n,part", [
    (64, [16, 16, 16, 16]), (100, [30, 30, 40]), (97, [10] * 9 + [7]), (33, None), (256, [64] * 4),
])
def test_blockwise_agrees_with_gj(n, part):
    A = wl.diag_dominant(n, n)
    X1 = oracle.gj_inverse(A)
    X2 = oracle.blockwise_inverse(A, part)
    assert rel_err(X2, X1) < 50 * n * U


def test_blockwise_spd_conditioned():
    A = wl.spd_haar(96, 2, cond=1e4)
    X2 = oracle.blockwise_inverse(A, [32, 32, 32])
    X1 = oracle.gj_inverse(A)
    assert rel_err(X2, X1) < 1e4 * 96 * U * 10


def test_eq_d_and_eq_ad_agree_with_eq_a():
    """k = 2: Eq. (d) and Eq. (ad) of §3, assembled here from Gauss-Jordan
    inverses of A, D and both Schur complements, give the same inverse."""
    n, ma = 60, 25
    M = wl.diag_dominant(n, 77)
    A, B, C, D = M[:ma, :ma], M[:ma, ma:], M[ma:, :ma], M[ma:, ma:]
    inv = oracle.gj_inverse
    Ai, Di = inv(A), inv(D)
    SA = D - C @ Ai @ B
    SD = A - B @ Di @ C
    SAi, SDi = inv(SA), inv(SD)
    Xd = np.block([[SDi, -SDi @ B @ Di], [-Di @ C @ SDi, Di + Di @ C @ SDi @ B @ Di]])
    Xad = np.block([[SDi, -Ai @ B @ SAi], [-Di @ C @ SDi, SAi]])
    Xa = oracle.blockwise_inverse(M, [ma, n - ma])
    assert rel_err(Xa, Xd) < 1e-13
    assert rel_err(Xa, Xad) < 1e-13


def test_blockwise_block_diagonal_has_exact_zero_off_blocks():
    rng = np.random.default_rng(5)
    part = [7, 5, 9, 4]
    n = sum(part)
    M = np.zeros((n, n))
    off = 0
    blocks = []
    for b in part:
        Bk = rng.uniform(-1, 1, (b, b)) + b * np.eye(b)
        M[off:off + b, off:off + b] = Bk
        blocks.append((off, b, Bk))
        off += b
    X = oracle.blockwise_inverse(M, part)
    mask = np.zeros((n, n), dtype=bool)
    for off, b, Bk in blocks:
        mask[off:off + b, off:off + b] = True
        assert rel_err(X[off:off + b, off:off + b], np.linalg.inv(Bk)) < 1e-14
    assert np.all(X[~mask] == 0.0)


def test_blockwise_block_upper_triangular():
    n, ma = 40, 16
    M = wl.diag_dominant(n, 9)
    M[ma:, :ma] = 0.0
    X = oracle.blockwise_inverse(M, [ma, n - ma])
    assert np.all(X[ma:, :ma] == 0.0)
    A, B, D = M[:ma, :ma], M[:ma, ma:], M[ma:, ma:]
    X12 = -np.linalg.inv(A) @ B @ np.linalg.inv(D)
    assert rel_err(X[:ma, ma:], X12) < 1e-13


@pytest.mark.parametrize("n", [2, 5, 8, 16])
def test_reversal_permutation_counterexample(n):
    """§3: a permutation matrix defeats every leading-block choice, so the
    blockwise method must report a singular pivot; GJ with pivoting inverts it."""
    J = np.eye(n)[::-1].copy()
    with pytest.raises(oracle.SingularError):
        oracle.blockwise_inverse(J, wl.uniform_partition(n, max(1, n // 2)) if n > 2 else [1, 1])
    assert np.array_equal(oracle.gj_inverse(J), J.T)


def test_blockwise_rejects_bad_partition():
    with pytest.raises(ValueError):
        oracle.blockwise_inverse(np.eye(5), [2, 2])


# --------------------------------------------------------------------------
# Partial sweep (state after eliminating a leading block)
# --------------------------------------------------------------------------

def test_partial_sweep_ends():
    A = wl.diag_dominant(30, 1)
    assert np.array_equal(oracle.partial_sweep(A, 0), A)
    assert np.array_equal(oracle.partial_sweep(A, 30), oracle.gj_inverse(A))


def test_partial_sweep_schur_block_inverts_to_trailing_block_of_inverse():
    """Eq. (a): the trailing block of A^-1 is the inverse of the Schur complement."""
    A = wl.diag_dominant(50, 4)
    h = 18
    W = oracle.partial_sweep(A, h)
    S = W[h:, h:]
    Xi = np.linalg.inv(A)
    assert rel_err(np.linalg.inv(S), Xi[h:, h:]) < 1e-13
    # det(A) = det(A11) det(S)
    s1, l1 = np.linalg.slogdet(A)
    s2, l2 = np.linalg.slogdet(A[:h, :h])
    s3, l3 = np.linalg.slogdet(S)
    assert s1 == s2 * s3 and abs(l1 - (l2 + l3)) < 1e-10


def test_partial_sweep_exact_on_unit_lu():
    rng = np.random.default_rng(3)
    A, _, _ = exact.unit_lower_times_upper(10, rng, mag=1)
    W = oracle.partial_sweep(A, 4)
    Af = exact.to_frac(A)
    A11 = [r[:4] for r in Af[:4]]
    A11i = exact.inverse_adjugate(A11)
    # the row panel solves A11 Y = A12 exactly
    Y = [[Fraction(float(x)) for x in row[4:]] for row in W[:4]]
    assert exact.matmul(A11, Y) == [r[4:] for r in Af[:4]]
    assert exact.to_float(A11i).tolist() == W[:4, :4].tolist()
    # the column panel Z satisfies Z A11 = -A21 exactly
    Z = [[Fraction(float(x)) for x in row[:4]] for row in W[4:]]
    assert exact.matmul(Z, A11) == [[-x for x in r[:4]] for r in Af[4:]]


# --------------------------------------------------------------------------
# O3: compensated residual
# --------------------------------------------------------------------------

def test_residual_exact_zero_for_exact_inverse():
    rng = np.random.default_rng(2)
    A, Ai, _ = exact.unit_lower_times_upper(12, rng, mag=2)
    R = oracle.residual_rows(A, Ai)
    assert np.all(R == 0.0)


def test_residual_matches_exact_rational():
    rng = np.random.default_rng(8)
    n = 7
    A = rng.uniform(-1, 1, (n, n)) + 3 * np.eye(n)
    X = np.linalg.inv(A)
    R = oracle.residual_rows(A, X)
    Re = exact.sub(exact.matmul(exact.to_frac(A), exact.to_frac(X)), exact.identity(n))
    Ref = exact.to_float(Re)
    # Dot2 is as accurate as the exact residual rounded once, plus an O(n u^2) term
    bound = 2 * U * np.abs(Ref) + n * n * U * U * (np.abs(A) @ np.abs(X))
    assert np.all(np.abs(R - Ref) <= bound)


def test_residual_rows_subset():
    A = wl.diag_dominant(20, 1)
    X = np.linalg.inv(A)
    Rall = oracle.residual_rows(A, X)
    rows = [3, 0, 19]
    assert np.array_equal(oracle.residual_rows(A, X, rows), Rall[rows])


def test_residual_stats_is_scaled_identity_error():
    """A = I, X = (1 + e) I: A X - I = e I, so rho = ||e I||_F / sqrt(n) = e
    exactly and the largest entry is e (e a power of two: no rounding)."""
    for n in (1, 5, 64):
        for e in (2.0 ** -20, 2.0 ** -40):
            st = oracle.residual_stats(np.eye(n), (1.0 + e) * np.eye(n))
            assert st["rho"] == e and st["rho_max"] == e and st["rows"] == n


def test_residual_stats_sampled_rows_rescale():
    """A = I, X = diag(1 + e_i): row i of A X - I is e_i e_i^T.  Over rows S
    the sampled rho is sqrt((n / |S|) sum_S e_i^2 / n) = sqrt(sum_S e_i^2 / |S|)
    and over all rows sqrt(sum e_i^2 / n); values chosen so both are exact."""
    e = np.array([2.0 ** -10, 0.0, 3 * 2.0 ** -12, 0.0, 2.0 ** -11, 0.0, 0.0, 4 * 2.0 ** -12])
    n = e.size
    X = np.diag(1.0 + e)
    full = oracle.residual_stats(np.eye(n), X)
    assert full["rho"] == np.sqrt(np.sum(e * e) / n)
    rows = [0, 2, 4, 7]
    samp = oracle.residual_stats(np.eye(n), X, rows)
    # sum_S e^2 = (16 + 9 + 4 + 16) 2^-24 = 45 2^-24 over 4 rows
    assert samp["rho"] == np.sqrt(45.0 * 2.0 ** -24 / 4)
    assert samp["rows"] == 4 and samp["rho_max"] == 2.0 ** -10
    assert oracle.residual_stats(np.eye(n), X, rows=list(range(n)))["rho"] == full["rho"]


@pytest.mark.parametrize("n", [3, 5, 7])
def test_residual_stats_matches_exact_rational_norm(n):
    """rho of a perturbed inverse against ||A X - I||_F / sqrt(n) formed in
    exact rationals (the square root taken once in floating point)."""
    rng = np.random.default_rng(30 + n)
    A = rng.integers(-5, 6, size=(n, n)).astype(np.float64) + 6 * np.eye(n)
    X = np.linalg.inv(A) + 2.0 ** -30 * rng.integers(-3, 4, size=(n, n))
    Re = exact.sub(exact.matmul(exact.to_frac(A), exact.to_frac(X)), exact.identity(n))
    fro2 = sum((x * x for row in Re for x in row), Fraction(0))
    rho_exact = float(fro2 / n) ** 0.5
    rho = oracle.residual_stats(A, X)["rho"]
    assert abs(rho - rho_exact) <= 4 * U * rho_exact


# --------------------------------------------------------------------------
# O4: Newton-Schulz step
# --------------------------------------------------------------------------

def test_ns_step_squares_the_residual_exactly_in_rationals():
    rng = np.random.default_rng(9)
    n = 4
    A = rng.integers(-5, 6, (n, n)).astype(np.float64) + 8 * np.eye(n)
    X0 = np.linalg.inv(A) + 1e-3 * rng.uniform(-1, 1, (n, n))
    Af, X0f = exact.to_frac(A), exact.to_frac(X0)
    I = exact.identity(n)
    R0 = exact.sub(I, exact.matmul(Af, X0f))
    X1e = exact.add(X0f, exact.matmul(X0f, R0))
    R1 = exact.sub(I, exact.matmul(Af, X1e))
    assert R1 == exact.matmul(R0, R0)
    X1 = oracle.ns_step(A, X0)
    assert np.max(np.abs(X1 - exact.to_float(X1e))) < 1e-14


def test_ns_step_fixed_point():
    rng = np.random.default_rng(1)
    A, Ai, _ = exact.unit_lower_times_upper(9, rng, mag=1)
    assert np.array_equal(oracle.ns_step(A, Ai), Ai)


def test_ns_converges_quadratically():
    A = wl.spd_haar(64, 3, cond=1e2)
    X = np.linalg.inv(A) * (1 + 1e-4)
    r = [oracle.residual_stats(A, X)["rho"]]
    for _ in range(2):
        X = oracle.ns_step(A, X)
        r.append(oracle.residual_stats(A, X)["rho"])
    assert r[1] < 10 * r[0] ** 2 + 1e-14 and r[2] < 1e-13

