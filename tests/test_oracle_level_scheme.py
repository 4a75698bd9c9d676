"""Pins for the oracle of the paper's parallel algorithm (§5; no GPU).

oracle.level_scheme runs the stepid / loopid schedule of Tables 4 and 5 with
the Eq. (ad) operations of Table 3.  It is checked against the paper's own
tables (golden fixtures), the closed-form flop count n^3 (3 - 1/k) of the
level scheme (the recurrence I(n) = 4 I(n/2) + 1.5 n^3 with I(b) = 2 b^3),
exact inverses of matrices whose every block, Schur complement and product
is exactly representable (Sylvester-Hadamard matrices and their Kronecker
products with unimodular integer blocks, block triangular integer matrices
checked against exact rational inverses), block-diagonal inputs, and
Gauss-Jordan with partial pivoting on SPD inputs within rounding.
"""
from __future__ import annotations

import copy
import os

import numpy as np
import pytest

import oracle
from oracle import level_scheme as ls
from paper_2305_11103_amd import workloads as wl
from tests import exact

U = np.finfo(np.float64).eps / 2
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split(":")
            out[int(k)] = [int(x) for x in v.split()]
    return out


def test_table2_rows():
    for m, blocks in _rows("table2_partitions.txt").items():
        assert ls.table2_partition(m) == blocks


def test_block_counts_of_section_5_1():
    assert ls.block_count(100) == 2 ** 5
    assert ls.block_count(10000) == 2 ** 12
    for m in range(2, 4097):
        p = ls.table2_partition(m)
        assert sum(p) == m and set(p) <= {2, 3, 4}
        assert len(p) & (len(p) - 1) == 0


def test_table4_loopid_rows_and_step_count():
    nk = 8
    assert ls.step_count(nk) == 15
    for s, row in _rows("table4_loopid.txt").items():
        assert ls.loopid(s, nk) == row
    with pytest.raises(ValueError):
        ls.loopid(16, nk)


def test_table5_operations_by_the_text_rules():
    ops = {s: ls.step_ops(s, 16) for s in range(1, 32)}
    assert ops[1] == [("diamond", 0)]
    assert ops[2] == [("arrows", 0, 1)]
    assert ops[3] == [("diamond", 1), ("updown", 1)]
    assert ops[4] == [("arrows", 0, 2)]
    assert ops[5] == [("diamond", 2)]
    assert ops[6] == [("arrows", 2, 1)]
    assert ops[7] == [("diamond", 1), ("updown", 1), ("updown", 2)]
    assert ops[8] == [("arrows", 0, 3)]
    assert ops[10] == [("arrows", 3, 1)]
    assert ops[11] == [("diamond", 1), ("updown", 1)]
    assert ops[31] == [("diamond", 1)] + [("updown", i) for i in range(1, 5)]
    # every T_i is written (arrows) before it is read, and every step starts
    # from M only at the powers of two
    for s, o in ops.items():
        assert (o[0][1] == 0) == (s & (s - 1) == 0 or s == 1) or o[0][0] == "diamond"


@pytest.mark.parametrize("nk,b", [(1, 3), (2, 3), (4, 2), (8, 3), (16, 2), (32, 4)])
def test_flop_count_closed_form(nk, b):
    n = nk * b
    assert ls.level_scheme_flops([b] * nk) == pytest.approx(n ** 3 * (3 - 1 / nk), rel=0, abs=1e-6)
    rng = np.random.default_rng(nk)
    B = rng.standard_normal((n, n))
    _, st = ls.level_scheme_inverse(B @ B.T + n * np.eye(n), [b] * nk, return_state=True)
    assert st.flops == ls.level_scheme_flops([b] * nk)


def sylvester(m):
    H = np.array([[1.0]])
    while H.shape[0] < m:
        H = np.block([[H, H], [H, -H]])
    return H


@pytest.mark.parametrize("m", [4, 8, 16, 32, 64, 128])
def test_hadamard_is_exact(m):
    H = sylvester(m)
    X = ls.level_scheme_inverse(H)
    assert ls.table2_partition(m) == [2] * (m // 2)
    assert np.array_equal(X, H.T / m)


@pytest.mark.parametrize("N", [2, 4, 8, 16])
def test_kronecker_with_unimodular_3x3_blocks_is_exact(N):
    B0 = np.array([[2.0, 1.0, 1.0], [1.0, 1.0, 0.0], [1.0, 0.0, 0.0]])
    d = round(np.linalg.det(B0))
    assert abs(d) == 1
    B0inv = exact.to_float(exact.inverse_adjugate(exact.to_frac(B0)))
    M = np.kron(sylvester(N), B0)
    assert ls.table2_partition(3 * N) == [3] * N
    X = ls.level_scheme_inverse(M)
    assert np.array_equal(X, np.kron(sylvester(N).T / N, B0inv))


@pytest.mark.parametrize("m,seed", [(7, 0), (9, 1), (21, 2), (13, 3)])
@pytest.mark.parametrize("upper", [True, False])
def test_block_triangular_integer_is_exact(m, seed, upper):
    """Unit-triangular integer diagonal blocks (of the Table 2 partition) and
    small integer off-diagonal blocks on one side: every Schur complement is a
    diagonal block, every product an integer, the inverse the exact rational
    (here integer) one."""
    rng = np.random.default_rng(seed)
    part = ls.table2_partition(m)
    M = np.zeros((m, m))
    o = 0
    for b in part:
        L = np.tril(rng.integers(-2, 3, (b, b)), -1) + np.eye(b)
        Ub = np.triu(rng.integers(-2, 3, (b, b)), 1) + np.eye(b)
        M[o:o + b, o:o + b] = L @ Ub
        o += b
    bounds = np.cumsum([0] + part)
    for i in range(len(part)):
        for j in range(len(part)):
            if (j > i) if upper else (j < i):
                M[bounds[i]:bounds[i + 1], bounds[j]:bounds[j + 1]] = rng.integers(-1, 2, (part[i], part[j]))
    Xe = exact.to_float(exact.inverse_rational_gj(exact.to_frac(M)))
    assert np.array_equal(ls.level_scheme_inverse(M), Xe)


def test_block_diagonal_gives_exact_zeros_and_leaf_inverses():
    rng = np.random.default_rng(5)
    m = 21
    part = ls.table2_partition(m)
    M = np.zeros((m, m))
    o = 0
    leaves = []
    for b in part:
        blk = rng.standard_normal((b, b)) + 3 * np.eye(b)
        M[o:o + b, o:o + b] = blk
        leaves.append((o, b, ls.leaf_inverse(blk)))
        o += b
    X = ls.level_scheme_inverse(M)
    mask = np.zeros_like(M, dtype=bool)
    for o, b, inv in leaves:
        assert np.array_equal(X[o:o + b, o:o + b], inv)
        mask[o:o + b, o:o + b] = True
    assert np.all(X[~mask] == 0.0)


def test_leaf_closed_form_against_exact_adjugate():
    rng = np.random.default_rng(9)
    for b in (1, 2, 3, 4):
        for _ in range(20):
            a = rng.integers(-5, 6, (b, b)).astype(float)
            if round(np.linalg.det(a)) == 0:
                continue
            Xe = exact.to_float(exact.inverse_adjugate(exact.to_frac(a)))
            Xl = ls.leaf_inverse(a)
            assert np.max(np.abs(Xl - Xe)) <= 4 * U * np.max(np.abs(Xe)) * max(1, abs(np.linalg.det(a)))


@pytest.mark.parametrize("m", [5, 7, 11, 16, 21, 33, 64, 100])
def test_spd_agrees_with_gauss_jordan(m):
    A = wl.spd_gram(m, wl.stream_seed(4, 500 + m))
    Xo = oracle.gj_inverse(A)
    X = ls.level_scheme_inverse(A)
    kappa = np.linalg.cond(A)
    assert np.max(np.abs(X - Xo)) <= 64 * m * U * kappa * np.max(np.abs(Xo))
    assert oracle.residual_stats(A, X)["rho"] <= 1e-12


def test_singular_leaf_is_reported():
    M = np.eye(8)
    M[2:4, 2:4] = [[1.0, 2.0], [2.0, 4.0]]
    with pytest.raises(ls.Singular):
        ls.level_scheme_inverse(M)


def test_stop_after_any_step_and_resume():
    """stepid as the control variable of a computation with breaks (§5): the
    state after any step, copied and resumed, gives the same inverse."""
    A = wl.spd_gram(21, wl.stream_seed(4, 77))
    ref = ls.level_scheme_inverse(A)
    for s in range(1, ls.step_count(8)):
        st = ls.LevelScheme(A)
        for _ in range(s):
            st.run_step()
        st2 = copy.deepcopy(st)
        while not st2.done():
            st2.run_step()
        assert np.array_equal(st2.Minv, ref)
