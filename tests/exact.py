"""Exact rational arithmetic used to pin the oracle (tests only).

Nothing here shares code with the oracle: determinants come from the Leibniz
permutation sum and inverses from the adjugate (Cramer's rule), both in Python
Fractions, so they are exact and independent of any elimination order.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def to_frac(A) -> list[list[Fraction]]:
    A = np.asarray(A, dtype=np.float64)
    return [[Fraction(float(x)) for x in row] for row in A]


def _perm_sign(p) -> int:
    s = 1
    p = list(p)
    for i in range(len(p)):
        while p[i] != i:
            j = p[i]
            p[i], p[j] = p[j], p[i]
            s = -s
    return s


def det_leibniz(M) -> Fraction:
    n = len(M)
    if n == 0:
        return Fraction(1)
    total = Fraction(0)
    for p in itertools.permutations(range(n)):
        term = Fraction(_perm_sign(p))
        for i in range(n):
            term *= M[i][p[i]]
            if term == 0:
                break
        total += term
    return total


def minor(M, i, j):
    return [row[:j] + row[j + 1:] for k, row in enumerate(M) if k != i]


def inverse_adjugate(M) -> list[list[Fraction]]:
    """Exact inverse by adjugate / determinant (n <= 7 keeps this quick)."""
    n = len(M)
    d = det_leibniz(M)
    if d == 0:
        raise ZeroDivisionError("singular")
    if n == 1:
        return [[1 / M[0][0]]]
    inv = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            cof = det_leibniz(minor(M, i, j)) * (1 if (i + j) % 2 == 0 else -1)
            inv[j][i] = cof / d
    return inv


def inverse_rational_gj(M) -> list[list[Fraction]]:
    """Exact inverse by Gauss-Jordan elimination in rationals (any nonzero
    pivot: exact arithmetic needs no pivoting for accuracy); O(n^3)."""
    n = len(M)
    W = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(M)]
    for c in range(n):
        r = next((i for i in range(c, n) if W[i][c] != 0), None)
        if r is None:
            raise ZeroDivisionError("singular")
        W[c], W[r] = W[r], W[c]
        q = 1 / W[c][c]
        W[c] = [x * q for x in W[c]]
        for i in range(n):
            if i != c and W[i][c] != 0:
                f = W[i][c]
                W[i] = [a - f * b for a, b in zip(W[i], W[c])]
    return [row[n:] for row in W]


def matmul(A, B):
    n, q, p = len(A), len(B), len(B[0])
    return [[sum((A[i][t] * B[t][j] for t in range(q)), Fraction(0)) for j in range(p)] for i in range(n)]


def identity(n):
    return [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]


def sub(A, B):
    return [[a - b for a, b in zip(ra, rb)] for ra, rb in zip(A, B)]


def add(A, B):
    return [[a + b for a, b in zip(ra, rb)] for ra, rb in zip(A, B)]


def to_float(M) -> np.ndarray:
    return np.array([[float(x) for x in row] for row in M], dtype=np.float64)


def unit_lower_times_upper(n: int, rng, mag: int = 2):
    """A = L U with L unit lower and U unit upper triangular small-integer
    matrices: every leading principal minor is 1, so every leading block and
    every Schur complement is unimodular and the exact inverse is integral."""
    L = np.eye(n, dtype=np.int64)
    U = np.eye(n, dtype=np.int64)
    for i in range(n):
        for j in range(i):
            L[i, j] = rng.integers(-mag, mag + 1)
            U[j, i] = rng.integers(-mag, mag + 1)
    A = L @ U
    # exact inverse U^-1 L^-1 by integer back substitution
    def tri_inv_lower(T):
        m = T.shape[0]
        Ti = np.eye(m, dtype=object)
        for j in range(m):
            for i in range(j + 1, m):
                Ti[i, j] = -sum(int(T[i, t]) * Ti[t, j] for t in range(j, i))
        return Ti
    Li = tri_inv_lower(L)
    Ui = tri_inv_lower(U.T).T
    Ai = np.dot(Ui, Li)
    return A.astype(np.float64), np.array(Ai, dtype=np.float64), np.array(Ai, dtype=object)


def hilbert(n: int) -> np.ndarray:
    return np.array([[1.0 / (i + j + 1) for j in range(n)] for i in range(n)])


def hilbert_inverse(n: int) -> np.ndarray:
    """Closed-form integer inverse of the order-n Hilbert matrix (1-based i, j):
    (-1)^(i+j) (i+j-1) C(n+i-1, n-j) C(n+j-1, n-i) C(i+j-2, i-1)^2."""
    from math import comb
    out = np.empty((n, n))
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            v = (-1) ** (i + j) * (i + j - 1) * comb(n + i - 1, n - j) * comb(n + j - 1, n - i) * comb(i + j - 2, i - 1) ** 2
            out[i - 1, j - 1] = v
    return out


def _tri_inv_frac(T, lower: bool):
    """Exact inverse of a triangular Fraction matrix by substitution."""
    n = len(T)
    X = [[Fraction(0)] * n for _ in range(n)]
    for j in range(n):
        rng_i = range(j, n) if lower else range(j, -1, -1)
        for i in rng_i:
            if i == j:
                X[i][j] = 1 / T[i][i]
                continue
            ks = range(j, i) if lower else range(i + 1, j + 1)
            X[i][j] = -sum((T[i][k] * X[k][j] for k in ks), Fraction(0)) / T[i][i]
    return X


def dyadic_plu(n: int, rng, lower: bool = True):
    """A = Pi L U with small dyadic factors and its exact inverse.

    L: unit lower triangular, off-diagonal entries from {-1/2, 0, 1/2} (so
    |l| < 1 and partial pivoting meets a unique largest entry in every column:
    it recovers Pi, L and U exactly); with lower=False, L = I.  U: upper
    triangular, diagonal from {+-1, +-2}, off-diagonal from {-1, 0, 1}.  Pi: a
    random row permutation (A[i] = (L U)[pi[i]]).  Every value met by
    elimination in the pivot order is a short dyadic rational, so FP64
    elimination in that order is exact.  Returns (A, exact inverse as floats,
    pi)."""
    half = Fraction(1, 2)
    L = [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    Uf = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            if lower and j < i:
                L[i][j] = half * int(rng.integers(-1, 2))
            if j > i:
                Uf[i][j] = Fraction(int(rng.integers(-1, 2)))
        Uf[i][i] = Fraction(int(rng.choice([-2, -1, 1, 2])))
    pi = rng.permutation(n)
    LU = matmul(L, Uf)
    A = [LU[int(pi[i])] for i in range(n)]
    # A^-1 = U^-1 L^-1 Pi^T: column pi[i] of (LU)^-1 is column i of A^-1
    LUi = matmul(_tri_inv_frac(Uf, lower=False), _tri_inv_frac(L, lower=True))
    Ai = [[LUi[r][int(pi[c])] for c in range(n)] for r in range(n)]
    Af, Aif = to_float(A), to_float(Ai)
    assert all(Fraction(float(Af[i, j])) == A[i][j] for i in range(n) for j in range(n))
    assert all(Fraction(float(Aif[i, j])) == Ai[i][j] for i in range(n) for j in range(n))
    return Af, Aif, pi
