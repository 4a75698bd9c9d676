"""The paper's parallel algorithm (§5): bottom-up inversion of a matrix
partitioned into a power-of-two number of diagonal blocks by Eq. (ad),
scheduled by `stepid` and `loopid`.  Test infrastructure: plain numpy in FP64,
slow and literal; only tests/ and the benchmark's CPU leg use it.

What it computes (§5.2, Eq. (adinvprl)): for every "unit" X^l of 2^j
consecutive diagonal blocks, split into halves A^l (first 2^(j-1) blocks) and
D^l (the rest) with off-diagonal blocks B^l and C^l,

    X^-1 = [[ S_D^-1,              -(A^-1 B) S_A^-1 ],
            [ -(D^-1 C) S_D^-1,    S_A^-1           ]],
    S_A = D - C A^-1 B,   S_D = A - B D^-1 C,

built from the inverses of the halves (known from the level below) with the
operations of Table 3:
    ◊  inverse of a diagonal block (closed form, orders <= 4, §5.1)
    →  R = -A^-1 B          ←  L = -D^-1 C
    ∼  S_A = D + C R,  S_D = A + B L
    ↑  X12 = R S_A^-1       ↓  X21 = L S_D^-1
The Schur complements S_A and S_D of a unit are general matrices of 2^(j-1)
blocks, so they are inverted by the same scheme one level down; the
provisional sets T_1 .. T_K (§5.3) hold, per level i, every level-i unit's
L, R and S blocks.  One array per level holds them in the unit's own square,
[[S_D, R], [L, S_A]] (the S blocks at the halves' diagonal positions, where
their inverses belong in X^-1), so T_i is block diagonal over level-i units.

Schedule (§5.3-§5.4, Tables 4 and 5): N_s = 2 N_k - 1 steps; the `loopid` of
step s lists the 1-based positions of the set bits of s, highest first (Table
4: 1 -> [1], 2 -> [2], 3 -> [2, 1], 4 -> [3], ..., N_s -> [n, n-1, .., 1]).
Reading of the step rules (§5.4 text; Table 5's "calculated using" column
contradicts them in rows 5 and 9 and is not followed): with z the last
non-zero loopid entry and p the one before it (absent when z is first),
    source = M if z is the only entry, else the S blocks of T_(p-1);
    z == 1: ◊ on every diagonal block of the source, into M_inv's diagonal;
            then, walking left while entries rise by exactly one (pairs
            (2,1), (3,2), ...), ↑↓ with T_(x-1) for each pair (x, x-1);
    z > 1:  →, ←, ∼ on the level-(z-1) units of the source, into T_(z-1).
M_inv's diagonal band doubles as the store of every ◊ and ↑↓ result, as
§5.4 describes ("stored in the inverted matrix"): after step s the level-j
units whose inversion the step completes hold their inverses there.
"""
from __future__ import annotations

import numpy as np


class Singular(Exception):
    """A diagonal block inverted by ◊ has determinant exactly 0."""


def block_count(m: int) -> int:
    """N_k = 2^(floor(log2 m) - 1) diagonal blocks for an m x m matrix (§5.1);
    one block for m < 4 (orders 2 and 3 are single leaves in Table 2, and
    m = 1 is taken as a single leaf too)."""
    if m < 1:
        raise ValueError("order must be positive")
    if m < 4:
        return 1
    return 1 << (int(np.floor(np.log2(m))) - 1)


def table2_partition(m: int) -> list:
    """Orders of the N_k diagonal blocks (Table 2): floor(m / N_k) each, the
    remainder added one by one to the last blocks (every printed row of
    Table 2 follows this rule: 5 -> [2, 3], 9 -> [2, 2, 2, 3],
    21 -> [2, 2, 2, 3, 3, 3, 3, 3]); orders lie in {2, 3, 4} for m >= 2."""
    k = block_count(m)
    q, r = divmod(m, k)
    return [q + (1 if i >= k - r else 0) for i in range(k)]


def step_count(nk: int) -> int:
    """N_s = 2 * blocksize - 1 (Table 4)."""
    return 2 * nk - 1


def loopid(s: int, nk: int) -> list:
    """The loopid array of step s for nk diagonal blocks (Table 4): the
    1-based positions of the set bits of s from the highest down, padded with
    zeros to log2(nk) + 1 entries."""
    if not 1 <= s <= step_count(nk):
        raise ValueError("step outside the schedule")
    width = int(np.log2(nk)) + 1
    bits = [b + 1 for b in range(s.bit_length() - 1, -1, -1) if (s >> b) & 1]
    return bits + [0] * (width - len(bits))


def step_ops(s: int, nk: int) -> list:
    """The operations of step s by the §5.4 rules, in order: ('diamond', src),
    ('arrows', src, level), ('updown', level); src 0 is the input matrix M,
    src i > 0 the S blocks of T_i."""
    ids = [v for v in loopid(s, nk) if v]
    z = ids[-1]
    src = 0 if len(ids) == 1 else ids[-2] - 1
    if z > 1:
        return [("arrows", src, z - 1)]
    ops = [("diamond", src)]
    x = len(ids) - 1
    while x >= 1 and ids[x - 1] == ids[x] + 1:
        ops.append(("updown", ids[x - 1] - 1))
        x -= 1
    return ops


def leaf_inverse(a: np.ndarray) -> np.ndarray:
    """◊ for an order <= 4 block: the closed form adj(a) / det(a) (§5.1: the
    leaves are inverted by algebraic expressions), cofactors by Laplace
    expansion in plain loops."""
    b = a.shape[0]
    if b == 1:
        if a[0, 0] == 0.0:
            raise Singular()
        return np.array([[1.0 / a[0, 0]]])

    def det(m):
        k = m.shape[0]
        if k == 1:
            return m[0, 0]
        if k == 2:
            return m[0, 0] * m[1, 1] - m[0, 1] * m[1, 0]
        total = 0.0
        for j in range(k):
            minor = np.delete(np.delete(m, 0, axis=0), j, axis=1)
            total += (-1.0) ** j * m[0, j] * det(minor)
        return total

    d = det(a)
    if d == 0.0:
        raise Singular()
    adj = np.empty_like(a)
    for i in range(b):
        for j in range(b):
            minor = np.delete(np.delete(a, j, axis=0), i, axis=1)
            adj[i, j] = (-1.0) ** (i + j) * det(minor)
    return adj / d


class LevelScheme:
    """State of the §5 algorithm for one matrix: the input M, the inverted
    matrix M_inv and the provisional sets T_1 .. T_K, advanced one stepid at
    a time (a computation that may stop after any step and resume, §5 design
    constraints)."""

    def __init__(self, M: np.ndarray, part=None):
        M = np.asarray(M, dtype=np.float64)
        m = M.shape[0]
        self.part = list(part) if part is not None else table2_partition(m)
        nk = len(self.part)
        if sum(self.part) != m or nk & (nk - 1):
            raise ValueError("block orders must sum to m and their count be a power of two")
        self.M = M
        self.nk = nk
        self.K = int(np.log2(nk))
        self.bounds = np.concatenate([[0], np.cumsum(self.part)]).astype(int)
        self.Minv = np.zeros_like(M)
        self.T = [None] + [np.zeros_like(M) for _ in range(self.K)]
        self.step = 0
        self.flops = 0.0

    def _rng(self, b0: int, b1: int) -> slice:
        return slice(self.bounds[b0], self.bounds[b1])

    def _units(self, level: int):
        """(a, d) element ranges of every level-`level` unit's halves."""
        w = 1 << level
        for u in range(self.nk // w):
            b0, bh, b1 = u * w, u * w + w // 2, (u + 1) * w
            yield self._rng(b0, bh), self._rng(bh, b1)

    def _src(self, src: int) -> np.ndarray:
        return self.M if src == 0 else self.T[src]

    def diamond(self, src: int):
        S = self._src(src)
        for j in range(self.nk):
            r = self._rng(j, j + 1)
            self.Minv[r, r] = leaf_inverse(S[r, r])
            self.flops += 2.0 * self.part[j] ** 3

    def arrows(self, src: int, level: int):
        S = self._src(src)
        T = self.T[level]
        for a, d in self._units(level):
            A, B, C, D = S[a, a], S[a, d], S[d, a], S[d, d]
            R = -(self.Minv[a, a] @ B)   # →
            L = -(self.Minv[d, d] @ C)   # ←
            T[a, d] = R
            T[d, a] = L
            T[d, d] = D + C @ R          # ∼  S_A
            T[a, a] = A + B @ L          # ∼  S_D
            na, nd = A.shape[0], D.shape[0]
            self.flops += 4.0 * na * na * nd + 4.0 * nd * nd * na

    def updown(self, level: int):
        T = self.T[level]
        for a, d in self._units(level):
            X12 = T[a, d] @ self.Minv[d, d]   # ↑  R S_A^-1
            X21 = T[d, a] @ self.Minv[a, a]   # ↓  L S_D^-1
            self.Minv[a, d] = X12
            self.Minv[d, a] = X21
            na, nd = X12.shape
            self.flops += 2.0 * na * nd * nd + 2.0 * nd * na * na

    def run_step(self):
        """Advance by one stepid."""
        if self.step >= step_count(self.nk):
            raise ValueError("already complete")
        self.step += 1
        for op in step_ops(self.step, self.nk):
            getattr(self, op[0])(*op[1:])

    def done(self) -> bool:
        return self.step == step_count(self.nk)


def level_scheme_inverse(M: np.ndarray, part=None, return_state: bool = False):
    """M^-1 by the §5 algorithm (all N_s steps).  Raises Singular when a ◊
    meets a block of determinant exactly 0 (the paper then changes the
    partition)."""
    st = LevelScheme(M, part)
    while not st.done():
        st.run_step()
    return (st.Minv, st) if return_state else st.Minv


def level_scheme_flops(part) -> float:
    """Flops of the §5 algorithm for a partition, counted over its schedule
    from the operand shapes alone (2 r c k per r x k by k x c product, 2 b^3
    per ◊ of order b): per unit with halves of na and nd rows, →, ← and ∼
    cost 4 na nd (na + nd) and ↑↓ 2 na nd (na + nd)."""
    nk = len(part)
    bounds = np.concatenate([[0], np.cumsum(part)]).astype(int)
    total = 0.0
    for s in range(1, step_count(nk) + 1):
        for op in step_ops(s, nk):
            if op[0] == "diamond":
                total += sum(2.0 * b ** 3 for b in part)
            else:
                w = 1 << op[-1]
                for u in range(nk // w):
                    na = bounds[u * w + w // 2] - bounds[u * w]
                    nd = bounds[(u + 1) * w] - bounds[u * w + w // 2]
                    total += (4.0 if op[0] == "arrows" else 2.0) * na * nd * (na + nd)
    return total
