"""FP64 CPU oracle for blockwise matrix inversion (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product library never loads it, and the oracle
never imports the product package: the two share no code.  Inputs reach both
sides from the seeded generators, which hold none of the method's arithmetic.

The arithmetic lives in ``oracle.c`` (plain C, FP64); this module only builds
it with gcc and marshals numpy arrays through ctypes.

  gj_inverse(A)                 Gauss-Jordan with partial pivoting (first
                                maximum wins): the plain definition of A^-1.
  blockwise_inverse(A, part)    Recursive Eq. (a) of §3 in the product order of
                                invertor_by_a (§4.1), closed-form leaves of
                                order <= 4 (§5.1).
  partial_sweep(A, h)           State after eliminating the leading h x h
                                block (first half of Eq. (a)).
  residual_rows(A, X, rows)     Rows of A X - I with compensated dot products.
  residual_stats(A, X)          rho = ||AX-I||_F / sqrt(n) and max |AX-I|.
  block_gj_inverse(A, part, pivot)
                                Block Gauss-Jordan over the partition (Eq. (a)
                                unrolled, §4.2): without pivoting across blocks
                                (pivot=False) or with block-row pivoting by
                                tournament selection (pivot=True).
  ns_step(A, X)                 One Newton-Schulz step X + X (I - A X).
  matmul(A, B)                  Plain product.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_oracle.so")
_lib = None


class SingularError(ValueError):
    """Raised when a pivot or leaf determinant is exactly zero."""

    def __init__(self, row: int):
        super().__init__(f"singular: exactly-zero pivot at (1-based) row {row}")
        self.row = int(row)


def build(force: bool = True) -> str:
    """Compile oracle.c into _oracle.so with gcc (no HIP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32 = ctypes.c_int32
    lib.orc_gj_inverse.argtypes = [i64, P, P]
    lib.orc_gj_inverse.restype = i64
    lib.orc_blockwise_inverse.argtypes = [i64, P, i32, P, P]
    lib.orc_blockwise_inverse.restype = i64
    lib.orc_partial_sweep.argtypes = [i64, P, i64, P]
    lib.orc_partial_sweep.restype = i64
    lib.orc_residual_rows.argtypes = [i64, P, P, i64, P, P]
    lib.orc_residual_rows.restype = None
    lib.orc_ns_step.argtypes = [i64, P, P, P]
    lib.orc_ns_step.restype = i64
    lib.orc_matmul.argtypes = [i64, i64, i64, P, P, P]
    lib.orc_matmul.restype = None
    lib.orc_block_gj.argtypes = [i64, P, i32, P, i32, i32, i32, i32, P, P]
    lib.orc_block_gj.restype = i64
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _square(A) -> np.ndarray:
    A = _f64(A)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError(f"expected a square matrix, got shape {A.shape}")
    return A


def gj_inverse(A) -> np.ndarray:
    A = _square(A)
    n = A.shape[0]
    X = np.empty_like(A)
    info = _load().orc_gj_inverse(n, _ptr(A), _ptr(X))
    if info > 0:
        raise SingularError(info)
    if info < 0:
        raise MemoryError("oracle allocation failed")
    return X


def blockwise_inverse(A, part=None) -> np.ndarray:
    A = _square(A)
    n = A.shape[0]
    X = np.zeros_like(A)
    if part is None:
        p = None
        k = 0
    else:
        p = np.ascontiguousarray(part, dtype=np.int32)
        k = int(p.size)
        if k == 0 or int(p.sum()) != n or (p <= 0).any():
            raise ValueError(f"partition {list(p)} does not split order {n}")
    info = _load().orc_blockwise_inverse(n, _ptr(A), k, _ptr(p) if p is not None else None, _ptr(X))
    if info > 0:
        raise SingularError(info)
    if info < 0:
        raise ValueError("invalid partition or allocation failure")
    return X


def partial_sweep(A, h: int) -> np.ndarray:
    A = _square(A)
    n = A.shape[0]
    if not 0 <= h <= n:
        raise ValueError("h out of range")
    W = np.zeros_like(A)
    info = _load().orc_partial_sweep(n, _ptr(A), int(h), _ptr(W))
    if info > 0:
        raise SingularError(info)
    if info < 0:
        raise MemoryError("oracle allocation failed")
    return W


def residual_rows(A, X, rows=None) -> np.ndarray:
    A = _square(A)
    X = _square(X)
    n = A.shape[0]
    if rows is None:
        rows = np.arange(n, dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if rows.size and (rows.min() < 0 or rows.max() >= n):
        raise ValueError("row index out of range")
    R = np.empty((rows.size, n), dtype=np.float64)
    _load().orc_residual_rows(n, _ptr(A), _ptr(X), int(rows.size), _ptr(rows), _ptr(R))
    return R


def residual_stats(A, X, rows=None) -> dict:
    """rho = ||AX - I||_F / sqrt(n) (over the chosen rows, rescaled to n rows
    when sampling), and max |AX - I| over those rows."""
    A = _square(A)
    n = A.shape[0]
    R = residual_rows(A, X, rows)
    m = R.shape[0]
    if m == 0:
        return {"rho": 0.0, "rho_max": 0.0, "rows": 0}
    fro2 = float(np.sum(R * R))
    rho = np.sqrt(fro2 * (n / m) / n)
    return {"rho": float(rho), "rho_max": float(np.max(np.abs(R))), "rows": int(m)}


def block_gj_inverse(A, part=None, pivot: bool = False, sub: int = 64, leaf_rows: int = 256,
                     arity: int = 4, return_perm: bool = False):
    """Block Gauss-Jordan over the diagonal blocks `part` (one block of order n
    when None), the two readings of oracle.c's orc_block_gj: pivot=False pivots
    only inside pivot blocks (leaves of `sub` rows for blocks above 128);
    pivot=True picks each block's pivot rows among all rows below by tournament
    selection (`sub`-wide strips, leaves of `leaf_rows` rows, `arity` nodes per
    merge).  return_perm: also the final row order (original row at each
    position)."""
    A = _square(A)
    n = A.shape[0]
    X = np.zeros_like(A)
    if part is None:
        p = None
        k = 0
    else:
        p = np.ascontiguousarray(part, dtype=np.int32)
        k = int(p.size)
        if k == 0 or int(p.sum()) != n or (p <= 0).any():
            raise ValueError(f"partition {list(p)} does not split order {n}")
    perm = np.zeros(max(n, 1), dtype=np.int64)
    info = _load().orc_block_gj(n, _ptr(A), k, _ptr(p) if p is not None else None, int(bool(pivot)), int(sub),
                                int(leaf_rows), int(arity), _ptr(X), _ptr(perm))
    if info > 0:
        raise SingularError(info)
    if info < 0:
        raise ValueError("invalid arguments or allocation failure")
    return (X, perm[:n]) if return_perm else X


def ns_step(A, X) -> np.ndarray:
    A = _square(A)
    X = _square(X)
    n = A.shape[0]
    Y = np.empty_like(A)
    _load().orc_ns_step(n, _ptr(A), _ptr(X), _ptr(Y))
    return Y


def matmul(A, B) -> np.ndarray:
    A = _f64(A)
    B = _f64(B)
    m, q = A.shape
    q2, p = B.shape
    if q != q2:
        raise ValueError("inner dimensions differ")
    C = np.empty((m, p), dtype=np.float64)
    _load().orc_matmul(m, q, p, _ptr(A), _ptr(B), _ptr(C))
    return C
