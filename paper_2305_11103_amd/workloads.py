"""Seeded synthetic inputs for blockwise inversion.

This module holds no arithmetic of the inversion method.  It only draws
matrices, partitions and request streams, so that the HIP path and the CPU
oracle can be fed identical inputs.

Random numbers come from a counter-based splitmix64 stream (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
value i of stream s is mix(s + (i + 1) * 0x9E3779B97F4A7C15).  Uniforms are
the top 53 bits times 2^-53; normals use Box-Muller on pairs of uniforms.

Workload recipes (all row-major float64):
  diag_dominant(n)          U[-1, 1] entries plus n * I.
  spd_haar(n, cond)         Q diag(s) Q^T, Q Haar-orthogonal (QR of a Gaussian
                            with the sign fix Q diag(sign(diag R))), s_i =
                            10^(log10(cond) u_i) with s_0 = 1 and s_1 = cond so
                            that the 2-norm condition number is exactly cond.
  general_haar(n, cond)     U diag(s) V^T, U and V Haar, s_i geometric from 1
                            down to 1/cond.
  spd_gram(m)               B B^T + 0.1 I with B Gaussian (small SPD matrices).
  spd_gram_batch(sizes)     the same for a whole uneven batch (PCG64 normals).
  *_device variants         the same recipes formed on the GPU from PCG64
                            draws (O'Neill 2014), for orders where the host QR
                            is too slow: spd_haar_device, general_haar_device;
                            householder_conditioned_device for request streams.
  near_equal_partition      floor(m/k) per block, remainder given one by one to
                            the last blocks (the convention of the paper's
                            Table 2 partition examples).
"""
from __future__ import annotations

import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK32 = (1 << 32) - 1


def _mix(z: np.ndarray) -> np.ndarray:
    z = z.copy()
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Values start..start+count-1 of the splitmix64 stream seeded with `seed`."""
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * _GOLDEN
    return _mix(z)


def stream_seed(config: int, index: int) -> int:
    """Per-config, per-item seed: splitmix64 value 0 of seed config*2^32+index."""
    return int(splitmix64((config << 32) + (index & _MASK32), 1)[0])


def uniform(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Uniforms in [0, 1) with 53 random bits."""
    x = splitmix64(seed, count, start)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, count: int) -> np.ndarray:
    """Standard normals by Box-Muller on consecutive uniform pairs."""
    m = (count + 1) // 2
    u = uniform(seed, 2 * m)
    u1 = 1.0 - u[0::2]  # (0, 1]: log stays finite
    u2 = u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * m)
    z[0::2] = r * np.cos(2.0 * math.pi * u2)
    z[1::2] = r * np.sin(2.0 * math.pi * u2)
    return z[:count]


def diag_dominant(n: int, seed: int) -> np.ndarray:
    """Entries i.i.d. uniform[-1, 1] plus n on the diagonal."""
    A = (2.0 * uniform(seed, n * n) - 1.0).reshape(n, n)
    A[np.diag_indices(n)] += float(n)
    return A


def haar_orthogonal(n: int, seed: int) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian, columns sign-fixed."""
    G = normal(seed, n * n).reshape(n, n)
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def spd_haar(n: int, seed: int, cond: float = 1e4) -> np.ndarray:
    """Q diag(s) Q^T with s log-uniform in [1, cond], s_0 = 1, s_1 = cond."""
    Q = haar_orthogonal(n, seed)
    s = 10.0 ** (math.log10(cond) * uniform(seed ^ 0x5A5A5A5A, n))
    s[0] = 1.0
    if n > 1:
        s[1] = cond
    A = (Q * s[None, :]) @ Q.T
    return 0.5 * (A + A.T)


def geometric_singular_values(n: int, cond: float) -> np.ndarray:
    if n == 1:
        return np.ones(1)
    i = np.arange(n, dtype=np.float64)
    return cond ** (-i / (n - 1))


def general_haar(n: int, seed: int, cond: float) -> np.ndarray:
    """U diag(s) V^T, U and V Haar, s geometric from 1 down to 1/cond."""
    U = haar_orthogonal(n, seed)
    V = haar_orthogonal(n, seed ^ 0x3C3C3C3C3C3C)
    s = geometric_singular_values(n, cond)
    return (U * s[None, :]) @ V.T


def spd_gram(m: int, seed: int, shift: float = 0.1) -> np.ndarray:
    """B B^T + shift * I with B an m x m standard Gaussian."""
    B = normal(seed, m * m).reshape(m, m)
    A = B @ B.T
    A = 0.5 * (A + A.T)
    A[np.diag_indices(m)] += shift
    return A


def uniform_partition(n: int, block: int) -> list[int]:
    """Blocks of order `block`; the last one ragged when block does not divide n."""
    if n <= 0:
        return []
    block = max(1, min(block, n))
    k = (n + block - 1) // block
    part = [block] * (k - 1)
    part.append(n - block * (k - 1))
    return part


def near_equal_partition(m: int, k: int) -> list[int]:
    """k blocks of order floor(m/k); the remainder goes one by one to the last blocks."""
    k = max(1, min(k, m))
    base = m // k
    rem = m - base * k
    return [base + (1 if i >= k - rem else 0) for i in range(k)]


def batch_spec(seed: int, count_small: int = 100000, count_large: int = 20000,
               small: int = 5, lo: int = 8, hi: int = 256):
    """Sizes and partitions of the uneven SPD batch: count_small matrices of order
    `small` then count_large of order uniform in [lo, hi]; each split into k
    diagonal blocks, k uniform in {2, 3, 4}, near-equal orders."""
    u = uniform(seed, count_large + count_small + count_large)
    sizes = [small] * count_small + [lo + int(x * (hi - lo + 1)) for x in u[:count_large]]
    ks = [2 + int(x * 3) for x in u[count_large:]]
    parts = [near_equal_partition(m, k) for m, k in zip(sizes, ks)]
    return sizes, parts


def spd_gram_batch(sizes, seed: int, shift: float = 0.1) -> list:
    """B B^T + shift * I for every order in `sizes` (B standard Gaussian), drawn
    in order from one stream of numpy's PCG64 generator (O'Neill 2014; normals
    by its ziggurat) seeded with `seed` -- about ten times faster than the
    splitmix64/Box-Muller stream for the ~5e8 values of the large batch -- and
    formed with one batched product per distinct order."""
    sizes = [int(m) for m in sizes]
    total = sum(m * m for m in sizes)
    z = np.random.Generator(np.random.PCG64(seed & 0xFFFFFFFFFFFFFFFF)).standard_normal(total)
    offs = np.concatenate([[0], np.cumsum([m * m for m in sizes])])
    out = [None] * len(sizes)
    by_size = {}
    for i, m in enumerate(sizes):
        by_size.setdefault(m, []).append(i)
    for m, idx in by_size.items():
        for i in idx:
            B = z[offs[i]:offs[i] + m * m].reshape(m, m)
            G = B @ B.T
            G = 0.5 * (G + G.T)
            G[np.diag_indices(m)] += shift
            out[i] = G
    return out


def general_haar_device(n: int, seed: int, cond: float, device):
    """general_haar on the GPU (torch): Gaussians from PCG64 on the host, QR
    and the product on the device.  For orders where the host QR is too slow."""
    import torch
    g = np.random.Generator(np.random.PCG64(seed & 0xFFFFFFFFFFFFFFFF))
    mats = []
    for _ in range(2):
        G = torch.from_numpy(g.standard_normal((n, n))).to(device)
        Q, R = torch.linalg.qr(G)
        d = torch.sign(torch.diagonal(R))
        d[d == 0] = 1.0
        mats.append(Q * d[None, :])
        del G, R
    U, V = mats
    s = torch.from_numpy(geometric_singular_values(n, cond)).to(device)
    return (U * s[None, :]) @ V.T.contiguous()


def spd_haar_device(n: int, seed: int, cond: float, device):
    """spd_haar's recipe on the GPU (torch): Q from the device QR of a PCG64
    Gaussian (sign-fixed), s = 10^(log10(cond) u) with u from PCG64, s_0 = 1 and
    s_1 = cond; symmetrised.  For orders where the host QR takes tens of seconds."""
    import torch
    g = np.random.Generator(np.random.PCG64(seed & 0xFFFFFFFFFFFFFFFF))
    G = torch.from_numpy(g.standard_normal((n, n))).to(device)
    Q, R = torch.linalg.qr(G)
    d = torch.sign(torch.diagonal(R))
    d[d == 0] = 1.0
    Q = Q * d[None, :]
    del G, R
    s = 10.0 ** (math.log10(cond) * g.random(n))
    s[0] = 1.0
    if n > 1:
        s[1] = cond
    A = (Q * torch.from_numpy(s).to(device)[None, :]) @ Q.T.contiguous()
    return 0.5 * (A + A.T)


def request_stream(count: int, seed: int, lo: int = 5, hi: int = 8192):
    """Order n = round(exp(U[ln lo, ln hi])), condition 10^U[1, 6] and a
    precision tag (fp64 or mixed, probability 1/2) for each request."""
    u = uniform(seed, 3 * count)
    n = np.rint(np.exp(np.log(lo) + u[:count] * (np.log(hi) - np.log(lo)))).astype(np.int64)
    cond = 10.0 ** (1.0 + 5.0 * u[count:2 * count])
    tag = np.where(u[2 * count:] < 0.5, "fp64", "mixed")
    return n, cond, tag


def householder_conditioned_device(n: int, seed: int, cond: float, device, reflectors: int = 4):
    """U diag(pi(s)) V^T with U and V each a product of `reflectors` random
    Householder reflectors and pi a random permutation of geometric singular
    values from 1 to 1/cond (so the condition number is exactly cond).

    Draws: the permutation, then the left reflector vectors u_1..u_r (applied
    in that order, U = H(u_r)...H(u_1)), then the right ones v_1..v_r (V^T =
    H(v_1)...H(v_r)), all from one PCG64 stream.  Formed on the device in
    O(n^2) work as diag(pi(s)) plus a rank-(3r) product: each reflector
    product is written I - W Y^T (compact WY: appending H(u) = I - 2 u u^T to
    I - W Y^T appends the column 2 (u - W Y^T u) to W and u to Y), and
    (I - Wu Yu^T) D (I - Wv Yv^T) = D - Wu (Yu^T D) - (D Wv) Yv^T
    + Wu (Yu^T D Wv) Yv^T is one GEMM of inner dimension 3r."""
    import torch
    g = np.random.Generator(np.random.PCG64(seed & 0xFFFFFFFFFFFFFFFF))
    s = torch.from_numpy(geometric_singular_values(n, cond)[g.permutation(n)]).to(device)
    vecs = []
    for _ in range(2 * reflectors):
        v = torch.from_numpy(g.standard_normal(n)).to(device)
        vecs.append(v / torch.linalg.vector_norm(v))

    def wy(seq):
        W = torch.zeros((n, 0), dtype=torch.float64, device=device)
        Y = torch.zeros((n, 0), dtype=torch.float64, device=device)
        for u in seq:
            w = 2.0 * (u - W @ (Y.T @ u))
            W = torch.cat([W, w[:, None]], dim=1)
            Y = torch.cat([Y, u[:, None]], dim=1)
        return W, Y

    Wu, Yu = wy(reversed(vecs[:reflectors]))   # U = H(u_r) ... H(u_1)
    Wv, Yv = wy(vecs[reflectors:])             # V^T = H(v_1) ... H(v_r)
    P = Yu.T * s[None, :]                      # Yu^T D
    Q = Wv * s[:, None]                        # D Wv
    M = P @ Wv                                 # Yu^T D Wv
    L = torch.cat([-Wu, -Q, Wu @ M], dim=1)
    R = torch.cat([P, Yv.T, Yv.T], dim=0)
    A = L @ R
    A.diagonal().add_(s)
    return A
