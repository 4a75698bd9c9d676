"""Input generators (not the method): recipes agree with their plain
definitions."""
import numpy as np


def test_householder_generator_matches_explicit_reflectors():
    """Input recipe check (not the method): the compact-WY formation of the
    serving workload's matrices equals applying the reflectors one by one, and
    its singular values are exactly the drawn ones."""
    import torch
    from paper_2305_11103_amd import workloads as w
    n, seed, cond = 37, 1234, 1e5
    A = w.householder_conditioned_device(n, seed, cond, "cpu").numpy()
    g = np.random.Generator(np.random.PCG64(seed))
    s = w.geometric_singular_values(n, cond)[g.permutation(n)]
    B = np.diag(s)
    us = [g.standard_normal(n) for _ in range(8)]
    us = [u / np.linalg.norm(u) for u in us]
    for u in us[:4]:
        B = B - 2.0 * np.outer(u, u @ B)
    for v in us[4:]:
        B = B - 2.0 * np.outer(B @ v, v)
    assert np.max(np.abs(A - B)) <= 1e-14
    sv = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(np.sort(sv), np.sort(s), rtol=1e-12, atol=0)
