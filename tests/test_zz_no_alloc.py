"""binv_invert_noalloc (the entry point that allocates no device memory)
against binv_invert, through the C ABI (needs a GPU).

The no-allocation variant runs the same serial sweep on the library's static
per-device workspace, so its result must equal binv_invert's bitwise (the
lookahead schedule gives bitwise-identical results too) and meet the oracle
tolerance |X - X_GJ| <= 64 n u kappa max|X_GJ|.  Two calls in a row, the
second on a smaller input, check that the workspace left by the first call
does not leak into the second.
"""
import numpy as np
import pytest

import oracle
from paper_2305_11103_amd import workloads as wl

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def _both(A_np, part):
    import torch
    from paper_2305_11103_amd import binv
    A = torch.from_numpy(np.ascontiguousarray(A_np)).cuda()
    Xa = torch.full_like(A, np.nan)
    binv.invert_noalloc(A, part=part, out=Xa)
    Xb = binv.invert(A, part=part)
    torch.cuda.synchronize()
    return Xa.cpu().numpy(), Xb.cpu().numpy()


def _kappa(A):
    s = np.linalg.svd(A, compute_uv=False)
    return s[0] / s[-1]


def test_noalloc_matches_invert_twice_second_smaller(gpu):
    cases = [(1536, [512, 512, 512]), (700, [200, 300, 150, 50])]
    for i, (n, part) in enumerate(cases):
        print(f"noalloc call {i}: n={n} part={part}", flush=True)
        A = wl.diag_dominant(n, wl.stream_seed(1, 900 + i))
        Xa, Xb = _both(A, part)
        assert np.array_equal(Xa, Xb), f"call {i}: differs from binv_invert"
        Xo = oracle.gj_inverse(A)
        tol = 64 * n * U * _kappa(A) * np.max(np.abs(Xo))
        assert np.max(np.abs(Xa - Xo)) <= tol


def test_noalloc_in_place_ragged_and_general(gpu):
    import torch
    from paper_2305_11103_amd import binv
    n, part = 1000, [300, 129, 64, 507]
    A_np = wl.spd_haar(n, wl.stream_seed(2, 901), 1e3)
    A = torch.from_numpy(A_np).cuda()
    W = A.clone()
    binv.invert_noalloc(W, part=part, inplace=True)
    Xb = binv.invert(A, part=part)
    torch.cuda.synchronize()
    assert torch.equal(W, Xb)


def test_noalloc_rejects_beyond_its_workspace(gpu):
    import torch
    from paper_2305_11103_amd import binv
    A = torch.zeros((8192, 8192), dtype=torch.float64, device="cuda")
    with pytest.raises(binv.BinvError, match="static workspace"):
        binv.invert_noalloc(A, block=512, out=torch.empty_like(A))
    B = torch.eye(64, dtype=torch.float64, device="cuda")
    with pytest.raises(binv.BinvError, match="pivot"):
        binv.invert(B, block=64, pivot=True, _noalloc=True)


def test_noalloc_singular_row(gpu):
    import torch
    from paper_2305_11103_amd import binv
    n = 256
    A_np = wl.diag_dominant(n, wl.stream_seed(1, 902))
    A_np[70, :] = 0.0
    A = torch.from_numpy(A_np).cuda()
    info = torch.full((1,), -5, dtype=torch.int64, device="cuda")
    binv.invert_noalloc(A, part=[64] * 4, out=torch.empty_like(A), sync=False, info=info)
    ref = torch.full((1,), -5, dtype=torch.int64, device="cuda")
    binv.invert(A, part=[64] * 4, sync=False, info=ref)
    torch.cuda.synchronize()
    assert int(info.item()) > 0 and int(info.item()) == int(ref.item())
    with pytest.raises(binv.SingularError):
        binv.invert_noalloc(A, part=[64] * 4, out=torch.empty_like(A))
