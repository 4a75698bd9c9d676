"""Out-of-core inversion (binv_invert_host; GPU): the matrix stays in host
memory and only panels and row slabs visit the device.  The result must be
bitwise binv_invert's (the same kernels apply the same arithmetic to every
element, whatever rows a launch covers) and meet the oracle's tolerance."""
import numpy as np
import pytest

import oracle
from paper_2305_11103_amd import workloads as wl

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def panels_bytes(n, b):
    return 8 * (4 * b * n + b * b + 4 * (64 * b + 4096)) + 256


@pytest.mark.parametrize("n,part,rows,pinned", [
    (2048, [512] * 4, 256, True),     # 8 slabs of 256 rows
    (2048, [512] * 4, 200, False),    # slabs of 128 rows, pageable host memory
    (1000, [300, 200, 500], 5, True),  # ragged slabs of 5 rows, ragged partition
    (777, [7] * 111, 100, False),
])
def test_out_of_core_is_bitwise_in_core(gpu, n, part, rows, pinned):
    import torch
    from paper_2305_11103_amd import binv
    A_np = wl.spd_haar(n, wl.stream_seed(2, 950 + n), 1e3) if n >= 1000 else wl.diag_dominant(n, 951)
    ref = binv.invert(torch.from_numpy(A_np).cuda(), part=part).cpu().numpy()
    W = torch.from_numpy(A_np.copy())
    if pinned:
        W = W.pin_memory()
    print(f"out of core n={n} slab rows {rows} pinned {pinned}", flush=True)
    binv.invert_host(W if pinned else W.numpy(), panels_bytes(n, max(part)) + rows * 16 * n, part=part)
    X = W.numpy()
    assert np.array_equal(X, ref)
    Xo = oracle.gj_inverse(A_np)
    assert np.max(np.abs(X - Xo)) <= 64 * n * U * np.linalg.cond(A_np) * np.max(np.abs(Xo))


def test_out_of_core_errors(gpu):
    import torch
    from paper_2305_11103_amd import binv
    n = 512
    A = wl.diag_dominant(n, 952)
    with pytest.raises(binv.BinvError):  # not even one row of slab fits
        binv.invert_host(A.copy(), panels_bytes(n, 128), block=128)
    bad = A.copy()
    bad[:, 300] = 0.0
    with pytest.raises(binv.SingularError) as e_host:
        binv.invert_host(bad.copy(), 64 << 20, block=128)  # (W is overwritten in place)
    info = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(binv.SingularError):  # the same row in core
        binv.invert(torch.from_numpy(bad).cuda(), block=128, info=info)
    assert int(info.item()) > 0 and f"row {int(info.item())}" in str(e_host.value)
    W0 = np.zeros((0, 0))
    binv.invert_host(W0, 1 << 20)
