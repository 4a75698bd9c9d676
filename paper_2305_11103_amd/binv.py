"""Python binding of the blockwise inversion library (argument marshalling only).

Every step of the inversion runs in the HIP kernels of ``libbinv.so``; this
module checks tensor shapes, passes device pointers and the current HIP stream
through ctypes, and turns status codes into exceptions.  PyTorch supplies the
device memory and the stream.  If the library is missing the import of the
binding fails: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbinv.so")

BINV_OK = 0
BINV_E_INVALID = 1
BINV_E_SINGULAR = 2
BINV_E_NOMEM = 3
BINV_E_NOCONVERGE = 4
BINV_E_HIP = 5
BINV_E_BUSY = 6
BINV_E_NOTFOUND = 7
BINV_PREC_FP64 = 0
BINV_PREC_MIXED_F32 = 1
BINV_F_SYNC = 1
BINV_F_NO_LOOKAHEAD = 2

# every exported entry point of include/binv.h
EXPORTS = ("binv_create", "binv_destroy", "binv_invert", "binv_invert_noalloc", "binv_sweep_steps", "binv_invert_host",
           "binv_set_timing", "binv_get_timing", "binv_lookahead_cus",
           "binv_invert_mixed", "binv_residual", "binv_residual_matrix",
           "binv_batch_create", "binv_batch_destroy", "binv_batch_query", "binv_invert_batched",
           "binv_batch_tune", "binv_batch_shape", "binv_batch_residual",
           "binv_invert_batched_levels", "binv_level_partition",
           "binv_server_create", "binv_submit", "binv_poll", "binv_next_done", "binv_server_stats",
           "binv_server_destroy",
           "binv_last_error", "binv_version")
BINV_F_GRAPH = 4
BINV_F_REFINE_FROM_FP64 = 8
BINV_F_SAMPLED_CHECK = 16
BINV_F_PIVOT = 32
BINV_F_LOOKAHEAD = 64
BINV_RESID_ESTIMATE = 1
BINV_RESID_COMPENSATED = 2
BINV_SERVER_STRICT_PRECISION = 1
BINV_SERVER_FULL_CHECK = 2
PHASES = ("pivot", "row", "schur", "other", "band", "small", "tail")
TIER_SHAPES = (4, 4, 4, 4, 3, 2)  # launch shapes per register tier (autotuned)
TIER_LIMITS = (8, 16, 32, 64, 128, 192)  # largest order of each register tier


class BinvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"binv status {status}: {msg}")
        self.status = status


class SingularError(BinvError):
    pass


class _Timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 7), ("launches", ctypes.c_int64 * 7), ("flops", ctypes.c_double * 7)]


class _Info(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("rho_steps", ctypes.c_double * 8), ("refine_steps", ctypes.c_int32),
                ("fell_back", ctypes.c_int32), ("converged", ctypes.c_int32), ("sampled", ctypes.c_int32),
                ("rho_count", ctypes.c_int32)]


class _Times(ctypes.Structure):
    _fields_ = [("queue_ms", ctypes.c_double), ("total_ms", ctypes.c_double)]


class _Opts(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32),
        ("part", ctypes.POINTER(ctypes.c_int32)),
        ("block", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]


_lib = None


def load_library():
    """Load libbinv.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: build it with paper_2305_11103_amd._build.build_library()")
    # torch ships its own HIP runtime; loading torch first makes the library
    # bind to that same runtime (its soname satisfies the library's), so the
    # tensors and streams passed in belong to the runtime the library calls.
    # Loaded the other way round, the process would hold two runtimes.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.binv_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
    lib.binv_create.restype = ctypes.c_int
    lib.binv_destroy.argtypes = [P]
    lib.binv_destroy.restype = ctypes.c_int
    lib.binv_invert.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, P, ctypes.c_int64,
                                ctypes.POINTER(_Opts), P, P]
    lib.binv_invert.restype = ctypes.c_int
    lib.binv_invert_noalloc.argtypes = lib.binv_invert.argtypes
    lib.binv_invert_noalloc.restype = ctypes.c_int
    lib.binv_sweep_steps.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, ctypes.POINTER(_Opts), ctypes.c_int32,
                                     ctypes.c_int32, P, P]
    lib.binv_sweep_steps.restype = ctypes.c_int
    lib.binv_invert_host.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, ctypes.POINTER(_Opts), ctypes.c_size_t, P,
                                     ctypes.POINTER(ctypes.c_int64)]
    lib.binv_invert_host.restype = ctypes.c_int
    lib.binv_set_timing.argtypes = [P, ctypes.c_uint32]
    lib.binv_set_timing.restype = ctypes.c_int
    lib.binv_get_timing.argtypes = [P, ctypes.POINTER(_Timing)]
    lib.binv_get_timing.restype = ctypes.c_int
    lib.binv_lookahead_cus.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
    lib.binv_lookahead_cus.restype = ctypes.c_int
    lib.binv_invert_mixed.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, P, ctypes.c_int64, ctypes.POINTER(_Opts),
                                      ctypes.c_double, ctypes.c_int32, P, ctypes.POINTER(_Info)]
    lib.binv_invert_mixed.restype = ctypes.c_int
    lib.binv_residual.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_uint32, P,
                                  ctypes.POINTER(ctypes.c_double)]
    lib.binv_residual.restype = ctypes.c_int
    lib.binv_residual_matrix.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, P, ctypes.c_int64, P, ctypes.c_int64,
                                         P, ctypes.POINTER(ctypes.c_double)]
    lib.binv_residual_matrix.restype = ctypes.c_int
    lib.binv_server_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.c_int32, ctypes.c_uint32,
                                       ctypes.POINTER(P)]
    lib.binv_server_create.restype = ctypes.c_int
    lib.binv_submit.argtypes = [P, ctypes.c_int64, P, ctypes.c_int, ctypes.c_int32, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_uint64)]
    lib.binv_submit.restype = ctypes.c_int
    lib.binv_poll.argtypes = [P, ctypes.c_uint64, P, ctypes.c_int, ctypes.POINTER(_Info), ctypes.POINTER(_Times)]
    lib.binv_poll.restype = ctypes.c_int
    lib.binv_next_done.argtypes = [P, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64)]
    lib.binv_next_done.restype = ctypes.c_int
    lib.binv_server_stats.argtypes = [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                      ctypes.POINTER(ctypes.c_int64)]
    lib.binv_server_stats.restype = ctypes.c_int
    lib.binv_server_destroy.argtypes = [P]
    lib.binv_server_destroy.restype = ctypes.c_int
    lib.binv_batch_create.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.POINTER(P)]
    lib.binv_batch_create.restype = ctypes.c_int
    lib.binv_batch_destroy.argtypes = [P]
    lib.binv_batch_destroy.restype = ctypes.c_int
    lib.binv_batch_query.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_double)]
    lib.binv_batch_query.restype = ctypes.c_int
    lib.binv_invert_batched.argtypes = [P, P, P, P, ctypes.c_uint32, P]
    lib.binv_invert_batched.restype = ctypes.c_int
    lib.binv_batch_tune.argtypes = [P, P, P, P, ctypes.c_int32, P, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_double)]
    lib.binv_batch_tune.restype = ctypes.c_int
    lib.binv_batch_shape.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.binv_batch_shape.restype = ctypes.c_int
    lib.binv_batch_residual.argtypes = [P, P, P, P, P]
    lib.binv_batch_residual.restype = ctypes.c_int
    lib.binv_invert_batched_levels.argtypes = [P, P, P, P, ctypes.c_uint32, P]
    lib.binv_invert_batched_levels.restype = ctypes.c_int
    lib.binv_level_partition.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32)]
    lib.binv_level_partition.restype = ctypes.c_int
    lib.binv_last_error.argtypes = []
    lib.binv_last_error.restype = ctypes.c_char_p
    lib.binv_version.argtypes = []
    lib.binv_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def last_error() -> str:
    """The library's thread-local message for the last non-OK status."""
    return load_library().binv_last_error().decode(errors="replace")


def _check(status: int):
    if status == BINV_OK:
        return
    msg = load_library().binv_last_error().decode(errors="replace")
    if status == BINV_E_SINGULAR:
        raise SingularError(status, msg)
    raise BinvError(status, msg)


class Context:
    """A library context on one device (owns the panel workspace)."""

    def __init__(self, device: int = 0):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.binv_create(ctypes.byref(h), int(device)))
        self._h = h
        self.device = int(device)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().binv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_timing(self, phases=()):
        """Time every later top-level launch of the named phases with events."""
        mask = 0
        for p in phases:
            mask |= 1 << PHASES.index(p)
        _check(load_library().binv_set_timing(self._h, mask))

    def lookahead_cus(self) -> int:
        """CUs reserved for the lookahead's pivot chain (0: masks refused)."""
        r = ctypes.c_int32()
        _check(load_library().binv_lookahead_cus(self._h, ctypes.byref(r)))
        return r.value

    def get_timing(self) -> dict:
        """Wait for the recorded events; return {phase: (total_ms, launches, flops)}."""
        t = _Timing()
        _check(load_library().binv_get_timing(self._h, ctypes.byref(t)))
        return {p: (t.ms[i], int(t.launches[i]), t.flops[i]) for i, p in enumerate(PHASES)}


_ctx: dict[int, Context] = {}


def default_context(device: int = 0) -> Context:
    if device not in _ctx:
        _ctx[device] = Context(device)
    return _ctx[device]


def _opts(part=None, block=None, sync=False, lookahead=None, pivot=False):
    o = _Opts()
    keep = None
    if part is not None:
        arr = (ctypes.c_int32 * len(part))(*[int(x) for x in part])
        keep = arr
        o.k = len(part)
        o.part = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
    else:
        o.k = 0
        o.part = None
    o.block = int(block) if block else 0
    # lookahead: None lets the library choose by order, True / False force it
    look = 0 if lookahead is None else (BINV_F_LOOKAHEAD if lookahead else BINV_F_NO_LOOKAHEAD)
    o.flags = (BINV_F_SYNC if sync else 0) | look | (BINV_F_PIVOT if pivot else 0)
    return o, keep


def _stream_handle(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def invert(A, part=None, block=None, out=None, inplace=False, sync=True, info=None, ctx=None, lookahead=None,
           pivot=False, graph=False, _noalloc=False):
    """Invert the square float64 CUDA tensor A by blockwise (Schur-complement)
    inversion over the diagonal blocks `part` (or uniform blocks of `block`).

    out:     optional float64 tensor for X (row stride >= n, unit column stride).
    inplace: overwrite A with its inverse.
    sync:    wait for completion and raise SingularError on an exactly-zero pivot.
    lookahead: form the next block's pivot and panels on a side stream while
             the current trailing update runs (True: BINV_F_LOOKAHEAD; False:
             BINV_F_NO_LOOKAHEAD; None: the library's choice, on from n = 2048).
             Results are bitwise identical either way.
    pivot:   block-row pivoting (BINV_F_PIVOT): each pivot block's rows are
             chosen among all rows not yet used as pivots.
    graph:   replay the call's launch sequence from a HIP graph cached in the
             context (BINV_F_GRAPH; captured on the first call of a key).
    info:    optional int64 CUDA tensor of one element receiving the singular row.
    """
    import torch

    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError(f"expected a square matrix, got {tuple(A.shape)}")
    if A.dtype != torch.float64 or not A.is_cuda:
        raise ValueError("A must be a float64 tensor on a GPU")
    if A.stride(1) != 1:
        raise ValueError("A must have unit column stride (row-major rows)")
    n = A.shape[0]
    if inplace:
        X = A
    elif out is not None:
        if out.shape != A.shape or out.dtype != torch.float64 or out.stride(1) != 1 or out.device != A.device:
            raise ValueError("out must be a float64 tensor like A")
        X = out
    else:
        X = torch.empty_like(A, memory_format=torch.contiguous_format)
    dev = A.device.index if A.device.index is not None else torch.cuda.current_device()
    ctx = ctx or default_context(dev)
    o, keep = _opts(part, block, sync, lookahead, pivot)
    if graph:
        o.flags |= BINV_F_GRAPH
    info_ptr = None
    if info is not None:
        if info.dtype != torch.int64 or not info.is_cuda or info.numel() < 1:
            raise ValueError("info must be an int64 CUDA tensor with one element")
        info_ptr = ctypes.c_void_p(info.data_ptr())
    lda = A.stride(0) if n > 0 else 1
    ldx = X.stride(0) if n > 0 else 1
    lib = load_library()
    fn = lib.binv_invert_noalloc if _noalloc else lib.binv_invert
    with torch.cuda.device(dev):
        st = fn(ctx.handle, n, ctypes.c_void_p(A.data_ptr()), max(lda, n), ctypes.c_void_p(X.data_ptr()),
                max(ldx, n), ctypes.byref(o), _stream_handle(torch, dev), info_ptr)
    del keep
    _check(st)
    return X


def sweep_steps(W, p_begin, p_end=-1, part=None, block=None, sync=True, info=None, ctx=None, lookahead=None):
    """Steps [p_begin, p_end) of the blockwise sweep in place on the float64
    CUDA tensor W (binv_sweep_steps); W holds A before step 0 and the state a
    previous range left otherwise.  Returns W."""
    import torch

    if W.dim() != 2 or W.shape[0] != W.shape[1] or W.dtype != torch.float64 or not W.is_cuda or W.stride(1) != 1:
        raise ValueError("W must be a square row-major float64 CUDA tensor")
    n = W.shape[0]
    dev = W.device.index if W.device.index is not None else torch.cuda.current_device()
    ctx = ctx or default_context(dev)
    o, keep = _opts(part, block, sync, lookahead, False)
    info_ptr = None
    if info is not None:
        if info.dtype != torch.int64 or not info.is_cuda or info.numel() < 1:
            raise ValueError("info must be an int64 CUDA tensor with one element")
        info_ptr = ctypes.c_void_p(info.data_ptr())
    with torch.cuda.device(dev):
        st = load_library().binv_sweep_steps(ctx.handle, n, ctypes.c_void_p(W.data_ptr()), max(W.stride(0), n, 1),
                                             ctypes.byref(o), int(p_begin), int(p_end), _stream_handle(torch, dev),
                                             info_ptr)
    del keep
    _check(st)
    return W


def invert_host(W, device_bytes, part=None, block=None, ctx=None, device=0):
    """Invert the host matrix W (a C-contiguous float64 numpy array or CPU
    tensor, pinned or not) in place out of core (binv_invert_host), using at
    most device_bytes of device memory.  Returns W."""
    import numpy as np
    import torch

    if isinstance(W, torch.Tensor):
        if (W.is_cuda or W.dtype != torch.float64 or W.dim() != 2 or W.shape[0] != W.shape[1]
                or (W.numel() and W.stride(1) != 1)):
            raise ValueError("W must be a square row-major float64 host tensor")
        ptr, n, ld = W.data_ptr(), W.shape[0], W.stride(0)
    else:
        # (an empty array's strides carry no layout, so they are not checked)
        if W.dtype != np.float64 or W.ndim != 2 or W.shape[0] != W.shape[1] or (W.size and W.strides[1] != 8):
            raise ValueError("W must be a square row-major float64 array")
        ptr, n, ld = W.ctypes.data, W.shape[0], (W.strides[0] // 8 if W.size else 1)
    ctx = ctx or default_context(device)
    o, keep = _opts(part, block, False, True, False)
    row = ctypes.c_int64(0)
    with torch.cuda.device(ctx.device):
        st = load_library().binv_invert_host(ctx.handle, n, ctypes.c_void_p(ptr), max(ld, n, 1), ctypes.byref(o),
                                             int(device_bytes), _stream_handle(torch, ctx.device), ctypes.byref(row))
    del keep
    _check(st)
    return W


def invert_noalloc(A, part=None, block=None, out=None, inplace=False, sync=True, info=None, ctx=None):
    """invert() through binv_invert_noalloc: the serial sweep on the library's
    static per-device workspace (no device allocation; sizes are limited, see
    include/binv.h).  The caller allocates `out` (or passes inplace=True)."""
    return invert(A, part=part, block=block, out=out, inplace=inplace, sync=sync, info=info, ctx=ctx,
                  lookahead=False, _noalloc=True)


def invert_mixed(A, part=None, block=None, out=None, target=1e-10, max_refine=5, ctx=None, lookahead=None,
                 from_fp64=False, sampled_check=False, pivot=False):
    """Mixed-precision inversion: FP32 blockwise sweep (FP64 pivot blocks), then
    FP64 Newton-Schulz refinement to rho = ||AX - I||_F / sqrt(n) <= target.
    Synchronous.  Returns (X, info dict)."""
    import torch

    if A.dim() != 2 or A.shape[0] != A.shape[1] or A.dtype != torch.float64 or not A.is_cuda or A.stride(1) != 1:
        raise ValueError("A must be a square row-major float64 CUDA tensor")
    n = A.shape[0]
    X = out if out is not None else torch.empty_like(A, memory_format=torch.contiguous_format)
    dev = A.device.index if A.device.index is not None else torch.cuda.current_device()
    ctx = ctx or default_context(dev)
    o, keep = _opts(part, block, False, lookahead, pivot)
    if from_fp64:
        o.flags |= BINV_F_REFINE_FROM_FP64
    if sampled_check:
        o.flags |= BINV_F_SAMPLED_CHECK
    inf = _Info()
    with torch.cuda.device(dev):
        st = load_library().binv_invert_mixed(ctx.handle, n, ctypes.c_void_p(A.data_ptr()), max(A.stride(0), n, 1),
                                              ctypes.c_void_p(X.data_ptr()), max(X.stride(0), n, 1), ctypes.byref(o),
                                              float(target), int(max_refine), _stream_handle(torch, dev),
                                              ctypes.byref(inf))
    del keep
    if st != BINV_E_NOCONVERGE:  # a missed target returns the best iterate (info["converged"] is False)
        _check(st)
    k = inf.refine_steps
    return X, {"rho": inf.rho, "rho_steps": list(inf.rho_steps[: inf.rho_count]), "refine_steps": k,
               "fell_back": bool(inf.fell_back), "converged": bool(inf.converged), "sampled": inf.sampled}


def residual(A, X, estimate=False, ctx=None, compensated=False):
    """rho = ||AX - I||_F / sqrt(n) on the GPU: the full FP64 residual (with
    compensated=True formed through an error-free split of A and X), or with
    estimate=True its 64-probe random-sign estimate (exact below order 192)."""
    import torch

    for M, nm in ((A, "A"), (X, "X")):
        if M.dim() != 2 or M.dtype != torch.float64 or not M.is_cuda or M.stride(1) != 1:
            raise ValueError(f"{nm} must be a row-major float64 CUDA matrix")
    n = A.shape[0]
    if A.shape != (n, n) or X.shape != (n, n) or A.device != X.device:
        raise ValueError("A and X must be square, of one order, on one device")
    dev = A.device.index if A.device.index is not None else torch.cuda.current_device()
    ctx = ctx or default_context(dev)
    rho = ctypes.c_double()
    with torch.cuda.device(dev):
        st = load_library().binv_residual(ctx.handle, n, ctypes.c_void_p(A.data_ptr()), max(A.stride(0), n, 1),
                                          ctypes.c_void_p(X.data_ptr()), max(X.stride(0), n, 1),
                                          (BINV_RESID_ESTIMATE if estimate else 0)
                                          | (BINV_RESID_COMPENSATED if compensated else 0),
                                          _stream_handle(torch, dev), ctypes.byref(rho))
    _check(st)
    return rho.value


def residual_matrix(A, X, ctx=None):
    """(R, rho): the compensated residual matrix R = I - A X on the GPU."""
    import torch

    n = A.shape[0]
    R = torch.empty((n, n), dtype=torch.float64, device=A.device)
    dev = A.device.index if A.device.index is not None else torch.cuda.current_device()
    ctx = ctx or default_context(dev)
    rho = ctypes.c_double()
    with torch.cuda.device(dev):
        st = load_library().binv_residual_matrix(ctx.handle, n, ctypes.c_void_p(A.data_ptr()), max(A.stride(0), n, 1),
                                                 ctypes.c_void_p(X.data_ptr()), max(X.stride(0), n, 1),
                                                 ctypes.c_void_p(R.data_ptr()), max(n, 1), _stream_handle(torch, dev),
                                                 ctypes.byref(rho))
    _check(st)
    return R, rho.value


def level_partition(m):
    """The diagonal-block orders of §5.1's partitioning scheme (Table 2)."""
    k = ctypes.c_int32()
    _check(load_library().binv_level_partition(int(m), 0, ctypes.byref(k), None))
    part = (ctypes.c_int32 * max(k.value, 1))()
    _check(load_library().binv_level_partition(int(m), k.value, ctypes.byref(k), part))
    return list(part[:k.value])


def batch_shape(tier, shape):
    """Launch shape (rows/lane, cols/wave, waves/matrix, matrices/workgroup)."""
    out = (ctypes.c_int32 * 4)()
    _check(load_library().binv_batch_shape(int(tier), int(shape), out))
    return tuple(out)


class Batch:
    """A plan for inverting many small matrices (orders 1..256) packed back to
    back in one float64 buffer; matrix i is split into ks[i] diagonal blocks
    (orders `parts[i]`, or a near-equal split)."""

    def __init__(self, sizes, ks=None, parts=None, ctx=None, device=0):
        import numpy as np
        lib = load_library()
        self.ctx = ctx or default_context(device)
        self.sizes = np.ascontiguousarray(sizes, dtype=np.int32)
        n = int(self.sizes.size)
        self._k = None if ks is None and parts is None else np.ascontiguousarray(
            [len(p) for p in parts] if parts is not None else ks, dtype=np.int32)
        self._part = None
        if parts is not None:
            self._part = np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.int32) for p in parts])
                                              if n else np.zeros(0, np.int32), dtype=np.int32)
        h = ctypes.c_void_p()
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a is not None else None  # noqa: E731
        _check(lib.binv_batch_create(self.ctx.handle, n, ptr(self.sizes), ptr(self._k), ptr(self._part),
                                     ctypes.byref(h)))
        self._h = h
        cnt, tot, fl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        _check(lib.binv_batch_query(self._h, ctypes.byref(cnt), ctypes.byref(tot), ctypes.byref(fl)))
        self.count, self.total_elems, self.flops = int(cnt.value), int(tot.value), float(fl.value)
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes.astype(np.int64) ** 2)])[:-1] if n else np.zeros(0)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().binv_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def invert(self, A, out=None, info=None, graph=True, sync=True, inplace=False):
        """Invert every matrix of the packed float64 CUDA buffer A; returns (X, info)."""
        import torch
        if A.dtype != torch.float64 or not A.is_cuda or A.numel() != self.total_elems or not A.is_contiguous():
            raise ValueError("A must be a contiguous float64 CUDA buffer of the plan's packed size")
        X = A if inplace else (out if out is not None else torch.empty_like(A))
        if info is None:
            info = torch.empty(max(self.count, 1), dtype=torch.int32, device=A.device)
        flags = (BINV_F_GRAPH if graph else 0) | (BINV_F_SYNC if sync else 0)
        with torch.cuda.device(A.device):
            st = load_library().binv_invert_batched(self._h, ctypes.c_void_p(A.data_ptr()),
                                                    ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(info.data_ptr()),
                                                    flags, _stream_handle(torch, A.device.index or 0))
        _check(st)
        return X, info

    def invert_levels(self, A, out=None, info=None, sync=True, inplace=False):
        """Every matrix by the paper's level scheme (binv_invert_batched_levels);
        returns (X, info)."""
        import torch
        if A.dtype != torch.float64 or not A.is_cuda or A.numel() != self.total_elems or not A.is_contiguous():
            raise ValueError("A must be a contiguous float64 CUDA buffer of the plan's packed size")
        X = A if inplace else (out if out is not None else torch.empty_like(A))
        if info is None:
            info = torch.empty(max(self.count, 1), dtype=torch.int32, device=A.device)
        with torch.cuda.device(A.device):
            st = load_library().binv_invert_batched_levels(self._h, ctypes.c_void_p(A.data_ptr()),
                                                           ctypes.c_void_p(X.data_ptr()),
                                                           ctypes.c_void_p(info.data_ptr()),
                                                           BINV_F_SYNC if sync else 0,
                                                           _stream_handle(torch, A.device.index or 0))
        _check(st)
        return X, info

    def tune(self, A, out, info=None, reps=3):
        """Autotune the launch shape of each register tier on this batch (A -> out,
        out != A).  Returns (chosen shape per tier, ms table [tier][shape],
        shapes [tier] as (rows/lane, cols/wave, waves/matrix, matrices/workgroup))."""
        import torch
        if A.dtype != torch.float64 or not A.is_cuda or A.numel() != self.total_elems or not A.is_contiguous():
            raise ValueError("A must be a contiguous float64 CUDA buffer of the plan's packed size")
        if out is None or out.data_ptr() == A.data_ptr():
            raise ValueError("tuning needs a separate output buffer")
        if info is None:
            info = torch.empty(max(self.count, 1), dtype=torch.int32, device=A.device)
        chosen = (ctypes.c_int32 * len(TIER_SHAPES))()
        ms = (ctypes.c_double * (4 * len(TIER_SHAPES)))()
        with torch.cuda.device(A.device):
            _check(load_library().binv_batch_tune(self._h, ctypes.c_void_p(A.data_ptr()),
                                                  ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(info.data_ptr()),
                                                  int(reps), _stream_handle(torch, A.device.index or 0), chosen, ms))
        nt = len(TIER_SHAPES)
        return list(chosen), [list(ms[4 * t:4 * t + TIER_SHAPES[t]]) for t in range(nt)], [
            [batch_shape(t, v) for v in range(TIER_SHAPES[t])] for t in range(nt)]

    def residual(self, A, X):
        """rho_i = ||A_i X_i - I||_F / sqrt(m_i) for every matrix (float64 CUDA tensor)."""
        import torch
        rho = torch.empty(max(self.count, 1), dtype=torch.float64, device=A.device)
        with torch.cuda.device(A.device):
            _check(load_library().binv_batch_residual(self._h, ctypes.c_void_p(A.data_ptr()),
                                                      ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(rho.data_ptr()),
                                                      _stream_handle(torch, A.device.index or 0)))
        return rho[: self.count]

    def pack(self, mats):
        """Pack a list of square numpy matrices into one flat float64 array."""
        import numpy as np
        return np.concatenate([np.ascontiguousarray(M, dtype=np.float64).ravel() for M in mats]) \
            if len(mats) else np.zeros(0)

    def unpack(self, flat):
        """Split a flat array (numpy) back into the plan's matrices."""
        return [flat[o:o + m * m].reshape(m, m) for o, m in zip(self.offsets, self.sizes)]


class Server:
    """Continuous-batching inversion server on one device (see binv_submit)."""

    def __init__(self, device=0, hbm_budget=64 << 30, max_inflight=0, strict_precision=False, full_check=False):
        lib = load_library()
        h = ctypes.c_void_p()
        flags = (BINV_SERVER_STRICT_PRECISION if strict_precision else 0) | (BINV_SERVER_FULL_CHECK if full_check else 0)
        _check(lib.binv_server_create(int(device), int(hbm_budget), int(max_inflight), flags, ctypes.byref(h)))
        self._h = h
        self._shapes = {}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().binv_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, A, prec="fp64", target=1e-10) -> int:
        """A: square float64 numpy array or CUDA tensor (copied at once)."""
        import numpy as np
        is_dev = hasattr(A, "is_cuda") and A.is_cuda
        if is_dev:
            if A.dtype.__str__() != "torch.float64" or not A.is_contiguous():
                raise ValueError("device A must be a contiguous float64 tensor")
            ptr, n = A.data_ptr(), A.shape[0]
        else:
            A = np.ascontiguousarray(A, dtype=np.float64)
            ptr, n = A.ctypes.data, A.shape[0]
        if A.shape[0] != A.shape[1]:
            raise ValueError("A must be square")
        p = BINV_PREC_MIXED_F32 if prec == "mixed" else BINV_PREC_FP64
        t = ctypes.c_uint64()
        _check(load_library().binv_submit(self._h, int(n), ctypes.c_void_p(ptr), int(is_dev), p, float(target),
                                          ctypes.byref(t)))
        self._shapes[t.value] = int(n)
        return t.value

    def poll(self, ticket, out=None, copy=True):
        """None while busy; else (X, info dict, times dict).  X is a numpy array
        unless `out` (a CUDA tensor of the right shape) is given; with
        copy=False the result is dropped and X is None."""
        import numpy as np
        n = self._shapes.get(ticket)
        if n is None:
            raise BinvError(BINV_E_NOTFOUND, "unknown ticket")
        if not copy:
            X, ptr, dev = None, None, 0
        elif out is None:
            X = np.empty((n, n), dtype=np.float64)
            ptr, dev = X.ctypes.data, 0
        else:
            X = out
            ptr, dev = out.data_ptr(), 1
        inf, tm = _Info(), _Times()
        st = load_library().binv_poll(self._h, ctypes.c_uint64(ticket), ctypes.c_void_p(ptr), dev, ctypes.byref(inf),
                                      ctypes.byref(tm))
        if st == BINV_E_BUSY:
            return None
        del self._shapes[ticket]
        if st != BINV_E_NOCONVERGE:  # a missed target still delivers X (info["converged"] is False)
            _check(st)
        info = {"rho": inf.rho, "refine_steps": inf.refine_steps, "fell_back": bool(inf.fell_back),
                "converged": bool(inf.converged), "sampled": inf.sampled}
        return X, info, {"queue_ms": tm.queue_ms, "total_ms": tm.total_ms}

    def next_done(self, wait_us=0):
        """The oldest finished, uncollected ticket (waiting up to wait_us), or None."""
        t = ctypes.c_uint64()
        st = load_library().binv_next_done(self._h, int(wait_us), ctypes.byref(t))
        if st == BINV_E_BUSY:
            return None
        _check(st)
        return t.value

    def stats(self):
        u, p, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int64()
        _check(load_library().binv_server_stats(self._h, ctypes.byref(u), ctypes.byref(p), ctypes.byref(c)))
        return {"used": u.value, "peak": p.value, "completed": c.value}
