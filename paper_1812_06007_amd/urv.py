"""Python binding of liburv (include/urv.h): argument marshalling only.

Every computation runs in the HIP kernels of liburv.so; this module turns
torch CUDA tensors into column-major device pointers and the current HIP
stream, and maps status codes to exceptions.  There is no fallback: if the
library is missing or no GPU is present, calls raise.

Matrices are torch tensors of shape (rows, cols).  Column-major storage
(stride (1, ld), ld >= rows) is passed through without a copy; anything else
is copied to column-major first.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liburv.so")

URV_OK, URV_EINVAL, URV_ENOMEM, URV_EDEVICE, URV_ENOTSUP, URV_ENONFINITE = 0, -1, -2, -3, -4, -5
URV_CHECK_FINITE, URV_A_FP32 = 1, 2
VARIANTS = {"full": 0, "half": 1, "none": 2}
PRECISIONS = {"fp64": 0, "mixed_bf16": 2, "mixed_fp16": 3}


class UrvError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__("liburv status %d (%s): %s" % (status, _strerror(status), detail))
        self.status = status
        self.detail = detail


class UrvOpts(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("orth_g", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("lda", ctypes.c_int64),
        ("ldu", ctypes.c_int64),
        ("ldr", ctypes.c_int64),
        ("ldv", ctypes.c_int64),
        ("G", ctypes.c_void_p),
        ("ldg", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class UrvGradOpts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("tape_mode", ctypes.c_int32),
        ("accumulate", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


TAPE_MODES = {"all": 0, "v": 1, "none": 2}

EXPORTS = ["urv_opts_init", "urv_factor_ex", "urv_sync_status", "urv_timing", "urv_timing_read", "urv_factor", "urv_workspace_size", "urv_gaussian",
           "urv_dgemm", "urv_dgemm_noalloc", "urv_qr_pos", "urv_qr_pos_f32", "urv_metrics", "urv_strerror", "urv_last_error",
           "urv_grad_opts_init", "urv_tape_bytes", "urv_grad_workspace_size", "urv_factor_tape",
           "urv_factor_backward", "urv_qr_adjoint", "urv_truncation_loss",
           "urv_batch_create", "urv_batch_set_buffers", "urv_batch_set_config", "urv_batch_get_config",
           "urv_batch_autotune", "urv_batch_run", "urv_batch_run_graph", "urv_batch_status",
           "urv_batch_destroy", "urv_max_rows"]

_lib = None


def lib() -> ctypes.CDLL:
    """Load liburv.so (built by ``python -m paper_1812_06007_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("URV_LIBRARY") or LIB_PATH  # another build of the same ABI, for comparisons
    if not os.path.exists(path):
        raise RuntimeError("liburv.so is not built (%s); run python -m paper_1812_06007_amd.build" % path)
    L = ctypes.CDLL(path)
    P, I32, I64, U32, U64, D, SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                    ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t)
    L.urv_opts_init.argtypes = [ctypes.POINTER(UrvOpts)]
    L.urv_opts_init.restype = None
    L.urv_factor_ex.argtypes = [P, I64, I64, I32, U64, P, P, P, ctypes.POINTER(UrvOpts)]
    L.urv_factor.argtypes = [P, I64, I64, I32, U64, P, P, P]
    L.urv_sync_status.argtypes = [P]
    L.urv_timing.argtypes = [I32]
    L.urv_timing_read.argtypes = [I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_double)]
    L.urv_workspace_size.argtypes = [I64, I64, I32, ctypes.POINTER(UrvOpts)]
    L.urv_workspace_size.restype = SZ
    L.urv_gaussian.argtypes = [P, I64, I64, I64, U64, U32, I32, P]
    L.urv_dgemm.argtypes = [I32, I32, I64, I64, I64, D, P, I64, P, I64, D, P, I64, P]
    L.urv_dgemm_noalloc.argtypes = [I32, I32, I64, I64, I64, D, P, I64, P, I64, D, P, I64, P]
    L.urv_qr_pos.argtypes = [P, I64, I64, I64, P, I64, P, I64, P]
    L.urv_qr_pos_f32.argtypes = [P, I64, I64, I64, P, I64, P, I64, P]
    L.urv_metrics.argtypes = [P, I64, I64, P, P, P, P, P, P]
    L.urv_strerror.argtypes = [ctypes.c_int]
    L.urv_strerror.restype = ctypes.c_char_p
    L.urv_last_error.argtypes = []
    L.urv_last_error.restype = ctypes.c_char_p
    GO = ctypes.POINTER(UrvGradOpts)
    L.urv_grad_opts_init.argtypes = [GO]
    L.urv_grad_opts_init.restype = None
    L.urv_tape_bytes.argtypes = [I64, I64, I32, GO]
    L.urv_tape_bytes.restype = SZ
    L.urv_grad_workspace_size.argtypes = [I64, I64, I32, GO]
    L.urv_grad_workspace_size.restype = SZ
    L.urv_factor_tape.argtypes = [P, I64, I64, I32, P, P, P, P, P, GO]
    L.urv_factor_backward.argtypes = [P, I64, I64, I32, P, P, P, P, P, P, P, P, P, GO]
    L.urv_qr_adjoint.argtypes = [P, P, I64, I64, P, P, P, I32, P]
    L.urv_truncation_loss.argtypes = [P, I64, I64, P, P, P, I64, P, P, P, P, P, GO]
    PI64 = ctypes.POINTER(ctypes.c_int64)
    PP = ctypes.POINTER(ctypes.c_void_p)
    L.urv_batch_create.argtypes = [I64, PI64, PI64, I32, U64, ctypes.POINTER(ctypes.c_void_p)]
    L.urv_batch_set_buffers.argtypes = [P, PP, PP, PP, PP]
    L.urv_batch_set_config.argtypes = [P, I32, I32, I32]
    L.urv_batch_get_config.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32)]
    L.urv_batch_status.argtypes = [P, P]
    L.urv_batch_autotune.argtypes = [P, P, ctypes.POINTER(D)]
    L.urv_batch_run.argtypes = [P, P]
    L.urv_batch_run_graph.argtypes = [P, P]
    L.urv_max_rows.argtypes = []
    L.urv_max_rows.restype = I64
    L.urv_batch_destroy.argtypes = [P]
    L.urv_batch_destroy.restype = None
    for name in ("urv_factor_ex", "urv_factor", "urv_gaussian", "urv_dgemm", "urv_dgemm_noalloc", "urv_qr_pos", "urv_qr_pos_f32",
                 "urv_metrics", "urv_factor_tape", "urv_factor_backward", "urv_qr_adjoint",
                 "urv_truncation_loss", "urv_batch_create", "urv_batch_set_buffers", "urv_batch_set_config",
                 "urv_batch_get_config", "urv_batch_autotune", "urv_batch_run", "urv_batch_run_graph",
                 "urv_batch_status", "urv_sync_status", "urv_timing", "urv_timing_read"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _strerror(status: int) -> str:
    try:
        return lib().urv_strerror(status).decode()
    except Exception:  # pragma: no cover - only when the library cannot load
        return "?"


def _check(status: int) -> None:
    if status != URV_OK:
        raise UrvError(status, lib().urv_last_error().decode())


def _torch():
    import torch

    return torch


def _stream_ptr():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _colmajor(t, dtype=None):
    """(tensor, ld): t itself if it is column-major on the GPU, else a column-major copy."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if not t.is_cuda:
        raise ValueError("liburv works on GPU tensors; got a tensor on %s" % t.device)
    dtype = dtype or torch.float64
    rows, cols = t.shape
    if t.dtype == dtype and (t.stride(0) == 1 or rows <= 1) and (t.stride(1) >= max(rows, 1) or cols <= 1):
        return t, max(t.stride(1) if cols > 1 else rows, rows, 1)
    c = empty_colmajor(rows, cols, dtype=dtype, device=t.device)
    c.copy_(t)
    return c, max(rows, 1)


def _packed(t):
    """Column-major with leading dimension == rows (copy if needed)."""
    c, ld = _colmajor(t)
    if ld == max(c.shape[0], 1) or c.shape[1] <= 1:
        return c
    p = empty_colmajor(*c.shape, device=c.device)
    p.copy_(c)
    return p


def empty_colmajor(rows: int, cols: int, dtype=None, device=None):
    """Uninitialised (rows, cols) tensor with column-major strides (1, rows)."""
    torch = _torch()
    return torch.empty((cols, rows), dtype=dtype or torch.float64, device=device or "cuda").t()


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() > 0 else 0)


def max_rows() -> int:
    """Largest row count of the tall problem the QR panel supports."""
    return int(lib().urv_max_rows())


def workspace_size(m: int, n: int, q: int = 0, variant: str = "full", precision: str = "fp64",
                   a_fp32: bool = False) -> int:
    o = UrvOpts()
    lib().urv_opts_init(ctypes.byref(o))
    o.variant = VARIANTS[variant]
    o.precision = PRECISIONS[precision]
    o.flags = URV_A_FP32 if a_fp32 else 0
    return int(lib().urv_workspace_size(m, n, q, ctypes.byref(o)))


def factor(A, q: int, seed: int = 0, variant: str = "full", precision: str = "fp64", G=None,
           orth_g: bool = False, workspace=None, out=None, check_finite: bool = False, check: bool = True):
    """PowerURV A = U R V^T (Section 3).  Returns (U, R, V) as column-major FP64 tensors:
    U m x p, R p x p, V n x p with p = min(m, n) (m < n: a ULV of A^T, transposed).

    A may be FP64 or FP32 (an FP32 A is passed as is: URV_A_FP32).  ``workspace``
    may be a uint8 CUDA tensor of at least ``workspace_size(...)`` bytes; ``out``
    may be a (U, R, V) triple of column-major tensors to write into.
    ``check_finite`` rejects a NaN or infinity in A (UrvError URV_ENONFINITE).
    With ``check`` (default) the call waits for the stream and raises UrvError
    (URV_EDEVICE) if a panel's device-side wait expired; with check=False it is
    asynchronous on the current stream and ``sync_status()`` reports that later.
    """
    torch = _torch()
    a32 = isinstance(A, torch.Tensor) and A.dtype == torch.float32
    A, lda = _colmajor(A, dtype=torch.float32 if a32 else None)
    m, n = A.shape
    p = min(m, n)
    if out is None:
        U = empty_colmajor(m, p, device=A.device)
        R = empty_colmajor(p, p, device=A.device)
        V = empty_colmajor(n, p, device=A.device)
    else:
        U, R, V = out
    o = UrvOpts()
    lib().urv_opts_init(ctypes.byref(o))
    o.variant = VARIANTS[variant]
    o.precision = PRECISIONS[precision]
    o.orth_g = int(bool(orth_g))
    o.flags = (URV_CHECK_FINITE if check_finite else 0) | (URV_A_FP32 if a32 else 0)
    o.lda = lda
    o.ldu = max(U.stride(1), m) if p > 1 else max(m, 1)
    o.ldr = max(R.stride(1), p) if p > 1 else max(p, 1)
    o.ldv = max(V.stride(1), n) if p > 1 else max(n, 1)
    Gk = None
    if G is not None:
        Gk, ldg = _colmajor(G)
        if tuple(Gk.shape) != (p, p):
            raise ValueError("G must be min(m, n) x min(m, n)")
        o.G = Gk.data_ptr()
        o.ldg = ldg
    o.stream = _stream_ptr().value
    if workspace is not None:
        if workspace.dtype != torch.uint8 or not workspace.is_cuda:
            raise ValueError("workspace must be a uint8 CUDA tensor")
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel()
    for t in (U, R, V):
        if t.stride(0) != 1 and t.shape[0] > 1:
            raise ValueError("outputs must be column-major")
    _check(lib().urv_factor_ex(_ptr(A), m, n, q, seed & (2**64 - 1), _ptr(U), _ptr(R), _ptr(V), ctypes.byref(o)))
    if check:
        sync_status()
    return U, R, V


TIMED_CLASSES = {"panel": 0, "gemm_nn": 1, "gemm_tn": 2, "gemm_nt": 3, "gemm_tt": 4}


def timing(enable: bool) -> None:
    """Start (clearing the counts) or stop HIP-event timing of the library's FP64 launches."""
    _check(lib().urv_timing(int(bool(enable))))


def timing_read(cls: str) -> dict:
    """Summed ms, launch count and algorithmic flops of one timed class (call after a sync)."""
    ms, n, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    _check(lib().urv_timing_read(TIMED_CLASSES[cls], ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl)))
    return {"ms": ms.value, "launches": n.value, "flops": fl.value}


def sync_status() -> None:
    """Waits for the current stream; raises UrvError (URV_EDEVICE) if a factorisation or
    QR queued since the last check had a panel's device-side wait expire."""
    _check(lib().urv_sync_status(_stream_ptr()))


def gaussian(rows: int, cols: int, seed: int, stream_id: int = 2, dtype=None, device=None):
    """The Gaussian of eq. power drawn on the GPU (Philox4x64-10 + Box-Muller)."""
    torch = _torch()
    dtype = dtype or torch.float64
    G = empty_colmajor(rows, cols, dtype=dtype, device=device)
    prec = 0 if dtype == torch.float64 else 1
    _check(lib().urv_gaussian(_ptr(G), rows, cols, max(rows, 1), seed & (2**64 - 1), stream_id, prec, _stream_ptr()))
    return G


def dgemm(A, B, transA: bool = False, transB: bool = False, alpha: float = 1.0, beta: float = 0.0, C=None,
          noalloc: bool = False):
    """C = alpha op(A) op(B) + beta C in FP64 (C column-major, written in place if given).
    noalloc=True calls urv_dgemm_noalloc (split-K partials in the library's static buffer)."""
    A, lda = _colmajor(A)
    B, ldb = _colmajor(B)
    M = A.shape[1] if transA else A.shape[0]
    K = A.shape[0] if transA else A.shape[1]
    N = B.shape[0] if transB else B.shape[1]
    if (B.shape[1] if transB else B.shape[0]) != K:
        raise ValueError("inner dimensions differ")
    if C is None:
        C = empty_colmajor(M, N, device=A.device)
        beta = 0.0
    elif C.stride(0) != 1 and C.shape[0] > 1:
        raise ValueError("C must be column-major")
    ldc = max(C.stride(1), M, 1) if N > 1 else max(M, 1)
    fn = lib().urv_dgemm_noalloc if noalloc else lib().urv_dgemm
    _check(fn(int(transA), int(transB), M, N, K, alpha, _ptr(A), lda, _ptr(B), ldb, beta, _ptr(C), ldc,
              _stream_ptr()))
    return C


def qr_pos(X, want_q: bool = True, want_r: bool = True, fp32: bool = False, check: bool = True):
    """Blocked Householder QR with diag(R) >= 0 (FP64, or FP32 with fp32=True).
    Returns (Q, R) (None where not wanted).  With ``check`` (default) waits for the
    stream and raises UrvError if a panel's device-side wait expired."""
    torch = _torch()
    dt = torch.float32 if fp32 else torch.float64
    Xw = empty_colmajor(*X.shape, dtype=dt, device=X.device)
    Xw.copy_(X)
    m, n = Xw.shape
    Q = empty_colmajor(m, n, dtype=dt, device=X.device) if want_q else None
    R = empty_colmajor(n, n, dtype=dt, device=X.device) if want_r else None
    fn = lib().urv_qr_pos_f32 if fp32 else lib().urv_qr_pos
    _check(fn(_ptr(Xw), m, n, max(m, 1), _ptr(Q), max(m, 1), _ptr(R), max(n, 1), _stream_ptr()))
    if check:
        sync_status()
    return Q, R


def metrics(A, U, R, V) -> dict:
    """Device checks: recon, orthU, orthV, normA and ek (rank-k errors, length n+1). Blocking."""
    import numpy as np

    A, U, R, V = (_packed(t) for t in (A, U, R, V))
    m, n = A.shape
    out = np.zeros(4)
    ek = np.zeros(min(m, n) + 1)
    _check(lib().urv_metrics(_ptr(A), m, n, _ptr(U), _ptr(R), _ptr(V),
                             out.ctypes.data_as(ctypes.c_void_p), ek.ctypes.data_as(ctypes.c_void_p),
                             _stream_ptr()))
    return {"recon": out[0], "orthU": out[1], "orthV": out[2], "normA": out[3], "ek": ek}


# ---------------------------------------------------------------- derivative (G held fixed)
def _real_dtype(t):
    torch = _torch()
    if t.dtype not in (torch.float32, torch.float64):
        raise TypeError("the derivative entry points take float32 or float64 tensors")
    return t.dtype


def _packed_as(t, dtype):
    """Column-major, leading dimension == rows, of the given dtype (copy if needed)."""
    c, ld = _colmajor(t, dtype)
    if ld == max(c.shape[0], 1) or c.shape[1] <= 1:
        return c
    p = empty_colmajor(*c.shape, dtype=dtype, device=c.device)
    p.copy_(c)
    return p


def _grad_opts(dtype, variant="full", tape_mode="all", accumulate=False, workspace=None) -> UrvGradOpts:
    torch = _torch()
    o = UrvGradOpts()
    lib().urv_grad_opts_init(ctypes.byref(o))
    o.precision = 1 if dtype == torch.float32 else 0
    o.variant = VARIANTS[variant]
    o.tape_mode = TAPE_MODES[tape_mode]
    o.accumulate = int(bool(accumulate))
    o.stream = _stream_ptr().value
    if workspace is not None:
        if workspace.dtype != torch.uint8 or not workspace.is_cuda:
            raise ValueError("workspace must be a uint8 CUDA tensor")
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel()
    return o


def tape_bytes(m: int, n: int, q: int, dtype=None, variant: str = "full", tape_mode: str = "all") -> int:
    torch = _torch()
    o = _grad_opts(dtype or torch.float64, variant, tape_mode)
    return int(lib().urv_tape_bytes(m, n, q, ctypes.byref(o)))


def grad_workspace_size(m: int, n: int, q: int = 0, dtype=None) -> int:
    torch = _torch()
    o = _grad_opts(dtype or torch.float64)
    return int(lib().urv_grad_workspace_size(m, n, q, ctypes.byref(o)))


def factor_tape(A, G, q: int, variant: str = "full", tape_mode: str = "all", workspace=None):
    """Forward pass of the differentiable factorisation from the fixed G.

    Returns (U, R, V, tape): column-major tensors of A's dtype (float32 or
    float64) and the uint8 tape that ``factor_backward`` reads."""
    torch = _torch()
    dt = _real_dtype(A)
    A = _packed_as(A, dt)
    m, n = A.shape
    G = _packed_as(G, dt)
    if tuple(G.shape) != (n, n):
        raise ValueError("G must be n x n")
    U = empty_colmajor(m, n, dtype=dt, device=A.device)
    R = empty_colmajor(n, n, dtype=dt, device=A.device)
    V = empty_colmajor(n, n, dtype=dt, device=A.device)
    o = _grad_opts(dt, variant, tape_mode, workspace=workspace)
    tape = torch.empty(max(int(lib().urv_tape_bytes(m, n, q, ctypes.byref(o))), 1), dtype=torch.uint8,
                       device=A.device)
    _check(lib().urv_factor_tape(_ptr(A), m, n, q, _ptr(G), _ptr(U), _ptr(R), _ptr(V), _ptr(tape),
                                 ctypes.byref(o)))
    return U, R, V, tape


def factor_backward(A, G, U, R, V, tape, q: int, dU=None, dR=None, dV=None, variant: str = "full",
                    tape_mode: str = "all", dA=None, accumulate: bool = False, workspace=None):
    """dL/dA for the adjoints dU, dR, dV (None = zero) of a loss L(U, R, V)."""
    dt = _real_dtype(A)
    A = _packed_as(A, dt)
    m, n = A.shape
    G, U, R, V = (_packed_as(t, dt) for t in (G, U, R, V))
    dU, dR, dV = (None if t is None else _packed_as(t, dt) for t in (dU, dR, dV))
    if dA is None:
        dA = empty_colmajor(m, n, dtype=dt, device=A.device)
        accumulate = False
    elif dA.dtype != dt or (dA.stride(0) != 1 and m > 1) or (n > 1 and dA.stride(1) != max(m, 1)):
        raise ValueError("dA must be packed column-major of A's dtype")
    o = _grad_opts(dt, variant, tape_mode, accumulate, workspace)
    _check(lib().urv_factor_backward(_ptr(A), m, n, q, _ptr(G), _ptr(U), _ptr(R), _ptr(V), _ptr(tape),
                                     _ptr(dU), _ptr(dR), _ptr(dV), _ptr(dA), ctypes.byref(o)))
    return dA


def qr_adjoint(Q, R, dQ=None, dR=None):
    """Adjoint of X = Q R: (dQ + Q S) R^{-T} (see include/urv.h)."""
    dt = _real_dtype(Q)
    Q, R = _packed_as(Q, dt), _packed_as(R, dt)
    dQ = None if dQ is None else _packed_as(dQ, dt)
    dR = None if dR is None else _packed_as(dR, dt)
    m, n = Q.shape
    dX = empty_colmajor(m, n, dtype=dt, device=Q.device)
    torch = _torch()
    _check(lib().urv_qr_adjoint(_ptr(Q), _ptr(R), m, n, _ptr(dQ), _ptr(dR), _ptr(dX),
                                1 if dt == torch.float32 else 0, _stream_ptr()))
    return dX


def truncation_loss(A, U, R, V, k: int, seeds: bool = True, workspace=None):
    """L = ||A - U(:,:k) R(:k,:) V^T||_F^2 on the device.

    Returns (L, dU, dR, dV, dA): L a 0-d float64 CUDA tensor; the adjoints
    (None unless ``seeds``) and dA = 2 (A - A_k), in A's dtype."""
    torch = _torch()
    dt = _real_dtype(A)
    A = _packed_as(A, dt)
    m, n = A.shape
    U, R, V = (_packed_as(t, dt) for t in (U, R, V))
    L = torch.empty((), dtype=torch.float64, device=A.device)
    dA = empty_colmajor(m, n, dtype=dt, device=A.device)
    dU = empty_colmajor(m, n, dtype=dt, device=A.device) if seeds else None
    dR = empty_colmajor(n, n, dtype=dt, device=A.device) if seeds else None
    dV = empty_colmajor(n, n, dtype=dt, device=A.device) if seeds else None
    o = _grad_opts(dt, workspace=workspace)
    _check(lib().urv_truncation_loss(_ptr(A), m, n, _ptr(U), _ptr(R), _ptr(V), k, ctypes.c_void_p(L.data_ptr()),
                                     _ptr(dU), _ptr(dR), _ptr(dV), _ptr(dA), ctypes.byref(o)))
    return L, dU, dR, dV, dA


# ---------------------------------------------------------------- batched factorisation
class BatchPlan:
    """Many FP32 matrices (1 <= n_i <= m_i <= 1024) factored by one persistent
    launch (include/urv.h, urv_batch_*).  Matrix i uses G from seed + i."""

    def __init__(self, ms, ns, q: int = 1, seed: int = 0):
        count = len(ms)
        if len(ns) != count:
            raise ValueError("ms and ns differ in length")
        self.ms, self.ns, self.q, self.seed = [int(x) for x in ms], [int(x) for x in ns], int(q), int(seed)
        marr = (ctypes.c_int64 * count)(*self.ms)
        narr = (ctypes.c_int64 * count)(*self.ns)
        self._plan = ctypes.c_void_p()
        _check(lib().urv_batch_create(count, marr, narr, self.q, self.seed & (2**64 - 1), ctypes.byref(self._plan)))
        self._keep = None

    def set_buffers(self, A, U, R, V) -> None:
        """Lists of packed column-major float32 CUDA tensors (A read only)."""
        torch = _torch()
        count = len(self.ms)
        for name, lst, shapes in (("A", A, [(m, n) for m, n in zip(self.ms, self.ns)]),
                                  ("U", U, [(m, n) for m, n in zip(self.ms, self.ns)]),
                                  ("R", R, [(n, n) for n in self.ns]), ("V", V, [(n, n) for n in self.ns])):
            if len(lst) != count:
                raise ValueError("%s: expected %d tensors" % (name, count))
            for t, shp in zip(lst, shapes):
                if (not t.is_cuda or t.dtype != torch.float32 or tuple(t.shape) != shp
                        or (shp[1] > 1 and t.stride(1) != shp[0]) or (shp[0] > 1 and t.stride(0) != 1)):
                    raise ValueError("%s: need packed column-major float32 CUDA tensors of the plan's sizes" % name)
        arrs = [(ctypes.c_void_p * count)(*[t.data_ptr() for t in lst]) for lst in (A, U, R, V)]
        _check(lib().urv_batch_set_buffers(self._plan, *arrs))
        self._keep = (list(A), list(U), list(R), list(V))

    def set_config(self, nb: int, grid: int, team_max: int = 1) -> None:
        _check(lib().urv_batch_set_config(self._plan, nb, grid, team_max))

    def config(self):
        """(nb, grid, team_max) of the next launch."""
        nb, grid, team = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().urv_batch_get_config(self._plan, ctypes.byref(nb), ctypes.byref(grid), ctypes.byref(team)))
        return nb.value, grid.value, team.value

    def status(self) -> None:
        """Raise if a team barrier's bounded wait expired in a run so far (blocking)."""
        _check(lib().urv_batch_status(self._plan, _stream_ptr()))

    def autotune(self) -> float:
        ms = ctypes.c_double()
        _check(lib().urv_batch_autotune(self._plan, _stream_ptr(), ctypes.byref(ms)))
        return ms.value

    def run(self, graph: bool = False) -> None:
        fn = lib().urv_batch_run_graph if graph else lib().urv_batch_run
        _check(fn(self._plan, _stream_ptr()))

    def close(self) -> None:
        if self._plan:
            _torch().cuda.synchronize()
            lib().urv_batch_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            if self._plan:
                lib().urv_batch_destroy(self._plan)
        except Exception:  # pragma: no cover - interpreter shutdown
            pass


def batch_outputs(ms, ns, device=None):
    """Packed column-major float32 (U, R, V) lists for the given sizes."""
    torch = _torch()
    U = [empty_colmajor(m, n, dtype=torch.float32, device=device) for m, n in zip(ms, ns)]
    R = [empty_colmajor(n, n, dtype=torch.float32, device=device) for n in ns]
    V = [empty_colmajor(n, n, dtype=torch.float32, device=device) for n in ns]
    return U, R, V
