"""TEST INFRASTRUCTURE ONLY -- ctypes binding of the FP64 CPU oracle.

The oracle (``urv_oracle.c``) is a plain, slow reference implementation of
PowerURV (Gopal & Martinsson, arXiv:1812.06007, Section 3).  Only the test
suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this module.  It never touches the GPU library and the GPU library
never touches it.

All matrices are numpy float64 arrays in Fortran (column-major) order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "urv_oracle.c")
_HDR = os.path.join(_HERE, "urv_oracle.h")
LIB_PATH = os.path.join(_HERE, "liburv_oracle.so")
# A prebuilt oracle variant to load instead (used by the planted-mistake test).
_OVERRIDE = os.environ.get("URV_ORACLE_LIB")

FULL, HALF, NONE = 0, 1, 2
VARIANTS = {"full": FULL, "half": HALF, "none": NONE}

_lib = None


def compile_library(src: str, out: str) -> None:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-std=c11", "-Wall", "-I", _HERE, "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc: -O2, no contraction, no fast-math, OpenMP."""
    if _OVERRIDE:
        return _OVERRIDE
    stale = (not os.path.exists(LIB_PATH)) or any(
        os.path.getmtime(p) > os.path.getmtime(LIB_PATH) for p in (_SRC, _HDR))
    if force or stale:
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        compile_library(_SRC, tmp)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        path = _OVERRIDE or LIB_PATH
        if not os.path.exists(path):
            build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I32 = ctypes.c_int32
        U64 = ctypes.c_uint64
        D = ctypes.c_double
        L.orc_set_sum_order.argtypes = [ctypes.c_int]
        L.orc_philox4x64_10.argtypes = [P, P, P]
        L.orc_gaussian.argtypes = [P, I64, I64, I64, U64, ctypes.c_uint32]
        L.orc_gemm.argtypes = [ctypes.c_int, ctypes.c_int, I64, I64, I64, D, P, I64, P, I64, D, P, I64]
        L.orc_qr_pos.argtypes = [P, I64, I64, I64, P, I64, P, I64]
        L.orc_qr_pos.restype = ctypes.c_int
        L.orc_urv.argtypes = [P, I64, I64, I64, I32, U64, P, I64, I32, I32, P, I64, P, I64, P, I64]
        L.orc_urv.restype = ctypes.c_int
        L.orc_metrics.argtypes = [P, I64, I64, I64, P, I64, P, I64, P, I64, P, P]
        L.orc_metrics.restype = ctypes.c_int
        L.orc_jacobi_svd.argtypes = [P, I64, I64, I64, P, I32]
        L.orc_jacobi_svd.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


class sum_order:
    """Context manager: run the oracle with descending inner-product order."""

    def __init__(self, descending: bool):
        self.descending = descending

    def __enter__(self):
        lib().orc_set_sum_order(1 if self.descending else 0)
        return self

    def __exit__(self, *exc):
        lib().orc_set_sum_order(0)
        return False


def philox4x64_10(counter, key) -> np.ndarray:
    c = np.asarray(counter, dtype=np.uint64).copy()
    k = np.asarray(key, dtype=np.uint64).copy()
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def gaussian(rows: int, cols: int, seed: int, stream_id: int = 2) -> np.ndarray:
    G = np.zeros((rows, cols), dtype=np.float64, order="F")
    lib().orc_gaussian(_ptr(G), rows, cols, max(rows, 1), seed, stream_id)
    return G


def gemm(A, B, transA=False, transB=False, alpha=1.0, beta=0.0, C=None) -> np.ndarray:
    A = _f64(A)
    B = _f64(B)
    M = A.shape[1] if transA else A.shape[0]
    K = A.shape[0] if transA else A.shape[1]
    N = B.shape[0] if transB else B.shape[1]
    Kb = B.shape[1] if transB else B.shape[0]
    assert K == Kb
    C = np.zeros((M, N), order="F") if C is None else _f64(C).copy(order="F")
    lib().orc_gemm(int(transA), int(transB), M, N, K, alpha, _ptr(A), max(A.shape[0], 1),
                   _ptr(B), max(B.shape[0], 1), beta, _ptr(C), max(M, 1))
    return C


def qr_pos(X):
    """(Q, R) with Q m x n orthonormal columns, R n x n upper, diag(R) >= 0."""
    X = _f64(X).copy(order="F")
    m, n = X.shape
    Q = np.zeros((m, n), order="F")
    R = np.zeros((n, n), order="F")
    rc = lib().orc_qr_pos(_ptr(X), m, n, max(m, 1), _ptr(Q), max(m, 1), _ptr(R), max(n, 1))
    if rc != 0:
        raise ValueError("orc_qr_pos failed")
    return Q, R


def urv(A, q: int, seed: int = 0, G=None, variant: str | int = "full", orth_g: bool = False):
    """PowerURV A = U R V^T (eqs. power / powerqr).  Returns (U, R, V): with
    p = min(m, n), U m x p, R p x p upper, V n x p (m < n: the ULV of A^T,
    transposed, Section 1)."""
    A = _f64(A)
    m, n = A.shape
    p = min(m, n)
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    Gf = None if G is None else _f64(G)
    U = np.zeros((m, p), order="F")
    R = np.zeros((p, p), order="F")
    V = np.zeros((n, p), order="F")
    rc = lib().orc_urv(_ptr(A), m, n, max(m, 1), q, seed, _ptr(Gf), max(p, 1), v, int(orth_g),
                       _ptr(U), max(m, 1), _ptr(R), max(p, 1), _ptr(V), max(n, 1))
    if rc != 0:
        raise ValueError("orc_urv failed")
    return U, R, V


def metrics(A, U, R, V):
    """dict(recon, orthU, orthV, normA, ek) for A = U R V^T."""
    A, U, R, V = _f64(A), _f64(U), _f64(R), _f64(V)
    m, n = A.shape
    p = min(m, n)
    out = np.zeros(4)
    ek = np.zeros(p + 1)
    rc = lib().orc_metrics(_ptr(A), m, n, m, _ptr(U), m, _ptr(R), max(p, 1), _ptr(V), n, _ptr(out), _ptr(ek))
    if rc != 0:
        raise ValueError("orc_metrics failed")
    return {"recon": out[0], "orthU": out[1], "orthV": out[2], "normA": out[3], "ek": ek}


def jacobi_svd(A, max_sweeps: int = 60) -> np.ndarray:
    A = _f64(A)
    m, n = A.shape
    s = np.zeros(n)
    rc = lib().orc_jacobi_svd(_ptr(A), m, n, m, _ptr(s), max_sweeps)
    if rc < 0:
        raise ValueError("Jacobi SVD did not converge")
    return s
