"""PowerURV (Gopal & Martinsson, arXiv:1812.06007) on AMD MI355X (gfx950).

The factorisation A = U R V^T runs in the HIP kernels of ``liburv.so``
behind the C ABI of ``include/urv.h``; this package is its Python binding.
"""
from .urv import (  # noqa: F401
    BatchPlan,
    UrvError,
    batch_outputs,
    dgemm,
    empty_colmajor,
    factor,
    factor_backward,
    factor_tape,
    gaussian,
    grad_workspace_size,
    lib,
    metrics,
    qr_adjoint,
    qr_pos,
    tape_bytes,
    truncation_loss,
    workspace_size,
)

__all__ = ["BatchPlan", "UrvError", "batch_outputs", "dgemm", "empty_colmajor", "factor", "factor_backward", "factor_tape", "gaussian",
           "grad_workspace_size", "lib", "metrics", "qr_adjoint", "qr_pos", "tape_bytes", "truncation_loss",
           "workspace_size"]
