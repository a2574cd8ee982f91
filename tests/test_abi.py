"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/urv.h, and rejects bad arguments with
URV_EINVAL before any device work."""
import ctypes
import os
import re

import pytest

from paper_1812_06007_amd import urv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "urv.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(urv_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("urv_factor", "urv_factor_ex", "urv_workspace_size", "urv_gaussian",
                     "urv_strerror", "urv_last_error"):
        assert required in names
    assert sorted(urv.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    L = urv.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_opts_struct_matches_header_layout():
    # int32 x4, int64 x4, ptr, int64, ptr, ptr, size_t
    assert ctypes.sizeof(urv.UrvOpts) == 4 * 4 + 8 * 4 + 8 + 8 + 8 + 8 + 8
    o = urv.UrvOpts()
    urv.lib().urv_opts_init(ctypes.byref(o))
    assert (o.variant, o.precision, o.orth_g, o.flags, o.lda, o.G, o.stream, o.workspace) == (
        0, 0, 0, 0, 0, None, None, None)


def test_strerror_and_last_error():
    L = urv.lib()
    assert L.urv_strerror(0) == b"success"
    assert L.urv_strerror(-1) == b"invalid argument"
    assert L.urv_strerror(12345) == b"unknown status"
    assert isinstance(L.urv_last_error(), bytes)


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


def _factor(m, n, q, ptrs=True, **fields):
    o = urv.UrvOpts()
    urv.lib().urv_opts_init(ctypes.byref(o))
    for k, v in fields.items():
        setattr(o, k, v)
    p = FAKE if ptrs else None
    return urv.lib().urv_factor_ex(p, m, n, q, 0, p, p, p, ctypes.byref(o))


@pytest.mark.parametrize("m,n,q,fields", [
    (5, -1, 1, {}),                     # n < 0
    (3, 5, 1, {"ldv": 3}),              # m < n: V is n x m, ldv >= n
    (3, 5, 1, {"ldr": 2}),              # m < n: R is m x m
    (5, 3, -1, {}),                     # q < 0
    (5, 3, 1, {"variant": 3}),          # unknown variant
    (5, 3, 1, {"precision": 1}),        # URV_FP32: not a mode of urv_factor_ex
    (5, 3, 1, {"flags": 4}),           # unknown flag bit
    (5, 3, 1, {"lda": 4}),              # ld < rows
    (5, 3, 1, {"ldu": 2}),
    (5, 3, 1, {"ldr": 2}),
    (5, 3, 1, {"ldv": 2}),
    (5, 3, 1, {"ldg": 2}),
    (5, 3, 1, {"lda": -5}),
    (5, 3, 1, {"workspace_bytes": 64}),  # bytes without a buffer
    (5, 3, 1, {"workspace": 0x2000, "workspace_bytes": 64}),  # too small
])
def test_factor_rejects_bad_arguments(m, n, q, fields):
    assert _factor(m, n, q, **fields) == urv.URV_EINVAL
    assert urv.lib().urv_last_error() != b""


def test_factor_null_pointers_rejected():
    assert _factor(5, 3, 1, ptrs=False) == urv.URV_EINVAL


def test_factor_empty_is_noop():
    assert _factor(5, 0, 2, ptrs=False) == urv.URV_OK
    assert _factor(0, 0, 0, ptrs=False) == urv.URV_OK


def test_too_many_rows_is_unsupported():
    assert _factor(1 << 20, 8, 1) == urv.URV_ENOTSUP


def test_fp32_a_adds_its_fp64_copy_to_the_workspace():
    base = urv.workspace_size(1000, 500, 2, precision="mixed_bf16")
    a32 = urv.workspace_size(1000, 500, 2, precision="mixed_bf16", a_fp32=True)
    assert a32 - base >= 1000 * 500 * 8
    # a workspace sized without the copy is too small for an FP32 A
    rc = _factor(1000, 500, 2, precision=2, flags=urv.URV_A_FP32, workspace=0x2000, workspace_bytes=base)
    assert rc == urv.URV_EINVAL


def test_status_codes_have_text():
    L = urv.lib()
    assert L.urv_strerror(urv.URV_ENONFINITE) == b"non-finite input"


def test_workspace_size_monotone():
    small = urv.workspace_size(100, 50)
    big = urv.workspace_size(1000, 500)
    assert 0 < small < big
    assert urv.workspace_size(10, 0) == 0
    assert urv.workspace_size(3, 5) > 0          # m < n: the transposed problem
    # the FP64 workspace of the 8000 x 8000 case stays far below 288 GB of HBM
    assert urv.workspace_size(8000, 8000, 2) < 4 * 2**30


def test_other_entry_points_validate():
    L = urv.lib()
    assert L.urv_gaussian(FAKE, 4, 3, 2, 0, 2, 0, None) == urv.URV_EINVAL   # ld < rows
    assert L.urv_gaussian(None, 4, 3, 4, 0, 2, 0, None) == urv.URV_EINVAL   # null
    assert L.urv_gaussian(None, 0, 3, 1, 0, 2, 0, None) == urv.URV_OK       # empty
    assert L.urv_dgemm(0, 0, 4, 4, 4, 1.0, FAKE, 3, FAKE, 4, 0.0, FAKE, 4, None) == urv.URV_EINVAL
    assert L.urv_dgemm(1, 0, 4, 4, 5, 1.0, FAKE, 4, FAKE, 5, 0.0, FAKE, 4, None) == urv.URV_EINVAL
    assert L.urv_dgemm(0, 0, -1, 4, 4, 1.0, FAKE, 4, FAKE, 4, 0.0, FAKE, 4, None) == urv.URV_EINVAL
    assert L.urv_dgemm(0, 0, 0, 4, 4, 1.0, None, 1, None, 4, 0.0, None, 1, None) == urv.URV_OK
    assert L.urv_qr_pos(FAKE, 3, 5, 3, None, 3, None, 5, None) == urv.URV_EINVAL
    assert L.urv_qr_pos(FAKE, 5, 3, 4, None, 5, None, 3, None) == urv.URV_EINVAL
    assert L.urv_qr_pos(None, 5, 0, 5, None, 5, None, 1, None) == urv.URV_OK
    assert L.urv_metrics(None, 5, 3, None, None, None, None, None, None) == urv.URV_EINVAL


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError):
        urv.factor(torch.zeros(4, 3, dtype=torch.float64), 1)


# ---------------------------------------------------------------- derivative entry points
def _gopts(**fields):
    o = urv.UrvGradOpts()
    urv.lib().urv_grad_opts_init(ctypes.byref(o))
    for k, v in fields.items():
        setattr(o, k, v)
    return o


def test_grad_opts_struct_matches_header_layout():
    # int32 x4, ptr, ptr, size_t
    assert ctypes.sizeof(urv.UrvGradOpts) == 4 * 4 + 8 + 8 + 8
    o = _gopts()
    assert (o.precision, o.variant, o.tape_mode, o.accumulate, o.stream, o.workspace) == (0, 0, 0, 0, None, None)


@pytest.mark.parametrize("m,n,q,fields", [
    (3, 5, 1, {}),                        # m < n
    (5, 3, -1, {}),                       # q < 0
    (5, 3, 1, {"precision": 2}),          # mixed precision has no derivative
    (5, 3, 1, {"variant": 2}),            # NONE has no derivative
    (5, 3, 1, {"tape_mode": 3}),
    (5, 3, 1, {"workspace_bytes": 64}),   # bytes without a buffer
])
def test_grad_entry_points_reject_bad_arguments(m, n, q, fields):
    L = urv.lib()
    o = _gopts(**fields)
    P = FAKE
    assert L.urv_factor_tape(P, m, n, q, P, P, P, P, P, ctypes.byref(o)) == urv.URV_EINVAL
    assert L.urv_factor_backward(P, m, n, q, P, P, P, P, P, P, P, P, P, ctypes.byref(o)) == urv.URV_EINVAL
    assert urv.lib().urv_last_error() != b""


def test_grad_entry_points_validate():
    L = urv.lib()
    o = _gopts()
    P = FAKE
    # null pointers, empty calls, k outside [0, n], too many rows
    assert L.urv_factor_tape(None, 5, 3, 1, P, P, P, P, P, ctypes.byref(o)) == urv.URV_EINVAL
    assert L.urv_factor_tape(P, 5, 3, 1, P, P, P, P, None, ctypes.byref(o)) == urv.URV_EINVAL
    assert L.urv_factor_tape(None, 5, 0, 1, None, None, None, None, None, ctypes.byref(o)) == urv.URV_OK
    assert L.urv_factor_backward(P, 5, 3, 1, P, P, P, P, P, None, None, None, None, ctypes.byref(o)) == urv.URV_EINVAL
    assert L.urv_factor_tape(P, 1 << 20, 8, 1, P, P, P, P, P, ctypes.byref(o)) == urv.URV_ENOTSUP
    assert L.urv_truncation_loss(P, 5, 3, P, P, P, 4, None, None, None, None, P, ctypes.byref(o)) == urv.URV_EINVAL
    assert L.urv_truncation_loss(P, 5, 3, P, P, P, -1, None, None, None, None, P, ctypes.byref(o)) == urv.URV_EINVAL
    assert L.urv_truncation_loss(P, 5, 3, P, P, P, 2, None, None, None, None, None, ctypes.byref(o)) == urv.URV_EINVAL
    assert L.urv_qr_adjoint(P, P, 3, 5, None, None, P, 0, None) == urv.URV_EINVAL
    assert L.urv_qr_adjoint(P, P, 5, 3, None, None, P, 3, None) == urv.URV_EINVAL
    assert L.urv_qr_adjoint(None, P, 5, 3, None, None, P, 0, None) == urv.URV_EINVAL
    # with URV_TAPE_NONE no tape is needed
    o_none = _gopts(tape_mode=2)
    assert L.urv_tape_bytes(5, 3, 2, ctypes.byref(o_none)) == 0


def test_tape_and_workspace_sizes():
    L = urv.lib()
    sizes = {}
    for mode in (0, 1, 2):
        sizes[mode] = L.urv_tape_bytes(1000, 500, 2, ctypes.byref(_gopts(tape_mode=mode)))
    assert sizes[0] > sizes[1] > sizes[2] == 0
    assert L.urv_tape_bytes(1000, 500, 0, ctypes.byref(_gopts())) == 0
    f64 = L.urv_tape_bytes(1000, 500, 2, ctypes.byref(_gopts()))
    f32 = L.urv_tape_bytes(1000, 500, 2, ctypes.byref(_gopts(precision=1)))
    assert f32 < f64
    half = L.urv_tape_bytes(1000, 500, 2, ctypes.byref(_gopts(variant=1)))
    assert half < f64  # HALF keeps no Rw
    w_small = L.urv_grad_workspace_size(100, 50, 2, ctypes.byref(_gopts()))
    w_big = L.urv_grad_workspace_size(1000, 500, 2, ctypes.byref(_gopts()))
    assert 0 < w_small < w_big
    assert L.urv_grad_workspace_size(3, 5, 2, ctypes.byref(_gopts())) == 0


# ---------------------------------------------------------------- batched entry points
def test_batch_create_validates_before_any_device_work():
    L = urv.lib()
    plan = ctypes.c_void_p()

    def create(ms, ns, q=1):
        arr_m = (ctypes.c_int64 * len(ms))(*ms)
        arr_n = (ctypes.c_int64 * len(ns))(*ns)
        return L.urv_batch_create(len(ms), arr_m, arr_n, q, 0, ctypes.byref(plan))

    assert create([10, 20], [5, 30]) == urv.URV_EINVAL      # n > m
    assert create([10, 20], [0, 3]) == urv.URV_EINVAL       # n = 0
    assert create([10], [5], q=-1) == urv.URV_EINVAL
    assert create([2000], [5]) == urv.URV_ENOTSUP           # more than 1024 rows
    assert L.urv_batch_create(0, None, None, 1, 0, ctypes.byref(plan)) == urv.URV_EINVAL
    assert L.urv_batch_create(1, None, None, 1, 0, None) == urv.URV_EINVAL
    assert plan.value is None


def test_batch_calls_reject_a_null_plan():
    L = urv.lib()
    assert L.urv_batch_run(None, None) == urv.URV_EINVAL
    assert L.urv_batch_run_graph(None, None) == urv.URV_EINVAL
    assert L.urv_batch_autotune(None, None, None) == urv.URV_EINVAL
    assert L.urv_batch_set_config(None, 16, 256, 1) == urv.URV_EINVAL
    assert L.urv_batch_status(None, None) == urv.URV_EINVAL
    assert L.urv_batch_set_buffers(None, None, None, None, None) == urv.URV_EINVAL
    L.urv_batch_destroy(None)


def test_dgemm_noalloc_rejects_shapes_beyond_its_static_scratch():
    L = urv.lib()
    # 256 x 256 output tiles (4) with a long sum: 64 splits of 256 x 256 doubles = 32 MiB fits;
    # 255 tiles of 128 x 128 with K = 3 * 256 split 3 ways need 3 * 255 * 16384 doubles = 100 MiB
    rc = L.urv_dgemm_noalloc(0, 0, 128 * 15, 128 * 17, 768, 1.0, FAKE, 128 * 15, FAKE, 768, 0.0, FAKE, 128 * 15, None)
    assert rc == -1
    assert b"static scratch" in L.urv_last_error()
    # bad arguments are rejected as by urv_dgemm
    assert L.urv_dgemm_noalloc(0, 0, -1, 4, 4, 1.0, FAKE, 4, FAKE, 4, 0.0, FAKE, 4, None) == -1
    assert L.urv_dgemm_noalloc(0, 0, 8, 4, 4, 1.0, FAKE, 7, FAKE, 4, 0.0, FAKE, 8, None) == -1
