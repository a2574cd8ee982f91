"""The QR pipeline's alternative schedules and its failure path, through the C ABI.

qr_pos runs the factorisation on several streams (block factorisations,
near and bulk trailing updates, the products with A, A^T and I).  The
schedule variants selectable for tuning -- 256-column outer blocks, targets
per 128-column block instead of per pair, the two panels of a 128-column
block in separate launches with GEMM updates between them, and with the T
join done by a GEMM and a separate kernel, and each block's factorisation
queued behind the update of its columns instead of ahead of it -- must give the oracle's factorisation to the
same 1e-11 tolerance as the default one.

The failure path: with URV_PANEL_EXPIRE_TEST=1 every device-wide wait of the
panel kernel expects a tag that is never published and gives up after a short
bounded spin (every kernel still returns).  The blocking urv_factor must then
report URV_EDEVICE, the outputs must be NaN, and the next call must succeed.
"""
import ctypes

import numpy as np
import pytest

import urv_inputs as gen
from gpu_helpers import announce, to_gpu, to_np

pytestmark = pytest.mark.gpu
TOL = 1e-11
URV_EDEVICE = -3


@pytest.fixture(scope="module")
def urv():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1812_06007_amd import urv as u

    u.lib()
    return u


def _parity(urv, orc, m, n, q, seed):
    A = gen.spectral_matrix(m, n, gen.spectrum("geometric8", n), seed=seed)
    G = gen.gaussian(n, n, seed + 1)
    U, R, V = (to_np(t) for t in urv.factor(to_gpu(A), q, G=to_gpu(G)))
    ref = orc.urv(A, q, G=G)
    na = np.linalg.norm(A)
    assert np.linalg.norm(R - ref[1]) <= TOL * na, np.linalg.norm(R - ref[1]) / na
    ek = np.sqrt(np.cumsum((np.triu(R) ** 2).sum(axis=1)[::-1])[::-1])
    ek_ref = np.sqrt(np.cumsum((np.triu(ref[1]) ** 2).sum(axis=1)[::-1])[::-1])
    assert np.max(np.abs(ek - ek_ref)) <= TOL * na
    assert np.linalg.norm(A - U @ R @ V.T) <= 1e-13 * na
    assert np.linalg.norm(U.T @ U - np.eye(n)) <= 1e-12 * n
    assert np.linalg.norm(V.T @ V - np.eye(n)) <= 1e-12 * n


@pytest.mark.parametrize("env", [
    {"URV_QR_BLOCK": "256"},
    {"URV_TARGET_PAIRS": "0"},
    {"URV_PANEL_FUSED": "0"},
    {"URV_PANEL_FUSED": "0", "URV_PANEL_JOIN": "0"},
    {"URV_PANEL_EARLY": "0"},
    {"URV_TARGET_LAG": "0"},
    {"URV_TARGET_LAG": "1000"},
    {"URV_QR_BLOCK": "256", "URV_PANEL_FUSED": "0", "URV_PANEL_JOIN": "0", "URV_TARGET_PAIRS": "0",
     "URV_PANEL_EARLY": "0", "URV_TARGET_LAG": "1"},
    {"URV_PANEL_EARLY": "1"},
    {"URV_PANEL_PREV": "0"},
    {"URV_PANEL_PREV": "0", "URV_PANEL_EARLY": "0"},
    {"URV_PANEL_CHOL": "0"},
    {"URV_PANEL_TSQR": "0"},
    {"URV_BULK_PAIRS": "1"},
    {"URV_BULK_PAIRS": "1", "URV_PANEL_PREV": "0"},
    {"URV_LOOKAHEAD": "1"},
    {"URV_LOOKAHEAD": "1", "URV_PANEL_PREV": "0", "URV_PANEL_EARLY": "0"},
    {"URV_DEFER_V": "0"},
    {"URV_LOOKAHEAD": "3"},
], ids=["block256", "no_pairs", "separate_panels", "no_join", "in_order", "targets_at_once", "targets_at_end",
        "all_off", "prev_flag_wait", "no_prev", "no_prev_in_order", "tall_skinny_only", "per_column_panel",
        "bulk_pairs", "bulk_pairs_no_prev", "lookahead1",
        "lookahead1_no_prev_in_order", "v_as_target", "lookahead3"])
@pytest.mark.parametrize("m,n", [(400, 400), (700, 520), (300, 197), (1100, 900)])
def test_schedule_variants_match_oracle(urv, orc, monkeypatch, env, m, n):
    announce("schedule", env, m, n)
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    _parity(urv, orc, m, n, 2, seed=m * 7 + n)


def test_target_lag_does_not_change_the_bits(urv, monkeypatch):
    """When the target products run (with their block, a few blocks later, or
    all after the last block) changes only the schedule: same operations in
    the same order, so the same bits."""
    announce("target lag bits")
    m, n = 900, 700
    A = to_gpu(gen.spectral_matrix(m, n, gen.spectrum("geometric8", n), seed=31))
    outs = []
    for lag in ("0", "3", "12", "1000"):
        monkeypatch.setenv("URV_TARGET_LAG", lag)
        outs.append([to_np(t) for t in urv.factor(A, 2, seed=32)])
    for other in outs[1:]:
        assert all(np.array_equal(a, b) for a, b in zip(outs[0], other))


def _blocking_factor(urv, A, q, seed):
    """urv_factor (FULL, FP64, blocking, packed) straight through the C ABI."""
    import torch

    m, n = A.shape
    Ad = to_gpu(A)
    assert Ad.stride(0) == 1
    U = urv.empty_colmajor(m, n)
    R = urv.empty_colmajor(n, n)
    V = urv.empty_colmajor(n, n)
    torch.cuda.synchronize()
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = urv.lib().urv_factor(p(Ad), m, n, q, seed, p(U), p(R), p(V))
    torch.cuda.synchronize()
    return rc, to_np(U), to_np(R), to_np(V)


def test_expired_panel_wait_is_reported_and_recovered(urv, monkeypatch):
    announce("expired wait")
    m, n = 600, 300
    A = gen.spectral_matrix(m, n, gen.spectrum("geometric8", n), seed=77)
    monkeypatch.setenv("URV_PANEL_EXPIRE_TEST", "1")
    rc, U, R, V = _blocking_factor(urv, A, 1, 5)
    assert rc == URV_EDEVICE
    assert b"wait expired" in urv.lib().urv_last_error()
    assert np.isnan(R).any() and np.isnan(U).any()
    monkeypatch.delenv("URV_PANEL_EXPIRE_TEST")
    rc, U, R, V = _blocking_factor(urv, A, 1, 5)
    assert rc == 0
    na = np.linalg.norm(A)
    assert np.all(np.isfinite(R))
    assert np.linalg.norm(A - U @ R @ V.T) <= 1e-13 * na


def test_async_expiry_is_reported_by_sync_status(urv, monkeypatch):
    """urv_factor_ex and urv_qr_pos are asynchronous: an expired panel wait reaches the caller
    through urv_sync_status, which the Python calls check by default."""
    import torch

    announce("expired wait, async")
    m, n = 600, 300
    A = to_gpu(gen.spectral_matrix(m, n, gen.spectrum("geometric8", n), seed=78))
    urv.sync_status()  # nothing pending
    monkeypatch.setenv("URV_PANEL_EXPIRE_TEST", "1")
    U, R, V = urv.factor(A, 1, seed=5, check=False)  # returns before the device work ends
    with pytest.raises(urv.UrvError) as ei:
        urv.sync_status()
    assert ei.value.status == urv.URV_EDEVICE
    assert torch.isnan(R).any()
    urv.sync_status()  # reported once, then clear
    with pytest.raises(urv.UrvError):
        urv.factor(A, 1, seed=5)  # check=True waits and raises
    with pytest.raises(urv.UrvError):
        urv.qr_pos(A)
    monkeypatch.delenv("URV_PANEL_EXPIRE_TEST")
    urv.sync_status()
    U, R, V = urv.factor(A, 1, seed=5)
    assert torch.isfinite(R).all()


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -float("inf")])
def test_check_finite_rejects_before_writing(urv, bad):
    import torch

    announce("check_finite", bad)
    m, n = 300, 200
    A = gen.spectral_matrix(m, n, gen.spectrum("geometric8", n), seed=3)
    A[17, 123] = bad
    Ad = to_gpu(A)
    outs = tuple(urv.empty_colmajor(r, c).fill_(7.0) for r, c in ((m, n), (n, n), (n, n)))
    with pytest.raises(urv.UrvError) as ei:
        urv.factor(Ad, 1, seed=2, check_finite=True, out=outs)
    assert ei.value.status == urv.URV_ENONFINITE
    for t in outs:
        assert bool((t == 7.0).all())
    # the same matrix, FP32, and without the check: NaN propagates, no error
    A32 = Ad.float()
    with pytest.raises(urv.UrvError):
        urv.factor(A32, 1, seed=2, check_finite=True)
    A[17, 123] = 0.5
    U, R, V = urv.factor(to_gpu(A), 1, seed=2, check_finite=True)
    assert torch.isfinite(R).all()


@pytest.mark.parametrize("prec", ["fp64", "mixed_bf16", "mixed_fp16"])
def test_fp32_a_equals_its_fp64_value(urv, prec):
    """An FP32 A gives bitwise the results of the FP64 matrix holding the same values: the
    16-bit casts round the same numbers and every FP64 step sees the exact values."""
    announce("fp32 A", prec)
    m, n = 700, 300
    A = gen.spectral_matrix(m, n, gen.spectrum("geometric8", n), seed=4).astype(np.float32)
    A32 = to_gpu(A.astype(np.float64)).float()
    A64 = to_gpu(A.astype(np.float64))
    got = [to_np(t) for t in urv.factor(A32, 2, seed=9, precision=prec, variant="half")]
    ref = [to_np(t) for t in urv.factor(A64, 2, seed=9, precision=prec, variant="half")]
    for g, r in zip(got, ref):
        np.testing.assert_array_equal(g, r)
