"""Oracle parity on the code paths the kernels take at the benchmark's heights.

The QR panel spreads a panel of mp rows over ceil(mp / 256) workgroups, so
the row count decides which exchange and reduction paths run: 4097 and 8193
rows leave a one-row tail workgroup, 8000 rows is the 8000 x 8000 workload's
height, 16000 rows the mixed-precision workload's, and the largest accepted
height is the limit of the panel's co-resident grid.  Tall-skinny shapes keep
the oracle in seconds while every panel runs at full height.

The GEMM case reaches the unsplit 128 x 128 tile with 4 x 4 waves (at least
256 tiles, k >= 512) on small integers, where every product is exact.

Metrics: urv_metrics (recon, orthogonality, rank-k errors) is compared with the
oracle's on the same (A, U, R, V), including perturbed factors whose residuals
are far above rounding level.
"""
import numpy as np
import pytest

import urv_inputs as gen
from gpu_helpers import announce, to_gpu, to_np

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps
EPS32 = float(np.finfo(np.float32).eps)
TOL = 1e-11  # FP64 parity, normwise relative to ||A||_F (R and every rank-k error)


@pytest.fixture(scope="module")
def urv():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1812_06007_amd import urv as u

    u.lib()
    return u


# ---------------------------------------------------------------- Qpos at full height
TALL = [(4097, 130), (8000, 130), (8000, 256), (8193, 256), (16000, 130), (16000, 256)]


@pytest.mark.parametrize("m,n", TALL)
def test_qr_fp64_full_height(urv, orc, m, n):
    announce("qr fp64 full height", m, n)
    rng = np.random.default_rng(m + 3 * n)
    X = rng.standard_normal((m, n))
    Q, R = urv.qr_pos(to_gpu(X))
    Q, R = to_np(Q), to_np(R)
    Qo, Ro = orc.qr_pos(X)
    nx = np.linalg.norm(X)
    assert np.linalg.norm(R - Ro) <= 50 * n * EPS * nx, np.linalg.norm(R - Ro) / nx
    assert np.all(np.diag(R) >= 0) and np.array_equal(R, np.triu(R))
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 20 * n * EPS
    np.testing.assert_allclose(Q, Qo, rtol=0, atol=1e-11)


@pytest.mark.parametrize("m,n", TALL)
def test_qr_fp32_full_height(urv, orc, m, n):
    announce("qr fp32 full height", m, n)
    rng = np.random.default_rng(7 * m + n)
    X = rng.standard_normal((m, n)).astype(np.float32).astype(np.float64)
    Q, R = urv.qr_pos(to_gpu(X), fp32=True)
    Q, R = to_np(Q), to_np(R)
    _, Ro = orc.qr_pos(X)
    nx = np.linalg.norm(X)
    assert np.linalg.norm(R - Ro) <= 50 * n * EPS32 * nx, np.linalg.norm(R - Ro) / nx
    assert np.all(np.diag(R) >= 0) and np.array_equal(R, np.triu(R))
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 20 * n * EPS32
    assert np.linalg.norm(Q @ R - X) <= 20 * n * EPS32 * nx


def test_qr_fp64_largest_accepted_height(urv, orc):
    """The tallest matrix the library accepts, factored and compared with the oracle."""
    m = urv.max_rows()
    n = 130
    announce("qr fp64 largest height", m, n)
    rng = np.random.default_rng(99)
    X = rng.standard_normal((m, n))
    Q, R = urv.qr_pos(to_gpu(X))
    Q, R = to_np(Q), to_np(R)
    _, Ro = orc.qr_pos(X)
    nx = np.linalg.norm(X)
    assert np.linalg.norm(R - Ro) <= 50 * n * EPS * nx, np.linalg.norm(R - Ro) / nx
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 20 * n * EPS
    assert np.linalg.norm(Q @ R - X) <= 20 * n * EPS * nx


def test_qr_above_largest_height_is_refused(urv):
    import torch

    m = urv.max_rows() + 1
    announce("qr refused height", m)
    X = torch.zeros((m, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(urv.UrvError) as e:
        urv.qr_pos(X)
    assert e.value.status == urv.URV_ENOTSUP


# ---------------------------------------------------------------- GEMM, unsplit 128 x 128 tiles
@pytest.mark.parametrize("ta", [False, True])
def test_dgemm_unsplit_large_tiles_bitwise(urv, orc, ta):
    M, N, K = 2048, 2048, 600
    announce("dgemm unsplit 128x128", ta)
    rng = np.random.default_rng(2048 + int(ta))
    A = rng.integers(-8, 9, size=(K, M) if ta else (M, K)).astype(np.float64)
    B = rng.integers(-8, 9, size=(K, N)).astype(np.float64)
    C0 = rng.integers(-8, 9, size=(M, N)).astype(np.float64)
    got = to_np(urv.dgemm(to_gpu(A), to_gpu(B), transA=ta, alpha=1.0, beta=-1.0, C=to_gpu(C0)))
    ref = orc.gemm(A, B, transA=ta, alpha=1.0, beta=-1.0, C=C0)
    np.testing.assert_array_equal(got, ref)


# ---------------------------------------------------------------- PowerURV at full height
def _factor(urv, A, q, **kw):
    U, R, V = urv.factor(to_gpu(A), q, **kw)
    return to_np(U), to_np(R), to_np(V)


@pytest.mark.parametrize("m", [8000, 16000])
def test_powerurv_full_fp64_full_height(urv, orc, m):
    n, q = 256, 2
    announce("powerurv full fp64", m, n, q)
    A = gen.spectral_matrix(m, n, gen.spectrum("geometric8", n), seed=m)
    G = gen.gaussian(n, n, m + 1)
    U, R, V = _factor(urv, A, q, G=to_gpu(G))
    Uo, Ro, Vo = orc.urv(A, q, G=G)
    na = np.linalg.norm(A)
    assert np.linalg.norm(R - Ro) <= TOL * na, np.linalg.norm(R - Ro) / na
    ek = orc.metrics(A, U, R, V)["ek"]
    eko = orc.metrics(A, Uo, Ro, Vo)["ek"]
    assert np.max(np.abs(ek - eko)) <= TOL * na
    met = urv.metrics(to_gpu(A), to_gpu(U), to_gpu(R), to_gpu(V))
    assert met["recon"] <= 20 * n * EPS and met["orthU"] <= 20 * n * EPS and met["orthV"] <= 20 * n * EPS, met


@pytest.mark.parametrize("m", [8000, 16000])
def test_powerurv_half_fp64_full_height(urv, orc, m):
    """HALF is compared with the oracle's own rounding spread between two summation orders."""
    n, q = 256, 2
    announce("powerurv half fp64", m, n, q)
    A = gen.spectral_matrix(m, n, gen.spectrum("geometric8", n), seed=m + 5)
    G = gen.gaussian(n, n, m + 6)
    ref = orc.urv(A, q, G=G, variant="half")
    with orc.sum_order(descending=True):
        ref2 = orc.urv(A, q, G=G, variant="half")
    na = np.linalg.norm(A)
    spread = max(np.linalg.norm(ref[1] - ref2[1]) / na, TOL)
    U, R, V = _factor(urv, A, q, G=to_gpu(G), variant="half")
    assert np.linalg.norm(R - ref[1]) / na <= 10 * spread
    ek = orc.metrics(A, U, R, V)["ek"]
    ek1 = orc.metrics(A, *ref)["ek"]
    ek2 = orc.metrics(A, *ref2)["ek"]
    assert np.max(np.abs(ek - ek1)) <= 10 * max(np.max(np.abs(ek1 - ek2)), TOL * na)


@pytest.mark.parametrize("m", [8000, 16000])
@pytest.mark.parametrize("variant", ["full", "half"])
def test_powerurv_mixed_bf16_full_height(urv, orc, m, variant):
    """16-bit products and FP32 QRs at full height: FP64-level reconstruction and orthogonality
    (the FP64 tail), and rank-k errors close to the FP64 oracle's where they are well above the
    16-bit rounding level."""
    n, q = 256, 2
    announce("powerurv mixed bf16", m, n, variant)
    sigma = np.exp(-10.0 * np.arange(1, n + 1) / n)
    A = gen.noisy_spectral_matrix(m, n, sigma, seed=m + 9, noise_var=1e-6)
    A = A.astype(np.float32).astype(np.float64)
    G = gen.gaussian(n, n, m + 10)
    U, R, V = _factor(urv, A, q, G=to_gpu(G), precision="mixed_bf16", variant=variant)
    met = urv.metrics(to_gpu(A), to_gpu(U), to_gpu(R), to_gpu(V))
    assert met["recon"] <= 1e-6 and met["recon"] <= 1e-12, met
    assert met["orthU"] <= 1e-12 and met["orthV"] <= 1e-12, met
    Uo, Ro, Vo = orc.urv(A, q, G=G, variant="full")
    eko = orc.metrics(A, Uo, Ro, Vo)["ek"]
    na = np.linalg.norm(A)
    sel = eko >= 0.05 * na
    ratio = met["ek"][sel] / eko[sel]
    print("[mixed full height] m=%d %s: max ek ratio %.4f, ||R-R64||/||A|| %.3e"
          % (m, variant, ratio.max(), np.linalg.norm(R - Ro) / na))
    assert ratio.max() <= 1.25
    s = np.linalg.svd(A, compute_uv=False)
    tail = np.sqrt(np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]]))
    assert np.all(met["ek"] >= tail * (1 - 1e-9) - 1e-13 * na)  # Eckart-Young


# ---------------------------------------------------------------- metrics against the oracle
def _metric_inputs(m, n, seed):
    A = gen.spectral_matrix(m, n, gen.spectrum("geometric8", n), seed=seed)
    rng = np.random.default_rng(seed)
    return A, rng


@pytest.mark.parametrize("m,n", [(300, 200), (2048, 700)])
def test_metrics_match_oracle_on_perturbed_factors(urv, orc, m, n):
    """Residuals around 1e-3: both sides compute them from the same bytes, so they agree to
    rounding relative to the residual itself."""
    announce("metrics perturbed", m, n)
    A, rng = _metric_inputs(m, n, 31 + m)
    Uo, Ro, Vo = orc.urv(A, 1, G=gen.gaussian(n, n, 32))
    U = Uo + 1e-3 * rng.standard_normal(Uo.shape) / np.sqrt(m)
    V = Vo + 2e-3 * rng.standard_normal(Vo.shape) / np.sqrt(n)
    R = np.triu(Ro + 1e-4 * rng.standard_normal(Ro.shape))
    got = urv.metrics(to_gpu(A), to_gpu(U), to_gpu(R), to_gpu(V))
    ref = orc.metrics(A, U, R, V)
    for key in ("recon", "orthU", "orthV", "normA"):
        assert ref[key] > 1e-5 or key == "normA"
        assert abs(got[key] - ref[key]) <= 1e-11 * ref[key], (key, got[key], ref[key])
    np.testing.assert_allclose(got["ek"], ref["ek"], rtol=1e-12, atol=1e-15 * ref["normA"])


def test_metrics_match_oracle_on_exact_factorisation(urv, orc):
    """At rounding level both sides' residuals are rounding noise: they agree absolutely."""
    m, n = 1000, 600
    announce("metrics exact", m, n)
    A, _ = _metric_inputs(m, n, 41)
    U, R, V = orc.urv(A, 2, G=gen.gaussian(n, n, 42))
    got = urv.metrics(to_gpu(A), to_gpu(U), to_gpu(R), to_gpu(V))
    ref = orc.metrics(A, U, R, V)
    for key in ("recon", "orthU", "orthV"):
        assert abs(got[key] - ref[key]) <= 20 * n * EPS, (key, got[key], ref[key])
    assert got["normA"] == pytest.approx(ref["normA"], rel=1e-14)
    np.testing.assert_allclose(got["ek"], ref["ek"], rtol=1e-12, atol=1e-15 * ref["normA"])


def test_metrics_closed_forms(urv):
    """U = [I; 0] D, V = P (a permutation), R diagonal: every metric has a closed form.
    With A = U R V^T + E for integer E, recon = ||E|| / ||A||."""
    m, n = 50, 20
    announce("metrics closed forms")
    rng = np.random.default_rng(5)
    d = rng.integers(1, 4, size=n).astype(np.float64)
    U = np.zeros((m, n))
    U[:n, :n] = np.diag(d)
    perm = rng.permutation(n)
    V = np.eye(n)[:, perm]
    R = np.diag(rng.integers(1, 9, size=n).astype(np.float64))
    E = rng.integers(-2, 3, size=(m, n)).astype(np.float64)
    A = U @ R @ V.T + E
    got = urv.metrics(to_gpu(A), to_gpu(U), to_gpu(R), to_gpu(V))
    assert got["recon"] == pytest.approx(np.sqrt(np.sum(E * E)) / np.sqrt(np.sum(A * A)), rel=1e-14)
    assert got["orthU"] == pytest.approx(np.sqrt(np.sum((d * d - 1) ** 2)), rel=1e-14)
    assert got["orthV"] == 0.0
    r = np.diag(R)
    assert got["ek"][0] == pytest.approx(np.sqrt(np.sum(r * r)), rel=1e-14)
    assert got["ek"][n] == 0.0
