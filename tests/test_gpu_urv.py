"""Parity of the GPU PowerURV (urv_factor_ex through the C ABI) with the FP64
oracle, and its invariants at the full benchmark sizes.

Tolerances (normwise, relative to ||A||_F): R and every rank-k error e_k
within 1e-11 for FP64 with re-orthonormalisation after every product
(Section 3).  U and V are compared through invariants and the leading
projector, since their trailing columns are determined only to
~eps sigma_1 / sigma_j.
"""
import numpy as np
import pytest

import urv_inputs as gen
from gpu_helpers import announce, to_gpu, to_np

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps
TOL = 1e-11


@pytest.fixture(scope="module")
def urv():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1812_06007_amd import urv as u

    u.lib()
    return u


def _gpu_factor(urv, A, q, **kw):
    U, R, V = urv.factor(to_gpu(A), q, **kw)
    return to_np(U), to_np(R), to_np(V)


def _assert_parity(A, got, ref, tol=TOL, orc=None):
    U, R, V = got
    Uo, Ro, Vo = ref
    na = np.linalg.norm(A)
    assert np.linalg.norm(R - Ro) <= tol * na, np.linalg.norm(R - Ro) / na
    ek = orc.metrics(A, U, R, V)["ek"]
    eko = orc.metrics(A, Uo, Ro, Vo)["ek"]
    assert np.max(np.abs(ek - eko)) <= tol * na


def _assert_invariants(urv, A, got, tol):
    U, R, V = got
    m, n = A.shape
    met = urv.metrics(to_gpu(A), to_gpu(U), to_gpu(R), to_gpu(V))
    assert met["recon"] <= tol, met
    assert met["orthU"] <= tol, met
    assert met["orthV"] <= tol, met
    assert np.array_equal(R, np.triu(R))
    assert np.all(np.diag(R) >= 0)
    return met


# ------------------------------------------------ the 400 x 400 parity case
def test_c1_parity_given_g(urv, orc):
    """400 x 400, sigma_j = 10^(-8(j-1)/399), q = 2, FULL, same G on both sides."""
    announce("c1 given G")
    n = 400
    A = gen.spectral_matrix(n, n, gen.spectrum("geometric8", n), seed=1812)
    G = gen.gaussian(n, n, 1812)
    got = _gpu_factor(urv, A, 2, G=to_gpu(G))
    ref = orc.urv(A, 2, G=G)
    _assert_parity(A, got, ref, orc=orc)
    _assert_invariants(urv, A, got, 20 * n * EPS)


def test_c1_parity_seeded_g(urv, orc):
    """Same case with G drawn from the seed on each side (Philox4x64-10 + Box-Muller)."""
    announce("c1 seeded")
    n = 400
    A = gen.spectral_matrix(n, n, gen.spectrum("geometric8", n), seed=1812)
    got = _gpu_factor(urv, A, 2, seed=1812)
    ref = orc.urv(A, 2, seed=1812)
    _assert_parity(A, got, ref, orc=orc)


@pytest.mark.parametrize("m,n", [(1, 1), (2, 1), (3, 3), (65, 64), (129, 128), (301, 197), (1000, 300), (700, 700)])
@pytest.mark.parametrize("q", [0, 1, 2])
def test_full_variant_parity_shapes(urv, orc, m, n, q):
    announce("full parity", m, n, q)
    A = gen.spectral_matrix(m, n, gen.spectrum("geometric8", n), seed=m + n)
    G = gen.gaussian(n, n, m * n)
    got = _gpu_factor(urv, A, q, G=to_gpu(G))
    ref = orc.urv(A, q, G=G)
    _assert_parity(A, got, ref, orc=orc)
    _assert_invariants(urv, A, got, 20 * max(n, 4) * EPS)


@pytest.mark.parametrize("q", [1, 2])
def test_half_variant_within_oracle_spread(urv, orc, q):
    """HALF loses directions below sqrt(eps) sigma_1; the GPU must sit within 10x the oracle's
    own spread between two summation orders."""
    announce("half", q)
    n = 300
    A = gen.spectral_matrix(n, n, gen.spectrum("geometric8", n), seed=2)
    G = gen.gaussian(n, n, 3)
    ref = orc.urv(A, q, G=G, variant="half")
    with orc.sum_order(descending=True):
        ref2 = orc.urv(A, q, G=G, variant="half")
    na = np.linalg.norm(A)
    spread = max(np.linalg.norm(ref[1] - ref2[1]) / na, TOL)
    got = _gpu_factor(urv, A, q, G=to_gpu(G), variant="half")
    assert np.linalg.norm(got[1] - ref[1]) / na <= 10 * spread
    _assert_invariants(urv, A, got, 20 * n * EPS)


@pytest.mark.parametrize("q", [1, 2])
def test_none_variant_mild_spectrum(urv, orc, q):
    announce("none", q)
    A = gen.spectral_matrix(500, 300, np.linspace(1.0, 0.1, 300), seed=4)
    G = gen.gaussian(300, 300, 5)
    got = _gpu_factor(urv, A, q, G=to_gpu(G), variant="none")
    ref = orc.urv(A, q, G=G, variant="none")
    _assert_parity(A, got, ref, orc=orc)


def test_orth_g_option(urv, orc):
    announce("orth_g")
    A = gen.spectral_matrix(200, 150, gen.spectrum("matrix2", 150), seed=8)
    G = gen.gaussian(150, 150, 9)
    got = _gpu_factor(urv, A, 1, G=to_gpu(G), orth_g=True)
    ref = orc.urv(A, 1, G=G, orth_g=True)
    _assert_parity(A, got, ref, orc=orc)


# ------------------------------------------------ reductions and exact cases
def test_kahan_q0_identity_start_exact(urv):
    """Unpivoted QR is a URV with V = I (Section 1): Kahan's triangular matrix comes back exactly."""
    announce("kahan exact")
    n = 300
    K = gen.kahan(n)
    U, R, V = _gpu_factor(urv, K, 0, G=to_gpu(np.eye(n)))
    np.testing.assert_array_equal(U, np.eye(n))
    np.testing.assert_array_equal(R, K)
    np.testing.assert_array_equal(V, np.eye(n))


def test_lemma_on_gpu_output(urv):
    """Section 6 Lemma: U(:,1:l) spans A (A^T A)^q G(:,1:l)."""
    announce("lemma")
    m, n, l, q = 300, 200, 60, 1
    A = gen.spectral_matrix(m, n, np.linspace(1.0, 0.2, n), seed=10)
    G = gen.gaussian(n, n, 11)
    U, _, _ = _gpu_factor(urv, A, q, G=to_gpu(G))
    Y = G[:, :l]
    for _ in range(q):
        Y = A.T @ (A @ Y)
    Ql, _ = np.linalg.qr(A @ Y)
    assert np.linalg.norm(U[:, :l] @ U[:, :l].T - Ql @ Ql.T, 2) < 1e-10


def test_determinism_scaling_and_prefix(urv):
    announce("determinism")
    m, n = 600, 300
    A = gen.spectral_matrix(m, n, gen.spectrum("geometric8", n), seed=12)
    G = gen.gaussian(n, n, 13)
    a = _gpu_factor(urv, A, 2, G=to_gpu(G))
    b = _gpu_factor(urv, A, 2, G=to_gpu(G))
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    s = _gpu_factor(urv, A * 2.0**6, 2, G=to_gpu(G))
    np.testing.assert_array_equal(s[0], a[0])
    np.testing.assert_array_equal(s[2], a[2])
    np.testing.assert_array_equal(s[1], a[1] * 2.0**6)
    G2 = G.copy()
    G2[:, 150:] = gen.gaussian(n, n - 150, 14)
    p = _gpu_factor(urv, A, 2, G=to_gpu(G2))
    np.testing.assert_array_equal(p[0][:, :150], a[0][:, :150])
    np.testing.assert_array_equal(p[1][:150, :150], a[1][:150, :150])
    np.testing.assert_array_equal(p[2][:, :150], a[2][:, :150])


def test_empty_and_tiny(urv):
    import torch

    announce("empty")
    U, R, V = urv.factor(torch.zeros((5, 0), dtype=torch.float64, device="cuda"), 1)
    assert U.shape == (5, 0) and R.shape == (0, 0) and V.shape == (0, 0)
    U, R, V = _gpu_factor(urv, np.array([[-3.0]]), 2, seed=1)
    assert abs(R[0, 0] - 3.0) < 1e-15 and abs(abs(U[0, 0]) - 1) < 1e-15 and abs(abs(V[0, 0]) - 1) < 1e-15
    assert abs(U[0, 0] * R[0, 0] * V[0, 0] + 3.0) < 1e-15


# ------------------------------------------------ full benchmark sizes
def _spectral_on_gpu(m, n, kind, seed):
    import torch

    sigma = gen.spectrum(kind, n)
    A = gen.spectral_matrix(m, n, sigma, seed, device="cuda")
    torch.cuda.synchronize()
    return A, sigma


@pytest.mark.parametrize("q", [0, 2])
def test_full_size_8000_properties(urv, q):
    """8000 x 8000, sigma_j = 1/j^2, FULL, in the benchmark's configuration: closed forms of
    the spectrum, invariants and the Eckart-Young bounds of every rank-k error."""
    announce("8000 properties", q)
    import torch

    n = 8000
    A, sigma = _spectral_on_gpu(n, n, "poly2", 1812)
    ws = torch.empty(urv.workspace_size(n, n, q), dtype=torch.uint8, device="cuda")
    U, R, V = urv.factor(A, q, seed=1812, workspace=ws)
    met = urv.metrics(A, U, R, V)
    assert met["recon"] < 1e-12 and met["orthU"] < 1e-10 and met["orthV"] < 1e-10, met
    sums = gen.sigma_sums(sigma)
    Rn = R.cpu().numpy()
    assert np.linalg.norm(Rn) == pytest.approx(sums["fro"], rel=1e-12)
    d = np.abs(np.diag(Rn))
    assert np.all(np.diag(Rn) >= 0)
    assert np.sum(np.log10(d)) == pytest.approx(sums["log10det"], abs=1e-2)
    ek = met["ek"]
    assert np.all(ek >= sums["tail"] * (1 - 1e-8) - 1e-13 * sums["fro"])
    if q == 2:
        # with two power steps the trailing blocks track the optimal errors closely (Section 3)
        k = np.arange(1, n, 500)
        assert np.all(ek[k] <= 10 * sums["tail"][k])


def test_full_size_kahan_4000(urv):
    announce("kahan 4000")
    import torch

    n = 4000
    K = torch.from_numpy(np.ascontiguousarray(gen.kahan(n).T)).cuda().t()
    for q in (0, 1, 2):
        U, R, V = urv.factor(K, q, seed=1812)
        met = urv.metrics(K, U, R, V)
        assert met["recon"] < 1e-12 and met["orthU"] < 1e-10 and met["orthV"] < 1e-10, (q, met)
        assert np.linalg.norm(R.cpu().numpy()) == pytest.approx(np.sqrt(n), rel=1e-12)


# ------------------------------------------------ mixed precision (BF16 / FP16 products, FP32 QR, FP64 tail)
@pytest.mark.parametrize("tile", ["128", "256"])
@pytest.mark.parametrize("prec", ["mixed_bf16", "mixed_fp16"])
@pytest.mark.parametrize("variant", ["full", "half"])
def test_mixed_precision_against_fp64_oracle(urv, orc, monkeypatch, prec, variant, tile):
    """Reconstruction and orthogonality stay at FP64 level (the FP64 re-orthonormalisation and
    tail); the rank-k errors stay close to the FP64 oracle's where sigma_k is well above the
    16-bit rounding level, and never beat the Eckart-Young bound.  Both tile shapes of the
    16-bit products (the 256 x 256 one is chosen by itself only for outputs of 256 such tiles)
    run here, with ragged edges and a K that ends inside a K step."""
    announce("mixed", prec, variant, tile)
    monkeypatch.setenv("URV_LOWP_TILE", tile)
    m, n = 1200, 600
    sigma = np.exp(-10.0 * np.arange(1, n + 1) / n)  # the same decay range as exp(-j/800), j <= 8000
    A = gen.noisy_spectral_matrix(m, n, sigma, seed=7, noise_var=1e-6)
    A = A.astype(np.float32).astype(np.float64)  # the input is an FP32 matrix
    G = gen.gaussian(n, n, 8)
    U, R, V = _gpu_factor(urv, A, 2, G=to_gpu(G), precision=prec, variant=variant)
    met = _assert_invariants(urv, A, (U, R, V), 1e-10)
    assert met["recon"] <= 1e-6
    Uo, Ro, Vo = orc.urv(A, 2, G=G, variant="full")
    eko = orc.metrics(A, Uo, Ro, Vo)["ek"]
    ek = met["ek"]
    na = np.linalg.norm(A)
    s = np.linalg.svd(A, compute_uv=False)
    tail = np.sqrt(np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]]))
    assert np.all(ek >= tail * (1 - 1e-9) - 1e-13 * na)
    sel = eko >= 0.05 * na
    ratio = ek[sel] / eko[sel]
    print("[mixed] %s %s: max ek ratio (ek >= 5%% ||A||) %.4f, ||R-R64||/||A|| %.3e"
          % (prec, variant, ratio.max(), np.linalg.norm(R - Ro) / na))
    assert ratio.max() <= 1.25


@pytest.mark.parametrize("itarget", ["1", "0"])
@pytest.mark.parametrize("variant", ["full", "half"])
def test_mixed_square_both_q_formations(urv, orc, monkeypatch, variant, itarget):
    """A square A: the FP32 QRs of X and Y form their explicit Q from I alongside the
    factorisation (the default) or backward after it; both meet the FP64 oracle as the tall
    case does."""
    announce("mixed square", variant, itarget)
    monkeypatch.setenv("URV_MIXED_ITARGET", itarget)
    n = 700
    sigma = np.exp(-10.0 * np.arange(1, n + 1) / n)
    A = gen.noisy_spectral_matrix(n, n, sigma, seed=17, noise_var=1e-6)
    A = A.astype(np.float32).astype(np.float64)
    G = gen.gaussian(n, n, 18)
    U, R, V = _gpu_factor(urv, A, 2, G=to_gpu(G), precision="mixed_bf16", variant=variant)
    met = _assert_invariants(urv, A, (U, R, V), 1e-10)
    assert met["recon"] <= 1e-6
    Uo, Ro, Vo = orc.urv(A, 2, G=G, variant="full")
    eko = orc.metrics(A, Uo, Ro, Vo)["ek"]
    na = np.linalg.norm(A)
    sel = eko >= 0.05 * na
    ratio = met["ek"][sel] / eko[sel]
    print("[mixed square] %s itarget=%s: max ek ratio %.4f" % (variant, itarget, ratio.max()))
    assert ratio.max() <= 1.25


@pytest.mark.parametrize("variant", ["full", "half", "none"])
def test_fp16_large_entries_scaled_not_overflowed(urv, orc, variant):
    """||A|| ~ 1e6, entries far beyond FP16's 65504: the FP16 casts scale each operand by a
    power of two (exact; Qpos is scale invariant), so the result matches the BF16 mode and the
    FP64 oracle's rank-k errors as it does at unit scale."""
    announce("fp16 scaled", variant)
    m, n = 800, 400
    sigma = 1e6 * np.exp(-8.0 * np.arange(1, n + 1) / n)
    A = gen.noisy_spectral_matrix(m, n, sigma, seed=21, noise_var=1e-6)
    G = gen.gaussian(n, n, 3)
    q = 1 if variant == "none" else 2
    U, R, V = _gpu_factor(urv, A, q, G=to_gpu(G), precision="mixed_fp16", variant=variant)
    assert np.all(np.isfinite(R))
    met = _assert_invariants(urv, A, (U, R, V), 1e-10)
    assert met["recon"] <= 1e-12
    Uo, Ro, Vo = orc.urv(A, q, G=G, variant="full")
    eko = orc.metrics(A, Uo, Ro, Vo)["ek"]
    na = np.linalg.norm(A)
    sel = eko >= 0.05 * na
    ratio = met["ek"][sel] / eko[sel]
    print("[fp16 scaled] %s: max ek ratio %.4f" % (variant, ratio.max()))
    assert ratio.max() <= 1.25
