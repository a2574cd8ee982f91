"""Parity of the HIP kernels with the FP64 oracle, through the C ABI:
the Gaussian of eq. power, the FP64 MFMA GEMM, and Qpos (blocked Householder QR
with diag(R) >= 0, Section 2.2)."""
import numpy as np
import pytest

import urv_inputs as gen
from gpu_helpers import announce, to_gpu, to_np

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def urv():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1812_06007_amd import urv as u

    u.lib()
    return u


# ---------------------------------------------------------------- Gaussian
@pytest.mark.parametrize("rows,cols,seed,stream", [(1, 1, 0, 2), (7, 9, 1812, 2), (400, 400, 1812, 2),
                                                    (1000, 37, 2**63 + 11, 3), (3, 1001, 5, 0)])
def test_gaussian_matches_oracle(urv, orc, rows, cols, seed, stream):
    announce("gaussian", rows, cols, seed, stream)
    import torch

    G = to_np(urv.gaussian(rows, cols, seed, stream_id=stream))
    ref = orc.gaussian(rows, cols, seed, stream_id=stream)
    # same Philox words; log/sin/cos differ between libm and the device library by a few ulp
    np.testing.assert_allclose(G, ref, rtol=0, atol=1e-14 * max(1.0, np.abs(ref).max()))
    G32 = urv.gaussian(rows, cols, seed, stream_id=stream, dtype=torch.float32)
    np.testing.assert_array_equal(G32.cpu().numpy(), torch.from_numpy(G).float().numpy())


def test_gaussian_layout(urv):
    announce("gaussian layout")
    G = to_np(urv.gaussian(33, 17, 9))
    flat = to_np(urv.gaussian(1, 33 * 17, 9)).reshape(-1)
    np.testing.assert_array_equal(G.reshape(-1, order="F"), flat)


# ---------------------------------------------------------------- GEMM
SHAPES = [(1, 1, 1), (7, 5, 3), (64, 64, 64), (65, 129, 17), (128, 128, 128), (300, 200, 513),
          (64, 300, 5000), (64, 64, 20000), (1, 700, 2049), (257, 1, 300),
          # short sums over >= 256 tiles of 128 x 128: the 128 x 64, k-step 16 variant (edge tiles in m and n)
          (2100, 2050, 200), (2048, 2048, 128)]


@pytest.mark.parametrize("ta", [False, True])
@pytest.mark.parametrize("tb", [False, True])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_dgemm_integer_inputs_bitwise(urv, orc, ta, tb, shape):
    M, N, K = shape
    announce("dgemm int", ta, tb, shape)
    rng = np.random.default_rng(M + 7 * N + 13 * K)
    A = rng.integers(-8, 9, size=(K, M) if ta else (M, K)).astype(np.float64)
    B = rng.integers(-8, 9, size=(N, K) if tb else (K, N)).astype(np.float64)
    C0 = rng.integers(-8, 9, size=(M, N)).astype(np.float64)
    got = to_np(urv.dgemm(to_gpu(A), to_gpu(B), transA=ta, transB=tb, alpha=2.0, beta=-3.0, C=to_gpu(C0)))
    ref = orc.gemm(A, B, transA=ta, transB=tb, alpha=2.0, beta=-3.0, C=C0)
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True)])
@pytest.mark.parametrize("shape", [(200, 150, 300), (64, 1000, 8000), (513, 64, 64)])
def test_dgemm_random_within_error_bound(urv, orc, ta, tb, shape):
    M, N, K = shape
    announce("dgemm rand", ta, tb, shape)
    rng = np.random.default_rng(3)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    got = to_np(urv.dgemm(to_gpu(A), to_gpu(B), transA=ta, transB=tb))
    ref = orc.gemm(A, B, transA=ta, transB=tb)
    bound = orc.gemm(np.abs(A), np.abs(B), transA=ta, transB=tb)
    assert np.all(np.abs(got - ref) <= 2 * K * EPS * bound)


def test_dgemm_leading_dimensions_and_beta_zero(urv, orc):
    import torch

    announce("dgemm ld")
    rng = np.random.default_rng(4)
    A = rng.integers(-4, 5, size=(70, 40)).astype(np.float64)
    B = rng.integers(-4, 5, size=(40, 50)).astype(np.float64)
    Abig = torch.zeros((60, 100), dtype=torch.float64, device="cuda").t()  # ld 100
    Abig[:70, :40] = to_gpu(A)
    Cbig = torch.full((60, 90), float("nan"), dtype=torch.float64, device="cuda").t()  # ld 90, NaN
    C = Cbig[:70, :50]
    urv.dgemm(Abig[:70, :40], to_gpu(B), beta=0.0, C=C)
    np.testing.assert_array_equal(to_np(C), A @ B)
    assert torch.isnan(Cbig[70:, :]).all()  # rows beyond M untouched


@pytest.mark.parametrize("ta", [False, True])
@pytest.mark.parametrize("tb", [False, True])
@pytest.mark.parametrize("layout", ["odd_ld", "offset_by_one", "aligned"])
def test_dgemm_operand_alignment(urv, ta, tb, layout):
    """Full 128 x 128 tiles load pairs of elements with one 16-byte load only
    when both operands are 16-byte aligned with even leading dimensions; odd
    leading dimensions and operands starting one element in take the
    element-by-element loads.  Small integers: every product is exact."""
    import torch

    announce("dgemm alignment", ta, tb, layout)
    rng = np.random.default_rng(11)
    M, N, K = 300, 260, 200
    A = rng.integers(-4, 5, size=(K, M) if ta else (M, K)).astype(np.float64)
    B = rng.integers(-4, 5, size=(N, K) if tb else (K, N)).astype(np.float64)

    def place(X):
        r, c = X.shape
        if layout == "aligned":
            return to_gpu(X)
        extra = 1 if layout == "odd_ld" else 2
        big = torch.zeros((c + 1, r + extra), dtype=torch.float64, device="cuda").t()  # ld r + extra
        off = 0 if layout == "odd_ld" else 1
        big[off:off + r, :c] = to_gpu(X)
        view = big[off:off + r, :c]
        assert view.stride(1) == r + extra
        assert (view.data_ptr() % 16 != 0) == (layout == "offset_by_one")
        return view

    C = urv.dgemm(place(A), place(B), ta, tb)
    ref = (A.T if ta else A) @ (B.T if tb else B)
    np.testing.assert_array_equal(to_np(C), ref)


def test_dgemm_is_deterministic(urv):
    announce("dgemm determinism")
    rng = np.random.default_rng(5)
    A = to_gpu(rng.standard_normal((5000, 64)))
    C = to_gpu(rng.standard_normal((5000, 900)))
    r1 = to_np(urv.dgemm(A, C, transA=True))
    r2 = to_np(urv.dgemm(A, C, transA=True))
    np.testing.assert_array_equal(r1, r2)


# ---------------------------------------------------------------- Qpos
QR_SHAPES = [(1, 1), (5, 1), (7, 3), (64, 64), (65, 64), (129, 65), (300, 300), (513, 200),
             (1000, 257), (2000, 130)]


@pytest.mark.parametrize("m,n", QR_SHAPES)
def test_qr_matches_oracle(urv, orc, m, n):
    announce("qr", m, n)
    rng = np.random.default_rng(m * 31 + n)
    X = rng.standard_normal((m, n))
    Q, R = urv.qr_pos(to_gpu(X))
    Q, R = to_np(Q), to_np(R)
    Qo, Ro = orc.qr_pos(X)
    nx = np.linalg.norm(X)
    assert np.linalg.norm(R - Ro) <= 50 * n * EPS * nx
    assert np.all(np.diag(R) >= 0)
    assert np.array_equal(R, np.triu(R))
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 20 * n * EPS
    assert np.linalg.norm(Q @ R - X) <= 20 * n * EPS * nx
    # a Gaussian X is well conditioned: Q is determined to ~eps
    np.testing.assert_allclose(Q, Qo, rtol=0, atol=1e-11)


@pytest.mark.parametrize("n", [10, 64, 65, 300])
def test_qr_of_positive_triangular_is_exact(urv, n):
    announce("qr kahan", n)
    K = gen.kahan(n)
    Q, R = urv.qr_pos(to_gpu(K))
    np.testing.assert_array_equal(to_np(Q), np.eye(n))
    np.testing.assert_array_equal(to_np(R), K)


def test_qr_rank_deficient(urv):
    announce("qr rank deficient")
    rng = np.random.default_rng(6)
    X = rng.standard_normal((300, 100))
    X[:, 10] = 0.0
    X[:, 70] = X[:, 3]
    Q, R = urv.qr_pos(to_gpu(X))
    Q, R = to_np(Q), to_np(R)
    assert abs(R[10, 10]) < 1e-14
    assert abs(R[70, 70]) < 1e-12
    assert np.linalg.norm(Q.T @ Q - np.eye(100)) < 1e-12
    assert np.linalg.norm(Q @ R - X) < 1e-13 * np.linalg.norm(X)


def test_qr_power_of_two_scaling_bitwise(urv):
    announce("qr scaling")
    rng = np.random.default_rng(7)
    X = rng.standard_normal((400, 150))
    Q1, R1 = urv.qr_pos(to_gpu(X))
    Q2, R2 = urv.qr_pos(to_gpu(X * 2.0**-9))
    np.testing.assert_array_equal(to_np(Q1), to_np(Q2))
    np.testing.assert_array_equal(to_np(R1) * 2.0**-9, to_np(R2))


# ---------------------------------------------------------------- Qpos in FP32 (mixed-precision form)
@pytest.mark.parametrize("m,n", [(1, 1), (7, 3), (65, 64), (300, 300), (1000, 257), (2000, 130)])
def test_qr_fp32_matches_oracle(urv, orc, m, n):
    announce("qr fp32", m, n)
    rng = np.random.default_rng(m * 17 + n)
    X = rng.standard_normal((m, n)).astype(np.float32).astype(np.float64)  # exactly representable
    Q, R = urv.qr_pos(to_gpu(X), fp32=True)
    Q, R = to_np(Q), to_np(R)
    Qo, Ro = orc.qr_pos(X)
    eps32 = float(np.finfo(np.float32).eps)
    nx = np.linalg.norm(X)
    assert np.linalg.norm(R - Ro) <= 50 * max(n, 4) * eps32 * nx
    assert np.all(np.diag(R) >= 0) and np.array_equal(R, np.triu(R))
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 20 * max(n, 4) * eps32
    assert np.linalg.norm(Q @ R - X) <= 20 * max(n, 4) * eps32 * nx


def test_qr_fp32_kahan_exact(urv):
    announce("qr fp32 kahan")
    K = gen.kahan(100).astype(np.float32).astype(np.float64)
    Q, R = urv.qr_pos(to_gpu(K), fp32=True)
    np.testing.assert_array_equal(to_np(Q), np.eye(100))
    np.testing.assert_array_equal(to_np(R), K)
