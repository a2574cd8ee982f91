"""Pins of the oracle's building blocks: matrix product, Householder QR with
positive diagonal (Section 2.2 and its footnote), Jacobi SVD.

Each pin comes from outside the oracle: exact integer arithmetic, worked
examples derived by hand (tests/golden), textbook Cholesky and modified
Gram-Schmidt written here, and LAPACK through numpy as a library check.
"""
import json
import math
import os

import numpy as np
import pytest

import urv_inputs as gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EPS = np.finfo(np.float64).eps


# ---------------------------------------------------------------- products
@pytest.mark.parametrize("ta", [False, True])
@pytest.mark.parametrize("tb", [False, True])
@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 3, 7), (33, 17, 65), (64, 1, 9)])
def test_gemm_small_integers_exact(orc, ta, tb, shape):
    M, N, K = shape
    rng = np.random.default_rng(M * 100 + N * 10 + K)
    A = rng.integers(-8, 9, size=(K, M) if ta else (M, K)).astype(np.float64)
    B = rng.integers(-8, 9, size=(N, K) if tb else (K, N)).astype(np.float64)
    C0 = rng.integers(-8, 9, size=(M, N)).astype(np.float64)
    opA = A.T if ta else A
    opB = B.T if tb else B
    got = orc.gemm(A, B, transA=ta, transB=tb)
    np.testing.assert_array_equal(got, opA @ opB)
    got = orc.gemm(A, B, transA=ta, transB=tb, alpha=-2.0, beta=3.0, C=C0)
    np.testing.assert_array_equal(got, -2.0 * (opA @ opB) + 3.0 * C0)
    with orc.sum_order(descending=True):
        np.testing.assert_array_equal(orc.gemm(A, B, transA=ta, transB=tb), opA @ opB)


def test_gemm_beta_zero_ignores_nan(orc):
    A = np.ones((3, 2))
    B = np.ones((2, 4))
    C = np.full((3, 4), np.nan)
    np.testing.assert_array_equal(orc.gemm(A, B, beta=0.0, C=C), np.full((3, 4), 2.0))


# ---------------------------------------------------------------- QR
def _ev(s):
    return eval(s, {"__builtins__": {}}, {"sqrt": math.sqrt})


def _golden_cases():
    with open(os.path.join(GOLDEN, "qr_worked_examples.json")) as f:
        d = json.load(f)
    out = []
    for c in d["cases"]:
        conv = lambda rows: np.array([[_ev(x) for x in r] for r in rows], dtype=np.float64)
        out.append((c["name"], conv(c["X"]), conv(c["Q"]), conv(c["R"])))
    return out


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c[0])
def test_qr_worked_examples(orc, case):
    _, X, Qe, Re = case
    Q, R = orc.qr_pos(X)
    np.testing.assert_allclose(Q, Qe, rtol=0, atol=4 * EPS)
    np.testing.assert_allclose(R, Re, rtol=0, atol=8 * EPS * np.abs(Re).max())


@pytest.mark.parametrize("n", [1, 2, 7, 60, 100])
def test_qr_of_positive_triangular_is_exact(orc, n):
    """Upper-triangular input with positive diagonal: Q = I and R = input, bitwise
    (every reflector is the identity because the part below the diagonal is 0)."""
    K = gen.kahan(n)
    Q, R = orc.qr_pos(K)
    np.testing.assert_array_equal(Q, np.eye(n))
    np.testing.assert_array_equal(R, K)


def _cholesky_upper(S):
    """Textbook Cholesky S = R^T R, R upper, computed row by row."""
    n = S.shape[0]
    R = np.zeros_like(S)
    for i in range(n):
        d = S[i, i] - sum(R[k, i] ** 2 for k in range(i))
        R[i, i] = math.sqrt(d)
        for j in range(i + 1, n):
            R[i, j] = (S[i, j] - sum(R[k, i] * R[k, j] for k in range(i))) / R[i, i]
    return R


def _mgs(X):
    """Modified Gram-Schmidt: positive-diagonal QR of a full-rank X."""
    X = X.copy()
    m, n = X.shape
    Q = np.zeros((m, n))
    R = np.zeros((n, n))
    for j in range(n):
        R[j, j] = math.sqrt(float(X[:, j] @ X[:, j]))
        Q[:, j] = X[:, j] / R[j, j]
        for k in range(j + 1, n):
            R[j, k] = Q[:, j] @ X[:, k]
            X[:, k] -= R[j, k] * Q[:, j]
    return Q, R


@pytest.mark.parametrize("m,n", [(5, 5), (12, 7), (40, 40), (65, 33)])
def test_qr_matches_cholesky_of_gram(orc, m, n):
    rng = np.random.default_rng(m * n)
    X = rng.standard_normal((m, n)) + 3 * np.eye(m, n)  # modest condition number
    assert np.linalg.cond(X) < 1e4
    _, R = orc.qr_pos(X)
    Rc = _cholesky_upper(X.T @ X)
    np.testing.assert_allclose(R, Rc, rtol=0, atol=1e-12 * np.abs(Rc).max())


@pytest.mark.parametrize("m,n", [(8, 8), (30, 10), (64, 64)])
def test_qr_matches_modified_gram_schmidt(orc, m, n):
    rng = np.random.default_rng(7 + m + n)
    X = rng.standard_normal((m, n))
    Q, R = orc.qr_pos(X)
    Qg, Rg = _mgs(X)
    np.testing.assert_allclose(R, Rg, rtol=0, atol=1e-12 * np.abs(R).max())
    np.testing.assert_allclose(Q, Qg, rtol=0, atol=1e-10)


@pytest.mark.parametrize("m,n", [(1, 1), (3, 1), (9, 9), (70, 31), (128, 128)])
def test_qr_matches_lapack_after_sign_fix(orc, m, n):
    rng = np.random.default_rng(m + 3 * n)
    X = rng.standard_normal((m, n))
    Q, R = orc.qr_pos(X)
    Ql, Rl = np.linalg.qr(X)
    d = np.sign(np.diag(Rl))
    d[d == 0] = 1
    np.testing.assert_allclose(R, d[:, None] * Rl, rtol=0, atol=50 * n * EPS * np.abs(R).max())
    np.testing.assert_allclose(Q, Ql * d, rtol=0, atol=1e-12)
    assert np.all(np.diag(R) >= 0)
    assert np.array_equal(R, np.triu(R))
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) < 10 * n * EPS
    assert np.linalg.norm(Q @ R - X) < 10 * n * EPS * np.linalg.norm(X)


def test_qr_zero_and_repeated_columns(orc):
    """Rank-deficient input: still Q orthonormal, Q R = X, R(j,j) = 0 on a zero column."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((10, 6))
    X[:, 2] = 0.0
    X[:, 4] = X[:, 1]
    Q, R = orc.qr_pos(X)
    assert abs(R[2, 2]) < 1e-15
    assert abs(R[4, 4]) < 1e-13
    assert np.linalg.norm(Q.T @ Q - np.eye(6)) < 1e-13
    assert np.linalg.norm(Q @ R - X) < 1e-13 * np.linalg.norm(X)
    Q0, R0 = orc.qr_pos(np.zeros((4, 3)))
    np.testing.assert_array_equal(Q0, np.eye(4, 3))
    np.testing.assert_array_equal(R0, np.zeros((3, 3)))


def test_qr_power_of_two_scaling_is_bitwise(orc):
    rng = np.random.default_rng(11)
    X = rng.standard_normal((20, 13))
    Q, R = orc.qr_pos(X)
    Q2, R2 = orc.qr_pos(X * 2.0**-7)
    np.testing.assert_array_equal(Q, Q2)
    np.testing.assert_array_equal(R * 2.0**-7, R2)


def test_qr_column_prefix(orc):
    """Column j of Q and R depends only on columns 0..j of X (bitwise)."""
    rng = np.random.default_rng(12)
    X = rng.standard_normal((30, 20))
    Y = X.copy()
    Y[:, 12:] = rng.standard_normal((30, 8))
    Q, R = orc.qr_pos(X)
    Qy, Ry = orc.qr_pos(Y)
    np.testing.assert_array_equal(Q[:, :12], Qy[:, :12])
    np.testing.assert_array_equal(R[:12, :12], Ry[:12, :12])


# ---------------------------------------------------------------- Jacobi SVD
def test_jacobi_diagonal_and_2x2(orc):
    D = np.diag([3.0, -7.0, 0.5, 2.0])
    np.testing.assert_array_equal(orc.jacobi_svd(D), [7.0, 3.0, 2.0, 0.5])
    # [[a, b], [0, d]]: sigma1 sigma2 = |a d|, sigma1^2 + sigma2^2 = a^2 + b^2 + d^2
    a, b, d = 2.0, 3.0, 1.0
    s = orc.jacobi_svd(np.array([[a, b], [0.0, d]]))
    assert s[0] * s[1] == pytest.approx(abs(a * d), rel=1e-15)
    assert s[0] ** 2 + s[1] ** 2 == pytest.approx(a * a + b * b + d * d, rel=1e-15)


@pytest.mark.parametrize("m,n", [(10, 10), (50, 30), (200, 160)])
def test_jacobi_matches_lapack_svd(orc, m, n):
    sigma = gen.spectrum("geometric8", n)
    A = gen.spectral_matrix(m, n, sigma, seed=4)
    s = orc.jacobi_svd(A)
    ref = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(s, ref, rtol=0, atol=20 * n * EPS)
    np.testing.assert_allclose(s, sigma, rtol=0, atol=20 * n * EPS)
