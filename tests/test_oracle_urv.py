"""Pins of the oracle's PowerURV driver (Section 3, eqs. power and powerqr).

What fixes the result without any other implementation:
  * reductions: q = 0 is DDH-URV (Section 2.2) and with G = I it is plain QR of A;
  * the Lemma of Section 6: span U(:,1:l) = span A (A^T A)^q G(:,1:l);
  * closed forms of the prescribed spectrum: ||R||_F = ||A||_F, |det R| = prod sigma,
    interlacing of the leading products, Eckart-Young lower bounds (Section 1);
  * |R(j,j)| approaches sigma_j as q grows (Section 3, Figure 3 discussion);
  * invariants A = U R V^T, U^T U = I, V^T V = I;
  * metamorphic relations: power-of-two scaling, orthogonal equivariance,
    column-prefix consistency.
"""
import math

import numpy as np
import pytest

import urv_inputs as gen

EPS = np.finfo(np.float64).eps


def _case(m, n, kind, seed=1812):
    sigma = gen.spectrum(kind, n)
    return gen.spectral_matrix(m, n, sigma, seed), sigma


# --------------------------------------------------------------- reductions
@pytest.mark.parametrize("variant", ["full", "half", "none"])
def test_q0_with_identity_start_is_plain_qr(orc, variant):
    # mild spectrum: U's trailing columns are then determined to ~eps (they are not for a graded A)
    A = gen.spectral_matrix(40, 30, np.linspace(1.0, 0.1, 30), seed=1812)
    U, R, V = orc.urv(A, 0, G=np.eye(30), variant=variant)
    np.testing.assert_array_equal(V, np.eye(30))
    Ql, Rl = np.linalg.qr(A)
    d = np.sign(np.diag(Rl))
    np.testing.assert_allclose(R, d[:, None] * Rl, rtol=0, atol=1e-13 * np.abs(Rl).max())
    np.testing.assert_allclose(U, Ql * d, rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [10, 60, 200])
def test_kahan_q0_identity_start_is_exact(orc, n):
    """Kahan's matrix is upper triangular with positive diagonal: U = I, R = K, V = I bitwise."""
    K = gen.kahan(n)
    U, R, V = orc.urv(K, 0, G=np.eye(n))
    np.testing.assert_array_equal(U, np.eye(n))
    np.testing.assert_array_equal(R, K)
    np.testing.assert_array_equal(V, np.eye(n))


def test_q0_is_ddh_urv(orc):
    """q = 0: V = Qpos(G) (a Haar matrix), and A V = U R."""
    A, _ = _case(50, 35, "matrix2")
    G = gen.gaussian(35, 35, 9)
    U, R, V = orc.urv(A, 0, G=G)
    Ql, Rl = np.linalg.qr(G)
    d = np.sign(np.diag(Rl))
    np.testing.assert_allclose(V, Ql * d, rtol=0, atol=1e-12)
    np.testing.assert_allclose(U @ R, A @ V, rtol=0, atol=1e-14 * np.linalg.norm(A))


def test_seeded_start_uses_stream_2(orc):
    A, _ = _case(24, 16, "geometric8")
    G = orc.gaussian(16, 16, 77, stream_id=2)
    for q in (0, 2):
        a = orc.urv(A, q, seed=77)
        b = orc.urv(A, q, G=G)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


# --------------------------------------------------------------- the Lemma
@pytest.mark.parametrize("q", [0, 1, 2])
@pytest.mark.parametrize("variant", ["full", "half"])
def test_lemma_range_of_leading_columns(orc, q, variant):
    """Section 6 Lemma: U(:,1:l) spans A (A^T A)^q G(:,1:l) (numpy QR of that product)."""
    m, n, l = 120, 80, 30
    sigma = np.linspace(1.0, 0.2, n)  # well conditioned: the product is computed stably in numpy
    A = gen.spectral_matrix(m, n, sigma, seed=3)
    G = gen.gaussian(n, n, 4)
    U, R, V = orc.urv(A, q, G=G, variant=variant)
    Y = G[:, :l]
    for _ in range(q):
        Y = A.T @ (A @ Y)
    Ql, _ = np.linalg.qr(A @ Y)
    P1 = U[:, :l] @ U[:, :l].T
    P2 = Ql @ Ql.T
    assert np.linalg.norm(P1 - P2, 2) < 1e-10


# --------------------------------------------------------------- closed forms
@pytest.mark.parametrize("q", [0, 1, 2])
def test_closed_forms_of_the_spectrum(orc, q):
    n = 150
    A, sigma = _case(n, n, "geometric8")
    U, R, V = orc.urv(A, q, seed=1812)
    sums = gen.sigma_sums(sigma)
    # ||R||_F = ||A||_F = sqrt(sum sigma^2)
    assert np.linalg.norm(R) == pytest.approx(sums["fro"], rel=1e-13)
    # |det R| = |det A| = prod sigma
    logdet = np.sum(np.log10(np.abs(np.diag(R))))
    assert logdet == pytest.approx(sums["log10det"], abs=1e-8 * n)
    # interlacing: prod_{j<=k} |R_jj| <= prod_{j<=k} sigma_j, since R11 = U1^T A V1 is a
    # compression of A.  Slack: R_jj carries relative error ~eps sigma_1 / sigma_j.
    lead = np.cumsum(np.log10(np.abs(np.diag(R))))
    slack = np.cumsum(EPS / sigma) * 10
    assert np.all(lead <= np.cumsum(np.log10(sigma)) + slack)
    # Eckart-Young: ||R22||_F >= optimal rank-k error sqrt(sum_{j>k} sigma_j^2)
    met = orc.metrics(A, U, R, V)
    assert np.all(met["ek"] >= sums["tail"] * (1 - 1e-10) - 1e-14 * sums["fro"])


def test_spectral_inequalities_small(orc):
    """sigma_min(R11) <= sigma_k(A) and ||R22||_2 >= sigma_{k+1}(A) (Section 1, eq. blocks)."""
    n = 40
    A, sigma = _case(60, n, "matrix2", seed=5)
    U, R, V = orc.urv(A, 1, seed=5)
    s = orc.jacobi_svd(A)
    for k in range(1, n):
        s11 = np.linalg.svd(R[:k, :k], compute_uv=False)[-1]
        s22 = np.linalg.svd(R[k:, k:], compute_uv=False)[0]
        assert s11 <= s[k - 1] * (1 + 1e-12)
        assert s22 >= s[k] * (1 - 1e-12)


def test_diag_r_approaches_singular_values(orc):
    """median_j |log10(|R_jj| / sigma_j)| does not grow from q = 0 to 1 to 2 (Section 3)."""
    n = 120
    ok = 0
    for seed in range(1812, 1822):
        A, _ = _case(n, n, "matrix2", seed=seed)
        s = orc.jacobi_svd(A)
        devs = []
        for q in (0, 1, 2):
            _, R, _ = orc.urv(A, q, seed=seed)
            devs.append(np.median(np.abs(np.log10(np.abs(np.diag(R)) / s))))
        ok += devs[0] >= devs[1] >= devs[2]
        assert devs[2] < devs[0]
    assert ok >= 9


def test_kahan_rank_revealing_with_power_steps(orc):
    """Kahan's matrix defeats plain QR (R_nn >> sigma_n) but not PowerURV with q >= 1."""
    n = 60
    K = gen.kahan(n)
    s = orc.jacobi_svd(K)
    assert K[-1, -1] / s[-1] > 1e5
    for q in (1, 2):
        _, R, _ = orc.urv(K, q, seed=1812)
        assert 0.5 < abs(R[-1, -1]) / s[-1] < 2.0


# --------------------------------------------------------------- invariants
@pytest.mark.parametrize("m,n", [(1, 1), (2, 1), (7, 7), (33, 17), (65, 64), (128, 127)])
@pytest.mark.parametrize("variant", ["full", "half", "none"])
@pytest.mark.parametrize("q", [0, 1, 2])
def test_invariants(orc, m, n, variant, q):
    sigma = np.linspace(1.0, 1e-3, n) if variant == "none" else gen.spectrum("geometric8", n)
    A = gen.spectral_matrix(m, n, sigma, seed=m * 1000 + n)
    U, R, V = orc.urv(A, q, seed=11, variant=variant)
    met = orc.metrics(A, U, R, V)
    tol = 10 * max(n, 2) * EPS
    assert met["recon"] < tol
    assert met["orthU"] < tol
    assert met["orthV"] < tol
    assert np.array_equal(R, np.triu(R))
    assert np.all(np.diag(R) >= 0)
    assert met["ek"][0] == pytest.approx(np.linalg.norm(R), rel=1e-14)
    # e_k = ||A - U(:,1:k) R(1:k,:) V^T||_F, the rank-k error of Section 5
    for k in {0, n // 2, n - 1}:
        Ak = U[:, :k] @ R[:k, :] @ V.T
        assert met["ek"][k] == pytest.approx(np.linalg.norm(A - Ak), rel=1e-6, abs=1e-13)


def test_metrics_closed_forms(orc):
    """orc_metrics against quantities fixed without it: U = [I; 0] D with D a diagonal of small
    integers, V a permutation that is not its own inverse, R diagonal and an integer residual E
    in A = U R V^T + E.  Then ||A - U R V^T||_F / ||A||_F = ||E||_F / ||A||_F,
    ||U^T U - I||_F = sqrt(sum (d^2 - 1)^2), ||V^T V - I||_F = 0, and e_k is the tail norm of
    diag(R); every sum is of integers, so only the final square roots round."""
    m, n = 50, 20
    rng = np.random.default_rng(5)
    d = rng.integers(1, 4, size=n).astype(np.float64)
    U = np.zeros((m, n))
    U[:n, :n] = np.diag(d)
    perm = np.roll(np.arange(n), 3)  # a cycle: V != V^T
    V = np.eye(n)[:, perm]
    r = rng.integers(1, 9, size=n).astype(np.float64)
    R = np.diag(r)
    E = rng.integers(-2, 3, size=(m, n)).astype(np.float64)
    A = np.asfortranarray(U @ R @ V.T + E)
    met = orc.metrics(A, U, R, V)
    assert met["normA"] == np.sqrt(np.sum(A * A))
    assert met["recon"] == pytest.approx(np.sqrt(np.sum(E * E)) / np.sqrt(np.sum(A * A)), rel=1e-15)
    assert met["orthU"] == pytest.approx(np.sqrt(np.sum((d * d - 1) ** 2)), rel=1e-15)
    assert met["orthV"] == 0.0
    tail = np.sqrt(np.cumsum((r * r)[::-1])[::-1])
    np.testing.assert_allclose(met["ek"][:n], tail, rtol=1e-15)
    assert met["ek"][n] == 0.0


def test_metrics_wide_closed_forms(orc):
    """The same closed forms for m < n (U m x m, V n x m)."""
    m, n = 12, 30
    rng = np.random.default_rng(6)
    d = rng.integers(1, 4, size=m).astype(np.float64)
    U = np.diag(d)
    V = np.zeros((n, m))
    V[np.arange(m) + 5, np.arange(m)] = 1.0
    R = np.triu(rng.integers(-3, 4, size=(m, m)).astype(np.float64))
    E = rng.integers(-2, 3, size=(m, n)).astype(np.float64)
    A = np.asfortranarray(U @ R @ V.T + E)
    met = orc.metrics(A, U, R, V)
    assert met["recon"] == pytest.approx(np.sqrt(np.sum(E * E)) / np.sqrt(np.sum(A * A)), rel=1e-15)
    assert met["orthU"] == pytest.approx(np.sqrt(np.sum((d * d - 1) ** 2)), rel=1e-15)
    assert met["orthV"] == 0.0


def test_empty_and_bad_arguments(orc):
    with pytest.raises(ValueError):
        orc.urv(np.zeros((5, 3)), -1)


# --------------------------------------------------------------- metamorphic
@pytest.mark.parametrize("variant", ["full", "half", "none"])
def test_power_of_two_scaling_bitwise(orc, variant):
    A, _ = _case(30, 20, "geometric8")
    U, R, V = orc.urv(A, 2, seed=3, variant=variant)
    U2, R2, V2 = orc.urv(A * 2.0**5, 2, seed=3, variant=variant)
    np.testing.assert_array_equal(U, U2)
    np.testing.assert_array_equal(V, V2)
    np.testing.assert_array_equal(R * 2.0**5, R2)


def test_orthogonal_equivariance(orc):
    """A -> P A Q with G -> Q^T G gives U -> P U, V -> Q^T V, R unchanged."""
    m, n = 50, 40
    A, _ = _case(m, n, "matrix2", seed=8)
    G = gen.gaussian(n, n, 8)
    P = gen.haar_columns(m, m, gen.generator(99, 0))
    Q = gen.haar_columns(n, n, gen.generator(99, 1))
    U, R, V = orc.urv(A, 1, G=G)
    U2, R2, V2 = orc.urv(P @ A @ Q, 1, G=Q.T @ G)
    np.testing.assert_allclose(R2, R, rtol=0, atol=1e-12)
    np.testing.assert_allclose(U2[:, :10], (P @ U)[:, :10], rtol=0, atol=1e-10)
    np.testing.assert_allclose(V2[:, :10], (Q.T @ V)[:, :10], rtol=0, atol=1e-10)


@pytest.mark.parametrize("variant", ["full", "half"])
def test_column_prefix_consistency(orc, variant):
    """U(:,1:l), R(1:l,1:l), V(:,1:l) depend on G(:,1:l) only (bitwise)."""
    A, _ = _case(45, 32, "geometric8")
    G = gen.gaussian(32, 32, 1)
    G2 = G.copy()
    G2[:, 20:] = gen.gaussian(32, 12, 2)
    U, R, V = orc.urv(A, 2, G=G, variant=variant)
    U2, R2, V2 = orc.urv(A, 2, G=G2, variant=variant)
    np.testing.assert_array_equal(U[:, :20], U2[:, :20])
    np.testing.assert_array_equal(R[:20, :20], R2[:20, :20])
    np.testing.assert_array_equal(V[:, :20], V2[:, :20])


def test_variants_agree_where_stable(orc):
    """FULL, HALF and NONE are equal in exact arithmetic; with a mild spectrum they agree."""
    A = gen.spectral_matrix(60, 40, np.linspace(1.0, 0.1, 40), seed=6)
    outs = [orc.urv(A, 2, seed=6, variant=v) for v in ("full", "half", "none")]
    for U, R, V in outs[1:]:
        np.testing.assert_allclose(R, outs[0][1], rtol=0, atol=1e-11)
        np.testing.assert_allclose(V, outs[0][2], rtol=0, atol=1e-9)


def test_half_rounding_spread_exceeds_full(orc):
    """Re-orthonormalising after every product keeps R within rounding of itself;
    one QR per A^T A step loses directions below sqrt(eps) sigma_1 (Section 3)."""
    n = 200
    A, _ = _case(n, n, "geometric8")
    spread = {}
    for v in ("full", "half"):
        _, R1, _ = orc.urv(A, 2, seed=1, variant=v)
        with orc.sum_order(descending=True):
            _, R2, _ = orc.urv(A, 2, seed=1, variant=v)
        spread[v] = np.linalg.norm(R1 - R2) / np.linalg.norm(A)
    assert spread["full"] < 1e-13
    assert spread["half"] > 10 * spread["full"]


# --------------------------------------------------------------- m < n (Section 1: a ULV of A^T, transposed)
WIDE = [(20, 35, 0), (20, 35, 2), (34, 35, 1), (1, 10, 1), (12, 40, 2)]


@pytest.mark.parametrize("m,n,q", WIDE)
@pytest.mark.parametrize("variant", ["full", "half"])
def test_wide_invariants_and_closed_forms(orc, m, n, q, variant):
    rng = np.random.default_rng(m * 100 + n + q)
    sigma = 10.0 ** (-3.0 * np.arange(m) / max(m - 1, 1))
    Q1, _ = np.linalg.qr(rng.standard_normal((m, m)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, m)))
    A = (Q1 * sigma) @ Q2.T
    U, R, V = orc.urv(A, q, seed=7, variant=variant)
    assert U.shape == (m, m) and R.shape == (m, m) and V.shape == (n, m)
    met = orc.metrics(A, U, R, V)
    assert met["recon"] < 1e-13 and met["orthU"] < 1e-13 and met["orthV"] < 1e-13
    assert np.array_equal(R, np.triu(R)) and np.all(np.diag(R) >= 0)
    assert met["ek"][0] == pytest.approx(np.linalg.norm(A), rel=1e-13)        # ||R||_F = ||A||_F
    assert np.sum(np.log(np.abs(np.diag(R)))) == pytest.approx(np.sum(np.log(sigma)), abs=1e-9 * m)


@pytest.mark.parametrize("m,n", [(24, 40), (30, 31)])
def test_wide_equals_the_tall_problem_of_the_transpose(orc, m, n):
    """U of the wide factorisation is V of the tall factorisation of B = A^T
    (the same power steps), and its rank-k errors are ||B V(:, k:)||_F: the
    leading block of R' over the reversed columns is the QR of B V(:, k:)."""
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n)) * (0.7 ** np.arange(n))
    U, R, V = orc.urv(A, 2, seed=11)
    Ut, Rt, Vt = orc.urv(A.T.copy(), 2, seed=11)
    assert np.array_equal(U, Vt)
    ek = orc.metrics(A, U, R, V)["ek"]
    BV = A.T @ Vt
    ref = np.array([np.linalg.norm(BV[:, k:]) for k in range(m + 1)])
    assert np.max(np.abs(ek - ref)) <= 1e-13 * np.linalg.norm(A)


def test_wide_reveals_rank(orc):
    """Decay 10^-8 over 40 values, q = 2: the rank-k errors stay within 2x of
    the optimum (Eckart-Young); they are ||B V(:, k:)||_F, which the tall
    problem's ||R22||_F does not exceed, so the bound is looser than there.
    Without the column reversal the ratio would be orders of magnitude."""
    m, n = 40, 64
    rng = np.random.default_rng(5)
    sigma = 10.0 ** (-8.0 * np.arange(m) / (m - 1))
    Q1, _ = np.linalg.qr(rng.standard_normal((m, m)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, m)))
    A = (Q1 * sigma) @ Q2.T
    U, R, V = orc.urv(A, 2, seed=3)
    ek = orc.metrics(A, U, R, V)["ek"]
    opt = np.sqrt(np.concatenate([np.cumsum((sigma ** 2)[::-1])[::-1], [0.0]]))
    keep = opt[1:m] > 1e-12
    ratio = ek[1:m][keep] / opt[1:m][keep]
    assert np.all(ratio >= 1 - 1e-9) and np.max(ratio) < 2.0
