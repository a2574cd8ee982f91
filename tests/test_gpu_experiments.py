"""The accuracy experiments of Section 5 (Matrices 1-3, 200 x 160) through the
GPU path, against the optimal rank-k errors that the prescribed spectra give
in closed form, and against the FP64 oracle.

The paper reports that PowerURV with q = 1 is close to the best rank-k
approximations and that without power iterations (q = 0, DDH-URV) it is a
factor 2-10 worse.  Checked here: the q = 0 errors exceed the optimum by at
least 1.5x at their worst, q = 1 and q = 2 stay within 1.6x and 1.5x, errors
never grow with q, the exact inequalities (Eckart-Young, interlacing) hold, and
the GPU's rank-k error curves equal the oracle's within 1e-11 ||A||_F."""
import numpy as np
import pytest

import urv_inputs as gen
from gpu_helpers import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def results():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1812_06007_amd import experiments

    announce("experiments of Section 5")
    return experiments.run()


def test_power_steps_approach_the_optimal_errors(results):
    for name in ("matrix1", "matrix2", "matrix3"):
        variants = ("full", "none") if name == "matrix2" else ("full",)
        for v in variants:
            r = [results["%s/%s/q%d" % (name, v, q)]["ratio_max"] for q in (0, 1, 2)]
            assert r[0] >= 1.5, (name, v, r)
            assert r[1] <= 1.6 and r[2] <= 1.5, (name, v, r)
            assert r[0] > r[1] >= r[2] * (1 - 1e-9), (name, v, r)


def test_exact_inequalities(results):
    for key, r in results.items():
        ek, opt = np.array(r["ek"]), np.array(r["opt"])
        scale = opt[0]
        assert np.all(ek >= opt - 1e-12 * scale), key                          # Eckart-Young
        assert all(x <= 1 + 1e-10 for x in r["sigma_min_R11_over_sigma_k"].values()), key
        assert all(x >= 1 - 1e-10 for x in r["norm_R22_over_sigma_k1"].values()), key
        assert r["recon"] <= 1e-13, key


def test_rank_revealing_profiles(results):
    """The figure of Section 3 over every k: sigma_min(R11) <= sigma_k and
    sigma_max(R22) >= sigma_{k+1} always (interlacing); with power steps both
    stay close to the singular values (median ratio within 2x), without them
    Matrix 1's are off by about an order of magnitude."""
    for key, r in results.items():
        p11, p22 = np.array(r["profile_R11"]), np.array(r["profile_R22"])
        assert np.all(p11 <= 1 + 1e-10) and np.all(p22 >= 1 - 1e-10), key
        print("[gpu-case]", key, "median profiles", r["profile_R11_median"], r["profile_R22_median"], flush=True)
        if r["q"] >= 1 and r["matrix"] in ("matrix1", "matrix2"):
            assert r["profile_R11_median"] >= 0.5 and r["profile_R22_median"] <= 2.0, key
    m1 = results["matrix1/full/q0"]
    assert m1["profile_R11_median"] <= 0.3 and m1["profile_R22_median"] >= 3.0


def test_curves_equal_the_oracle(results, orc):
    for name in ("matrix1", "matrix2", "matrix3"):
        sigma = gen.spectrum(name, 160)
        A = gen.spectral_matrix(200, 160, sigma, 1812)
        for q in (0, 1, 2):
            U, R, V = orc.urv(A, q, seed=1812)
            ek = orc.metrics(A, U, R, V)["ek"]
            gpu = np.array(results["%s/full/q%d" % (name, q)]["ek"])
            assert np.max(np.abs(gpu - ek)) <= 1e-11 * np.linalg.norm(A), (name, q)


# ------------------------------------------- PowerURV and the RSVD (Matrix 2, l = 60)
@pytest.fixture(scope="module")
def rsvd():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1812_06007_amd import experiments

    announce("RSVD comparison, Matrix 2, l = 60, q = 0 and 1")
    return experiments.rsvd_comparison()


def test_rsvd_lemma_at_l(rsvd):
    """The Lemma of the RSVD section: from the same G, the leading l columns of
    U and U_rsvd span the same space, so the two projections of A agree."""
    for key, r in rsvd.items():
        print("[gpu-case]", key, "projector gap", r["projector_gap_at_l"], "error gap", r["lemma_gap_at_l"], flush=True)
        assert r["projector_gap_at_l"] <= 1e-10, key
        assert r["lemma_gap_at_l"] <= 1e-12, key


def test_rsvd_curves_against_host_computations(rsvd, orc):
    """Both error curves recomputed on the host in FP64 from the same A and G:
    PowerURV through the oracle, the RSVD through numpy's QR and SVD.  Every
    error is at least the optimal rank-k error (Eckart-Young)."""
    m, n, l, seed = 200, 160, 60, 1812
    sigma = gen.spectrum("matrix2", n)
    A = gen.spectral_matrix(m, n, sigma, seed)
    G = orc.gaussian(n, n, seed, stream_id=2)
    na = np.linalg.norm(A)
    for key, r in rsvd.items():
        q = r["q"]
        U, _, V = orc.urv(A, q, G=G)
        Y = G[:, :l]
        for _ in range(q):
            Y = A.T @ (A @ Y)
        Q, _ = np.linalg.qr(A @ Y)
        W, _, _ = np.linalg.svd(Q.T @ A)
        Ur = Q @ W
        ks = range(1, l + 1)
        eu = np.array([np.linalg.norm(A - U[:, :k] @ (U[:, :k].T @ A)) for k in ks])
        er = np.array([np.linalg.norm(A - Ur[:, :k] @ (Ur[:, :k].T @ A)) for k in ks])
        assert np.max(np.abs(eu - r["powerurv_left"])) <= 1e-10 * na, key
        assert np.max(np.abs(er - r["rsvd_left"])) <= 1e-8 * na, key
        opt = np.array(r["opt"])
        for curve in ("powerurv_left", "rsvd_left", "powerurv_right", "rsvd_right"):
            assert np.all(np.array(r[curve]) >= opt * (1 - 1e-12)), (key, curve)


def test_rsvd_leading_columns_are_closer_to_optimal(rsvd):
    """The section's observation: with one more application of A, the RSVD's
    leading columns (left and right) give smaller errors than PowerURV's for
    k < l; the curves meet at k = l."""
    for key, r in rsvd.items():
        print("[gpu-case]", key, "median RSVD/PowerURV left", r["left_ratio_median_k_lt_l"],
              "right", r["right_ratio_median_k_lt_l"], flush=True)
        assert r["left_ratio_median_k_lt_l"] < 1.0, key
        assert r["right_ratio_median_k_lt_l"] < 1.0, key
