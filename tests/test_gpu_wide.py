"""m < n (Section 1: a URV of A from a ULV of A^T, transposed) through the C ABI,
against the FP64 oracle: every rank-k error e_k within 1e-11 ||A||_F, the
invariants (reconstruction, orthonormal columns of U and V), the shapes
U m x m, R m x m, V n x m, and the rank-k errors against the optimum.

R itself is compared entrywise (1e-11 ||A||_F) on mildly conditioned inputs
only: with the columns reversed, the first reflector is built from the
weakest direction B v_p, which two correct computations agree on only to
eps sigma_1 / sigma_p, and that error reaches R's last column multiplied by
the strong columns' norms (about 1e-8 ||A|| for a spread of 1e8).  The
rank-k errors do not inherit it: e_k = ||B V(:, k:)||_F depends on the
leading subspace only.  The 1e-11 bound is the FULL variant's; HALF squares
the condition of each iterate and NONE skips the re-orthonormalisations, so
their V (and the e_k over its trailing directions) are determined less
tightly: 1e-8 and 1e-9 ||A||_F here, as for the tall problem's spread."""
import numpy as np
import pytest

import urv_inputs as gen
from gpu_helpers import announce, to_gpu, to_np

pytestmark = pytest.mark.gpu
TOL = 1e-11
VTOL = {"full": 1e-11, "half": 1e-8, "none": 1e-9}


@pytest.fixture(scope="module")
def urv():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1812_06007_amd import urv as u

    u.lib()
    return u


def _wide(m, n, kind, seed):
    """A = Q1 diag(sigma) Q2^T with Q1 m x m and Q2 n x m Haar: the transpose
    of the tall construction."""
    return np.asfortranarray(gen.spectral_matrix(n, m, gen.spectrum(kind, m), seed).T)


CASES = [(150, 260, 2, "full"), (200, 201, 1, "half"), (64, 500, 0, "full"), (1, 70, 1, "full"),
         (130, 300, 2, "none"), (257, 400, 2, "full")]


def _mild(m, n, seed):
    sigma = 10.0 ** (-2.0 * np.arange(m) / max(m - 1, 1))
    return np.asfortranarray(gen.spectral_matrix(n, m, sigma, seed).T)


@pytest.mark.parametrize("spectrum", ["mild", "graded"])
@pytest.mark.parametrize("m,n,q,variant", CASES)
def test_wide_matches_oracle(urv, orc, m, n, q, variant, spectrum):
    announce("wide", m, n, q, variant, spectrum)
    if spectrum == "mild":
        A = _mild(m, n, m + n)
    else:
        A = _wide(m, n, "geometric8" if variant != "none" else "matrix2", m + n)
    U, R, V = (to_np(t) for t in urv.factor(to_gpu(A), q, seed=1812, variant=variant))
    assert U.shape == (m, m) and R.shape == (m, m) and V.shape == (n, m)
    Uo, Ro, Vo = orc.urv(A, q, seed=1812, variant=variant)
    na = np.linalg.norm(A)
    met = urv.metrics(to_gpu(A), to_gpu(U), to_gpu(R), to_gpu(V))
    mo = orc.metrics(A, Uo, Ro, Vo)
    if spectrum == "mild":
        assert np.linalg.norm(R - Ro) <= VTOL[variant] * na
    assert np.max(np.abs(met["ek"] - mo["ek"])) <= VTOL[variant] * na
    assert met["recon"] <= 1e-13 and met["orthU"] <= 1e-12 and met["orthV"] <= 1e-12
    assert np.array_equal(R, np.triu(R)) and np.all(np.diag(R) >= 0)


def test_wide_given_g_and_mixed(urv, orc):
    m, n = 180, 320
    announce("wide given G, mixed")
    A = _mild(m, n, 3)
    G = gen.gaussian(m, m, 4)
    U, R, V = (to_np(t) for t in urv.factor(to_gpu(A), 2, G=to_gpu(G)))
    Uo, Ro, Vo = orc.urv(A, 2, G=G)
    assert np.linalg.norm(R - Ro) <= TOL * np.linalg.norm(A)
    # the mixed form keeps the FP64 tail: FP64-level invariants
    U, R, V = urv.factor(to_gpu(A), 2, seed=5, precision="mixed_bf16")
    met = urv.metrics(to_gpu(A), U, R, V)
    assert met["recon"] <= 1e-13 and met["orthU"] <= 1e-12 and met["orthV"] <= 1e-12


def test_wide_rank_revealing(urv):
    m, n = 160, 240
    announce("wide rank revealing")
    sigma = gen.spectrum("geometric8", m)
    A = _wide(m, n, "geometric8", 9)
    U, R, V = urv.factor(to_gpu(A), 2, seed=1812)
    ek = urv.metrics(to_gpu(A), U, R, V)["ek"]
    opt = np.sqrt(np.concatenate([np.cumsum((sigma ** 2)[::-1])[::-1], [0.0]]))
    keep = opt[1:m] > 1e-13 * np.linalg.norm(A)
    ratio = ek[1:m][keep] / opt[1:m][keep]
    assert np.all(ratio >= 1 - 1e-9) and np.max(ratio) < 2.0
