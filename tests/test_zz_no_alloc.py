"""urv_dgemm_noalloc (split-K partial sums in the library's static device buffer)
against urv_dgemm on the same inputs: the same plan, so the results agree bit for
bit.  Two calls in a row, the second smaller, so stale contents of the shared
buffer from the first call would show."""
import numpy as np
import pytest

from gpu_helpers import announce, to_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def urv():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1812_06007_amd import urv as u

    u.lib()
    return u


@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True)])
def test_noalloc_matches_dgemm_twice(urv, ta, tb):
    # split-K shapes (few output tiles, long sums), then a smaller one
    for M, N, K in [(128, 192, 9000), (96, 64, 3000)]:
        announce("dgemm noalloc", ta, tb, M, N, K)
        rng = np.random.default_rng(M + N + K + 7 * ta + 11 * tb)
        A = to_gpu(rng.standard_normal((K, M) if ta else (M, K)))
        B = to_gpu(rng.standard_normal((N, K) if tb else (K, N)))
        C0 = rng.standard_normal((M, N))
        ref = to_np(urv.dgemm(A, B, transA=ta, transB=tb, alpha=1.5, beta=-0.5, C=to_gpu(C0)))
        got = to_np(urv.dgemm(A, B, transA=ta, transB=tb, alpha=1.5, beta=-0.5, C=to_gpu(C0), noalloc=True))
        np.testing.assert_array_equal(got, ref)


def test_noalloc_without_split_k_and_empty(urv):
    announce("dgemm noalloc plain")
    rng = np.random.default_rng(5)
    A = to_gpu(rng.standard_normal((700, 300)))
    B = to_gpu(rng.standard_normal((300, 500)))
    ref = to_np(urv.dgemm(A, B))
    got = to_np(urv.dgemm(A, B, noalloc=True))
    np.testing.assert_array_equal(got, ref)
    # K == 0 scales C by beta
    C = to_gpu(np.ones((4, 3)))
    Z = to_gpu(np.zeros((4, 0)))
    W = to_gpu(np.zeros((0, 3)))
    np.testing.assert_array_equal(to_np(urv.dgemm(Z, W, beta=2.0, C=C, noalloc=True)), 2.0 * np.ones((4, 3)))
