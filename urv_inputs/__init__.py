"""Seeded synthetic inputs for PowerURV tests and benchmarks.

This module only *draws* inputs: test matrices with prescribed singular
values, Kahan's matrix and Gaussian starting matrices.  It holds none of the
factorisation's arithmetic and is shared by the oracle-side and GPU-side
tests so that both see the same bytes.

Every random draw comes from ``numpy.random.Generator(Philox(key=[seed,
stream]))``; the stream ids are fixed: 0 = left Haar factor, 1 = right Haar
factor, 2 = starting matrix G, 3 = additive noise, 4 and 5 = left and right
factors of a rank spike.
Haar factors are Q-factors of Gaussian matrices with the sign of the
diagonal of R fixed positive, which makes them exactly Haar distributed
(footnote to Section 2.2 of the paper).

Large matrices (n in the thousands) can be drawn on a GPU with torch
(``device="cuda"``): the construction is the same, the random stream is
torch's own, so those bytes differ from the numpy ones.  They are used only
where a test checks size-independent properties.
"""
from __future__ import annotations

import math

import numpy as np

STREAM_LEFT, STREAM_RIGHT, STREAM_G, STREAM_NOISE, STREAM_SPIKE = 0, 1, 2, 3, 4
STREAM_SPIKE_RIGHT = 5


def generator(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=np.array([int(seed), int(stream)], dtype=np.uint64)))


# --------------------------------------------------------------------------
# Spectra sigma_j, j = 1..n
def spectrum(kind: str, n: int) -> np.ndarray:
    """Singular values used by the workloads.

    geometric8 : 10^(-8 (j-1)/(n-1))        (400 x 400 parity case)
    poly2      : 1/j^2                       (8000 x 8000 case)
    exp800     : exp(-j/800)                 (mixed-precision case)
    geometric6 : 10^(-6 (j-1)/(n-1))        (batched case)
    matrix1    : 10^(-20 (j-1)/(n-1))       (paper's Matrix 1, rescaled: the
                 printed (10^-20)^(k-1) underflows after a few entries)
    matrix2    : 1/j                         (paper's Matrix 2)
    matrix3    : 10^-(1 + tanh(5(-1 + 2j/80))) for j <= 80, 10^-2 after
                 (paper's Matrix 3, read with 80 in the tanh)
    """
    j = np.arange(1, n + 1, dtype=np.float64)
    d = max(n - 1, 1)
    if kind == "geometric8":
        return 10.0 ** (-8.0 * (j - 1) / d)
    if kind == "geometric6":
        return 10.0 ** (-6.0 * (j - 1) / d)
    if kind == "poly2":
        return 1.0 / (j * j)
    if kind == "exp800":
        return np.exp(-j / 800.0)
    if kind == "matrix1":
        return 10.0 ** (-20.0 * (j - 1) / d)
    if kind == "matrix2":
        return 1.0 / j
    if kind == "matrix3":
        s = np.full(n, 1e-2)
        k = j[j <= 80]
        s[: k.size] = 10.0 ** (-(1.0 + np.tanh(5.0 * (-1.0 + 2.0 * k / 80.0))))
        return s
    raise ValueError(kind)


# --------------------------------------------------------------------------
def haar_columns(m: int, n: int, rng: np.random.Generator) -> np.ndarray:
    """m x n with Haar-distributed orthonormal columns (QR of a Gaussian)."""
    X = rng.standard_normal((m, n))
    Q, R = np.linalg.qr(X)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return np.asfortranarray(Q * d)


def spectral_matrix(m: int, n: int, sigma: np.ndarray, seed: int, device=None):
    """A = Q1 diag(sigma) Q2^T with Q1 m x n and Q2 n x n Haar.

    numpy float64 (Fortran order) by default; a torch float64 tensor on
    ``device`` when one is given (column-major storage, see ``to_colmajor``).
    """
    sigma = np.asarray(sigma, dtype=np.float64)
    assert sigma.shape == (n,) and m >= n
    if device is None:
        Q1 = haar_columns(m, n, generator(seed, STREAM_LEFT))
        Q2 = haar_columns(n, n, generator(seed, STREAM_RIGHT))
        return np.asfortranarray((Q1 * sigma) @ Q2.T)
    import torch

    def haar_t(rows, cols, stream):
        g = torch.Generator(device=device)
        g.manual_seed(int(seed) * 16 + stream)
        X = torch.randn(rows, cols, dtype=torch.float64, device=device, generator=g)
        Q, R = torch.linalg.qr(X)
        d = torch.sign(torch.diagonal(R))
        d[d == 0] = 1.0
        return Q * d

    Q1 = haar_t(m, n, STREAM_LEFT)
    Q2 = haar_t(n, n, STREAM_RIGHT)
    s = torch.as_tensor(sigma, dtype=torch.float64, device=device)
    A = (Q1 * s) @ Q2.T
    del Q1, Q2
    return to_colmajor(A)


def to_colmajor(A):
    """Column-major copy of a 2-D torch tensor (stride (1, rows))."""
    return A.t().contiguous().t()


def kahan(n: int, c: float = 0.285) -> np.ndarray:
    """Kahan's matrix: K(i,i) = s^i, K(i,j) = -c s^i for j > i (0-based i),
    s = sqrt(1 - c^2).  Every column has unit 2-norm."""
    s = math.sqrt(1.0 - c * c)
    powers = s ** np.arange(n, dtype=np.float64)
    K = np.triu(np.full((n, n), -c), 1) + np.eye(n)
    return np.asfortranarray(K * powers[:, None])


def gaussian(rows: int, cols: int, seed: int, stream: int = STREAM_G) -> np.ndarray:
    """i.i.d. N(0,1) matrix, Fortran order."""
    return np.asfortranarray(generator(seed, stream).standard_normal((rows, cols)))


def noisy_spectral_matrix(m: int, n: int, sigma: np.ndarray, seed: int, noise_var: float, device=None):
    """Q1 diag(sigma) Q2^T + E with E i.i.d. N(0, noise_var) (variance)."""
    A = spectral_matrix(m, n, sigma, seed, device=device)
    std = math.sqrt(noise_var)
    if device is None:
        return np.asfortranarray(A + std * generator(seed, STREAM_NOISE).standard_normal((m, n)))
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 16 + STREAM_NOISE)
    A += std * torch.randn(A.shape[1], A.shape[0], dtype=torch.float64, device=device, generator=g).t()
    return A


def sigma_sums(sigma: np.ndarray) -> dict:
    """Closed forms of a matrix with singular values sigma (used by tests):
    Frobenius norm, log10 |det|, tail norms sqrt(sum_{j>k} sigma_j^2)."""
    s = np.sort(np.asarray(sigma, dtype=np.float64))[::-1]
    tail = np.sqrt(np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]]))
    return {"fro": float(np.sqrt(np.sum(s * s))), "log10det": float(np.sum(np.log10(s))), "tail": tail}


def spiked_gaussian(m: int, n: int, rank: int, scale: float, seed: int) -> np.ndarray:
    """i.i.d. N(0, 1/n) noise (stream 3) plus scale * P Q^T with P (m x rank)
    and Q (n x rank) Haar columns (streams 4 and 5): a rank-`rank` spike of
    singular value `scale` over a Gaussian bulk of spectral radius about 2
    (the differentiation workload)."""
    E = generator(seed, STREAM_NOISE).standard_normal((m, n)) / math.sqrt(n)
    P = haar_columns(m, rank, generator(seed, STREAM_SPIKE))
    Q = haar_columns(n, rank, generator(seed, STREAM_SPIKE_RIGHT))
    return np.asfortranarray(E + scale * (P @ Q.T))
