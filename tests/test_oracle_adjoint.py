"""Pins of the FP64 adjoint oracle (oracle/adjoint.py) against facts outside it.

- central finite differences of the QR factors and of the whole chain
  (Section 3, eqs. power and powerqr, G fixed), entry by entry on tiny inputs;
- an independent implementation: torch.autograd through torch.linalg.qr
  (LAPACK's QR and PyTorch's own QR backward) with the same sign fix;
- the triangular solve against scipy's;
- special cases: k = n makes A_k = A (A = U R V^T), so the loss and its
  gradient vanish; with a wide spectral gap U(:,1:k) is the dominant
  subspace, where the rank-k error is stationary (Eckart-Young), so the
  gradient is 2 (A - A_k);
- the forward pass equals the oracle's factorisation bit for bit;
- planted mistakes in the adjoint (a dropped term, the wrong triangle, a
  transposed solve, a missing product term) each fail a finite-difference pin.

The truncation loss depends, in exact arithmetic, only on spans of leading
columns, so the within-span terms of the QR adjoints cancel in it; a linear
loss reading every entry of U, R and V is therefore pinned as well.
"""
import numpy as np
import pytest
import scipy.linalg
import torch

from oracle import adjoint, oracle


def _rng(seed):
    return np.random.default_rng(seed)


def _spectrum_matrix(m, n, sigma, seed):
    r = _rng(seed)
    Q1, _ = np.linalg.qr(r.standard_normal((m, n)))
    Q2, _ = np.linalg.qr(r.standard_normal((n, n)))
    return (Q1 * sigma) @ Q2.T


def _fd_grad(f, A, h):
    g = np.zeros_like(A)
    for i in range(A.shape[0]):
        for j in range(A.shape[1]):
            E = np.zeros_like(A)
            E[i, j] = h
            g[i, j] = (f(A + E) - f(A - E)) / (2 * h)
    return g


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_copyltu_small():
    M = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0], [7.0, 8.0, 9.0]])
    S = adjoint.copyltu(M)
    assert np.array_equal(S, np.array([[1.0, 4.0, 7.0], [4.0, 5.0, 8.0], [7.0, 8.0, 9.0]]))


@pytest.mark.parametrize("m,n", [(9, 6), (7, 7), (40, 25)])
def test_solve_rt_against_scipy(m, n):
    r = _rng(m * 100 + n)
    R = np.triu(r.standard_normal((n, n))) + 3 * np.eye(n)
    B = r.standard_normal((m, n))
    X = adjoint.solve_rt(B, R)
    ref = scipy.linalg.solve_triangular(R, B.T, lower=False).T
    assert np.abs(X - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(X @ R.T - B).max() <= 1e-12 * np.abs(B).max()


@pytest.mark.parametrize("m,n", [(7, 5), (6, 6), (9, 3)])
def test_qr_adjoint_finite_differences(m, n):
    r = _rng(m * 10 + n)
    X = r.standard_normal((m, n))
    Cq = r.standard_normal((m, n))
    Cr = r.standard_normal((n, n))

    def f(Z):
        Q, R = oracle.qr_pos(Z)
        return float(np.sum(Cq * Q) + np.sum(Cr * R))

    Q, R = oracle.qr_pos(X)
    g = adjoint.qr_adjoint(Q, R, Cq, Cr)
    assert _rel(g, _fd_grad(f, X, 1e-6)) < 1e-7



@pytest.mark.parametrize("n", [1, 6, 40])
def test_qr_adjoint_square_last_column(n):
    # Q of a square X does not depend on X's last column (it completes the
    # others to an orthonormal basis) and R's last column is Q^T x_n, so the
    # last column of the adjoint is Q Rb(:, n): (I - Q Q^T) Qb(:, n) = 0.
    r = _rng(900 + n)
    X = r.standard_normal((n, n))
    Cq = r.standard_normal((n, n))
    Cr = r.standard_normal((n, n))
    Q, R = oracle.qr_pos(X)
    g = adjoint.qr_adjoint(Q, R, Cq, Cr)
    assert np.abs(g[:, -1] - Q @ np.triu(Cr)[:, -1]).max() <= 1e-12 * np.abs(g).max()
    g0 = adjoint.qr_adjoint(Q, R, Cq, None)
    assert np.abs(g0[:, -1]).max() <= 1e-12 * np.abs(g0).max()

def _chain_fd_error(m, n, q, k, variant, seed):
    r = _rng(seed)
    A = r.standard_normal((m, n))
    G = r.standard_normal((n, n))
    _, g = adjoint.loss_and_grad(A, G, q, k, variant)
    fd = _fd_grad(lambda Z: adjoint.loss_only(Z, G, q, k, variant), A, 1e-6)
    return _rel(g, fd)


@pytest.mark.parametrize("q", [0, 1, 2])
@pytest.mark.parametrize("variant", ["full", "half"])
def test_chain_finite_differences(q, variant):
    assert _chain_fd_error(9, 7, q, 3, variant, 11 + q) < 1e-6


def test_chain_finite_differences_square_k1():
    assert _chain_fd_error(6, 6, 2, 1, "full", 5) < 1e-6


def _linear_fd_error(m, n, q, variant, seed):
    """A loss that reads every entry of U, R and V: <Cu,U> + <Cr,R> + <Cv,V>.

    The truncation loss depends, in exact arithmetic, only on the spans of
    leading columns, which hides the within-span terms of the QR adjoints;
    this one does not."""
    r = _rng(seed)
    A = r.standard_normal((m, n))
    G = r.standard_normal((n, n))
    # Cr is full: R's strictly lower entries are constant zeros and must get no weight
    Cu, Cr, Cv = r.standard_normal((m, n)), r.standard_normal((n, n)), r.standard_normal((n, n))

    def f(Z):
        U, R, V, _ = adjoint.forward(Z, G, q, variant)
        return float(np.sum(Cu * U) + np.sum(Cr * R) + np.sum(Cv * V))

    U, R, V, tape = adjoint.forward(A, G, q, variant)
    g = adjoint.backward(A, U, R, V, tape, Cu, Cr, Cv, variant)
    return _rel(g, _fd_grad(f, A, 1e-6))


@pytest.mark.parametrize("q", [0, 1, 2])
@pytest.mark.parametrize("variant", ["full", "half"])
def test_chain_linear_loss_finite_differences(q, variant):
    assert _linear_fd_error(8, 6, q, variant, 21 + q) < 1e-6


def _torch_qrpos(X):
    Q, R = torch.linalg.qr(X)
    d = torch.sign(torch.diagonal(R))
    d = torch.where(d == 0, torch.ones_like(d), d)
    return Q * d, R * d[:, None]


def _torch_loss(A, G, q, k, variant):
    V = G
    if q == 0:
        V, _ = _torch_qrpos(G)
    for _ in range(q):
        X = A @ V
        P = _torch_qrpos(X)[0] if variant == "full" else X
        V, _ = _torch_qrpos(A.T @ P)
    U, R = _torch_qrpos(A @ V)
    E = A - U[:, :k] @ R[:k] @ V.T
    return (E * E).sum()


@pytest.mark.parametrize("variant", ["full", "half"])
@pytest.mark.parametrize("m,n,q,k", [(40, 30, 2, 8), (32, 32, 1, 5), (50, 20, 0, 4)])
def test_chain_against_torch_autograd(variant, m, n, q, k):
    r = _rng(m + n + q)
    sigma = 10.0 ** (-3.0 * np.arange(n) / (n - 1))
    A = _spectrum_matrix(m, n, sigma, m * n)
    G = r.standard_normal((n, n))
    L, g = adjoint.loss_and_grad(A, G, q, k, variant)
    At = torch.tensor(A, dtype=torch.float64, requires_grad=True)
    Lt = _torch_loss(At, torch.tensor(G, dtype=torch.float64), q, k, variant)
    Lt.backward()
    assert abs(L - Lt.item()) <= 1e-10 * abs(L)
    assert np.linalg.norm(g - At.grad.numpy()) <= 1e-8 * np.linalg.norm(g)


def test_k_equals_n_gives_zero():
    r = _rng(3)
    A = r.standard_normal((12, 9))
    G = r.standard_normal((9, 9))
    L, g = adjoint.loss_and_grad(A, G, 2, 9)
    assert L <= 1e-26 * np.sum(A * A)
    assert np.abs(g).max() <= 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("q", [1, 2])
def test_wide_gap_gradient_is_twice_the_residual(q):
    m, n, k = 30, 20, 5
    sigma = np.concatenate([np.linspace(2.0, 1.0, k), 1e-4 * np.linspace(1.0, 0.5, n - k)])
    A = _spectrum_matrix(m, n, sigma, 17)
    G = _rng(18).standard_normal((n, n))
    U, R, V, tape = adjoint.forward(A, G, q)
    L, dU, dR, dV, dA = adjoint.truncation_loss(A, U, R, V, k)
    g = dA + adjoint.backward(A, U, R, V, tape, dU, dR, dV)
    E = dA / 2
    assert abs(L - np.sum(sigma[k:] ** 2)) <= 1e-6 * L
    assert np.linalg.norm(g - 2 * E) <= 1e-6 * np.linalg.norm(2 * E)


@pytest.mark.parametrize("variant", ["full", "half"])
@pytest.mark.parametrize("q", [0, 1, 2])
def test_forward_is_the_oracle_factorisation(variant, q):
    r = _rng(q)
    A = r.standard_normal((23, 17))
    G = r.standard_normal((17, 17))
    U, R, V, _ = adjoint.forward(A, G, q, variant)
    U0, R0, V0 = oracle.urv(A, q, G=G, variant=variant)
    assert np.array_equal(U, U0) and np.array_equal(R, R0) and np.array_equal(V, V0)


def test_variant_none_refused():
    with pytest.raises(ValueError):
        adjoint.forward(np.eye(3), np.eye(3), 1, "none")


# ---------------------------------------------------------------- planted mistakes
def _upper_copy(M):
    return np.triu(M) + np.triu(M, 1).T


def _qr_adjoint_no_qs(Q, R, dQ=None, dR=None):
    B = np.zeros_like(Q) if dQ is None else np.asarray(dQ, dtype=np.float64).copy()
    return adjoint.solve_rt(B, R)


def _solve_r_not_rt(B, R):
    return B @ np.linalg.inv(R)  # X R = B instead of X R^T = B


def _qr_adjoint_sign(Q, R, dQ=None, dR=None):
    n = R.shape[0]
    M = np.zeros((n, n))
    if dR is not None:
        M += R @ np.asarray(dR).T
    B = np.zeros_like(Q)
    if dQ is not None:
        M += np.asarray(dQ).T @ Q       # wrong sign of Qb^T Q
        B += dQ
    B += Q @ adjoint.copyltu(M)
    return adjoint.solve_rt(B, R)


@pytest.mark.parametrize("name,attr,bad", [
    ("upper triangle", "copyltu", _upper_copy),
    ("dropped Q S term", "qr_adjoint", _qr_adjoint_no_qs),
    ("R^{-1} instead of R^{-T}", "solve_rt", _solve_r_not_rt),
    ("sign of Qb^T Q", "qr_adjoint", _qr_adjoint_sign),
])
def test_planted_mistakes_fail_the_pin(monkeypatch, name, attr, bad):
    monkeypatch.setattr(adjoint, attr, bad)
    assert max(_chain_fd_error(9, 7, 1, 3, "full", 4), _linear_fd_error(8, 6, 1, "full", 4)) > 1e-3, name


def test_planted_missing_product_term_fails(monkeypatch):
    # the reverse sweep without the Y = A^T W term (Ab += W Yb^T) of the last step
    orig = adjoint.backward

    def bad_backward(A, U, R, V, tape, dU=None, dR=None, dV=None, variant="full"):
        Xb = adjoint.qr_adjoint(U, R, dU, dR)
        Vb = np.asarray(A).T @ Xb + (0 if dV is None else dV)
        st = tape.steps[-1]
        Yb = adjoint.qr_adjoint(st["V_out"], st["Rv"], Vb, None)
        return orig(A, U, R, V, tape, dU, dR, dV, variant) - st["P"] @ Yb.T

    monkeypatch.setattr(adjoint, "backward", bad_backward)
    assert _linear_fd_error(8, 6, 1, "full", 4) > 1e-3
