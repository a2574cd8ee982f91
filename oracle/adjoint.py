"""TEST INFRASTRUCTURE ONLY -- FP64 CPU oracle of the PowerURV adjoint.

Reverse-mode derivative of the PowerURV factorisation (Gopal & Martinsson,
arXiv:1812.06007, Section 3, eqs. power and powerqr) with the Gaussian G held
fixed, for losses on the rank-k truncation A_k = U(:,1:k) R(1:k,:) V^T whose
Frobenius error is the rank-k error of Section 5 (e_k = ||R22||_F, eq. blocks).
The paper itself does not differentiate the factorisation; the adjoint of one
Householder QR used here is the published one for a tall matrix of full
column rank (Walter & Lehmann 2018; Seeger et al. 2017), derived below.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the GPU library.
The forward pass calls the C oracle (``oracle.gemm``, ``oracle.qr_pos``) in
the same order as ``orc_urv``, so its U, R, V equal the oracle's factorisation
bit for bit; the adjoint's own products use numpy matmul (FP64) and its
triangular solves are plain back substitution.

QR adjoint (X = Q R, X m x n, m >= n, R upper with non-zero diagonal).
Differentiating X = Q R gives Q^T dX R^{-1} = Q^T dQ + dR R^{-1}.  Call the
left side F.  Q^T dQ is skew-symmetric (Q^T Q = I) and dR R^{-1} is upper
triangular, so Q^T dQ = C with C = tril(F,-1) - tril(F,-1)^T, dR = (F - C) R,
and dQ = dX R^{-1} - Q (F - C).  Pairing with the adjoints Qb, Rb:
  <Qb,dQ> + <Rb,dR> = <Qb R^{-T}, dX> + <Rb R^T - Q^T Qb, F - C>,
and F - C = triu(F) + tril(F,-1)^T, so the second term is <S, F> with S the
symmetric matrix taken from the lower triangle of M = R Rb^T - Qb^T Q.  With
<S, F> = <Q S R^{-T}, dX>:
  Xb = (Qb + Q S) R^{-T}.
The sign convention diag(R) >= 0 is a fixed diagonal D = diag(sign) applied
to a QR; D is locally constant, so the same formula holds for Qpos.

Chain (FULL, q >= 1, V_0 = G):  X_t = A V_{t-1}, (W_t, Rw_t) = QRpos(X_t),
Y_t = A^T W_t, (V_t, Rv_t) = QRpos(Y_t) for t = 1..q, then (U, R) = QRpos(A V_q),
V = V_q.  HALF takes Y_t = A^T X_t and no W.  q = 0 takes V = Qpos(G), a
constant.  The reverse sweep visits the products in the opposite order: a
product P = A B contributes Ab += Pb B^T and Bb = A^T Pb; P = A^T B
contributes Ab += B Pb^T and Bb = A Pb.
"""
from __future__ import annotations

import numpy as np

from . import oracle

FULL, HALF = 0, 1
_VARIANTS = {"full": FULL, "half": HALF}


def _variant(v) -> int:
    code = _VARIANTS.get(v, -1) if isinstance(v, str) else int(v)
    if code not in (FULL, HALF):
        raise ValueError("the adjoint covers the FULL and HALF variants")
    return code


def copyltu(M: np.ndarray) -> np.ndarray:
    """Symmetric matrix whose lower triangle (diagonal included) is M's."""
    L = np.tril(M)
    return L + np.tril(M, -1).T


def solve_rt(B: np.ndarray, R: np.ndarray) -> np.ndarray:
    """X with X R^T = B for R upper triangular (n x n), by back substitution.

    Column j of X R^T is sum_{l >= j} X(:,l) R(j,l), so the last column is
    found first: X(:,j) = (B(:,j) - X(:,j+1:) R(j,j+1:)^T) / R(j,j).
    """
    n = R.shape[0]
    X = np.zeros_like(B, dtype=np.float64)
    for j in range(n - 1, -1, -1):
        X[:, j] = (B[:, j] - X[:, j + 1:] @ R[j, j + 1:]) / R[j, j]
    return X


def qr_adjoint(Q, R, dQ=None, dR=None) -> np.ndarray:
    """Adjoint of X = Q R (m x n, m >= n): Xb = (Qb + Q S) R^{-T}, S from M = R Rb^T - Qb^T Q."""
    Q = np.asarray(Q, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    n = R.shape[0]
    M = np.zeros((n, n))
    if dR is not None:
        # R's strictly lower entries are structural zeros, not functions of X,
        # so only the upper triangle of Rb carries a derivative (the lower
        # triangle of M reads only that part of Rb in any case)
        M += R @ np.triu(np.asarray(dR, dtype=np.float64)).T
    B = np.zeros_like(Q)
    if dQ is not None:
        dQ = np.asarray(dQ, dtype=np.float64)
        M -= dQ.T @ Q
        B += dQ
    B += Q @ copyltu(M)
    return solve_rt(B, R)


class Tape:
    """Intermediates of one forward pass: per power step t the V it starts from,
    the factored product (W_t or X_t) and the R factors."""

    def __init__(self):
        self.steps = []  # dicts: V_in, P (W_t for FULL, X_t for HALF), Rw (FULL), V_out, Rv


def forward(A, G, q: int, variant="full"):
    """PowerURV of A from the fixed starting matrix G, with the tape of the
    reverse sweep.  Returns U, R, V, tape (U, R, V as ``oracle.urv``)."""
    v = _variant(variant)
    A = np.asfortranarray(np.asarray(A, dtype=np.float64))
    m, n = A.shape
    V = np.asfortranarray(np.asarray(G, dtype=np.float64)).copy(order="F")
    tape = Tape()
    if q == 0:
        V, _ = oracle.qr_pos(V)  # DDH-URV (Section 2.2): V = Qpos(G)
    for _ in range(q):
        X = oracle.gemm(A, V)                                  # X = A V
        step = {"V_in": V}
        if v == FULL:
            W, Rw = oracle.qr_pos(X)                           # W = Qpos(X)
            Y = oracle.gemm(A, W, transA=True)                 # Y = A^T W
            step.update(P=W, Rw=Rw)
        else:
            Y = oracle.gemm(A, X, transA=True)                 # Y = A^T X
            step.update(P=X)
        V, Rv = oracle.qr_pos(Y)                               # V = Qpos(Y)
        step.update(V_out=V, Rv=Rv)
        tape.steps.append(step)
    X = oracle.gemm(A, V)                                      # eq. (powerqr): A V = U R
    U, R = oracle.qr_pos(X)
    return U, R, V, tape


def backward(A, U, R, V, tape: Tape, dU=None, dR=None, dV=None, variant="full") -> np.ndarray:
    """dL/dA for a loss L(U, R, V) with the given adjoints (None = zero), G fixed."""
    v = _variant(variant)
    A = np.asarray(A, dtype=np.float64)
    Xb = qr_adjoint(U, R, dU, dR)                   # final QR of X = A V_q
    Ab = Xb @ np.asarray(V, dtype=np.float64).T     # X = A V: Ab += Xb V^T
    if not tape.steps:
        return Ab                                   # q = 0: V = Qpos(G) is constant
    Vb = A.T @ Xb                                   #          Vb = A^T Xb
    if dV is not None:
        Vb = Vb + np.asarray(dV, dtype=np.float64)
    for t in range(len(tape.steps) - 1, -1, -1):
        st = tape.steps[t]
        Yb = qr_adjoint(st["V_out"], st["Rv"], Vb, None)   # V_t = Qpos(Y_t)
        Ab += st["P"] @ Yb.T                               # Y = A^T P: Ab += P Yb^T
        Pb = A @ Yb                                        #            Pb = A Yb
        if v == FULL:
            Xb = qr_adjoint(st["P"], st["Rw"], Pb, None)   # W_t = Qpos(X_t)
        else:
            Xb = Pb                                        # HALF: P is X_t itself
        Ab += Xb @ st["V_in"].T                            # X_t = A V_{t-1}
        if t > 0:
            Vb = A.T @ Xb                                  # V_0 = G is held fixed
    return Ab


def truncation_loss(A, U, R, V, k: int):
    """L = ||A - A_k||_F^2 with A_k = U(:,1:k) R(1:k,:) V^T, and the adjoints
    (dU, dR, dV, dA_direct) of L with respect to U, R, V and to A's own term."""
    A = np.asarray(A, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    Uk, Rk = U[:, :k], R[:k, :]
    E = A - Uk @ (Rk @ V.T)
    L = float(np.sum(E * E))
    Akb = -2.0 * E                          # dL/dA_k
    dU = np.zeros_like(U)
    dR = np.zeros_like(R)
    EV = Akb @ V
    dU[:, :k] = EV @ Rk.T                   # A_k = Uk (Rk V^T)
    dR[:k, :] = Uk.T @ EV                   #     = (Uk Rk) V^T
    dV = Akb.T @ (Uk @ Rk)
    return L, dU, dR, dV, 2.0 * E


def loss_and_grad(A, G, q: int, k: int, variant="full"):
    """(L, dL/dA) for L = ||A - A_k||_F^2 through the whole factorisation."""
    U, R, V, tape = forward(A, G, q, variant)
    L, dU, dR, dV, dA = truncation_loss(A, U, R, V, k)
    return L, dA + backward(A, U, R, V, tape, dU, dR, dV, variant)


def loss_only(A, G, q: int, k: int, variant="full") -> float:
    U, R, V, _ = forward(A, G, q, variant)
    return truncation_loss(A, U, R, V, k)[0]
