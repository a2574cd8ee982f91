"""Parity of the derivative of PowerURV (G held fixed) with the FP64 oracle,
through the C ABI: the adjoint of one QR, the reverse sweep through the power
steps of Section 3 (eqs. power and powerqr), the rank-k truncation loss of
Section 5, the tape modes, and the torch.autograd functions.

Tolerances (normwise, relative to the oracle's FP64 result):
- FP64: 1e-11 for one QR adjoint and 1e-10 for the chain.  Rounding enters
  as eps64 = 1.1e-16 times the condition of the R factors (up to ~1e4 on
  these inputs) and a growth of order n.
- FP32: 2e-5 for one QR adjoint, 1e-4 for the small chains, 2e-4 at the
  full 2048 x 2048 workload.  An FP32 emulation of the same formulas with
  LAPACK's FP32 QR and BLAS differs from FP64 by 2e-7 .. 7e-7 for one QR
  adjoint, 4e-7 .. 2.3e-6 on the small chains and 3.2e-5 at 2048 x 2048
  (q = 2, k = 256).  HALF squares the condition of each iterate (A^T A V),
  and the blocked QR and the MFMA GEMM sum in other orders than LAPACK, so
  single cases land up to ~10x from the emulation either way (2.2e-5 for the
  129 x 129 HALF case, 1.8e-6 at 2048 x 2048).
The forward factors are held to the bar of the factorisation tests
(||R - R_orc||_F <= 1e-11 ||A||_F in FP64).
"""
import numpy as np
import pytest

import urv_inputs as gen
from gpu_helpers import announce, to_gpu, to_np
from oracle import adjoint

pytestmark = pytest.mark.gpu

TOL = {("fp64", "qr"): 1e-11, ("fp64", "chain"): 1e-10, ("fp32", "qr"): 2e-5, ("fp32", "chain"): 1e-4}


@pytest.fixture(scope="module")
def urv():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1812_06007_amd import urv as u

    u.lib()
    return u


def _dt(name):
    import torch

    return torch.float64 if name == "fp64" else torch.float32


def _dev(a, dtype):
    return to_gpu(a).to(_dt(dtype))


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ---------------------------------------------------------------- one QR
QR_SHAPES = [(300, 200), (257, 257), (130, 64), (200, 65), (129, 128), (70, 1), (64, 64)]


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", QR_SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("which", ["both", "dQ", "dR"])
def test_qr_adjoint_matches_oracle(urv, orc, dtype, shape, which):
    m, n = shape
    announce("qr_adjoint", dtype, shape, which)
    rng = gen.generator(m * n, 7)
    X = rng.standard_normal((m, n))
    dQ = rng.standard_normal((m, n)) if which in ("both", "dQ") else None
    dR = rng.standard_normal((n, n)) if which in ("both", "dR") else None
    Q, R = orc.qr_pos(X)
    if dtype == "fp32":  # the reference takes the same FP32-rounded inputs
        Q, R = Q.astype(np.float32).astype(np.float64), R.astype(np.float32).astype(np.float64)
        dQ = None if dQ is None else dQ.astype(np.float32).astype(np.float64)
        dR = None if dR is None else dR.astype(np.float32).astype(np.float64)
    ref = adjoint.qr_adjoint(Q, R, dQ, dR)
    out = urv.qr_adjoint(_dev(Q, dtype), _dev(R, dtype), None if dQ is None else _dev(dQ, dtype),
                         None if dR is None else _dev(dR, dtype))
    assert _rel(to_np(out), ref) <= TOL[(dtype, "qr")]



@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [129, 64, 1])
def test_qr_adjoint_square_zero_last_pivot(urv, orc, dtype, n):
    # A numerically singular square X can leave R(n, n) = 0 exactly.  The
    # adjoint then stays finite and equals the limit R(n, n) -> 0 of the
    # oracle's: at R(n, n) = 1e-6 the oracle differs from that limit by terms
    # of order 1e-6 (R(n, n) Rb) and 1e-16 / 1e-6 ((I - Q Q^T) Qb / R(n, n)).
    announce("qr_adjoint zero pivot", dtype, n)
    rng = gen.generator(n + 31, 7)
    Q, R = orc.qr_pos(rng.standard_normal((n, n)))
    dQ, dR = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    Rz, Re = R.copy(), R.copy()
    Rz[-1, -1], Re[-1, -1] = 0.0, 1e-6
    ref = adjoint.qr_adjoint(Q, Re, dQ, dR)
    out = to_np(urv.qr_adjoint(_dev(Q, dtype), _dev(Rz, dtype), _dev(dQ, dtype), _dev(dR, dtype)))
    assert np.isfinite(out).all()
    assert _rel(out, ref) <= (1e-5 if dtype == "fp64" else 1e-4)

# ---------------------------------------------------------------- the chain
def _inputs(kind, m, n, k, seed):
    if kind == "spike":
        return gen.spiked_gaussian(m, n, max(k, 1), 10.0, seed)
    sigma = 10.0 ** (-3.0 * np.arange(n) / max(n - 1, 1))
    return gen.spectral_matrix(m, n, sigma, seed)


CHAIN = [  # m, n, q, k, variant, input
    (260, 200, 2, 20, "full", "spike"),
    (200, 200, 1, 30, "half", "geometric3"),
    (150, 130, 0, 10, "full", "spike"),
    (300, 140, 2, 140, "full", "geometric3"),
    (129, 129, 2, 64, "half", "spike"),
    (257, 193, 3, 65, "full", "spike"),
]


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CHAIN, ids=lambda c: "%dx%d-q%d-k%d-%s-%s" % c)
def test_gradient_matches_oracle(urv, dtype, case):
    m, n, q, k, variant, kind = case
    announce("grad chain", dtype, case)
    A = _inputs(kind, m, n, k, m + n)
    G = gen.gaussian(n, n, 1812)
    if dtype == "fp32":
        A, G = A.astype(np.float32).astype(np.float64), G.astype(np.float32).astype(np.float64)
    U0, R0, V0, tape0 = adjoint.forward(A, G, q, variant)
    L0, dU0, dR0, dV0, dA0 = adjoint.truncation_loss(A, U0, R0, V0, k)
    ref = dA0 + adjoint.backward(A, U0, R0, V0, tape0, dU0, dR0, dV0, variant)

    Ad, Gd = _dev(A, dtype), _dev(G, dtype)
    U, R, V, tape = urv.factor_tape(Ad, Gd, q, variant)
    L, dU, dR, dV, dA = urv.truncation_loss(Ad, U, R, V, k)
    urv.factor_backward(Ad, Gd, U, R, V, tape, q, dU, dR, dV, variant, dA=dA, accumulate=True)
    normA = np.linalg.norm(A)
    eps = np.finfo(np.float64 if dtype == "fp64" else np.float32).eps
    if k == n:  # A_k = A: the loss and the gradient vanish up to rounding
        assert L.item() <= (1e3 * eps * normA) ** 2
        assert np.abs(to_np(dA)).max() <= 1e3 * eps * np.abs(A).max()
    else:
        assert abs(L.item() - L0) <= (1e-10 if dtype == "fp64" else 1e-4) * L0
        assert _rel(to_np(dA), ref) <= TOL[(dtype, "chain")]
    # the forward R: in FP32 the trailing columns of V carry eps32 times the
    # condition of the iterate (squared by HALF's A^T A), hence the wider bound
    fwd_tol = 1e-11 if dtype == "fp64" else (1e-3 if variant == "half" else 1e-4)
    assert np.linalg.norm(to_np(R) - R0) <= fwd_tol * normA


@pytest.mark.parametrize("variant", ["full", "half"])
def test_linear_loss_gradient_matches_oracle(urv, variant):
    """A loss that reads every entry of U, R and V exercises every term of the
    QR adjoints (the truncation loss cancels the within-span ones)."""
    m, n, q = 190, 150, 2
    announce("grad linear", variant)
    sigma = np.linspace(1.0, 0.1, n)
    A = gen.spectral_matrix(m, n, sigma, 77)
    G = gen.gaussian(n, n, 78)
    r = gen.generator(79, 0)
    Cu, Cr, Cv = r.standard_normal((m, n)), r.standard_normal((n, n)), r.standard_normal((n, n))
    U0, R0, V0, tape0 = adjoint.forward(A, G, q, variant)
    ref = adjoint.backward(A, U0, R0, V0, tape0, Cu, Cr, Cv, variant)
    Ad, Gd = to_gpu(A), to_gpu(G)
    U, R, V, tape = urv.factor_tape(Ad, Gd, q, variant)
    dA = urv.factor_backward(Ad, Gd, U, R, V, tape, q, to_gpu(Cu), to_gpu(Cr), to_gpu(Cv), variant)
    assert _rel(to_np(dA), ref) <= TOL[("fp64", "chain")]


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("variant,q", [("full", 2), ("full", 3), ("half", 2), ("full", 1)])
def test_tape_modes_give_identical_gradients(urv, dtype, variant, q):
    """Keeping every factor, only the V's, or nothing (recomputing from G)
    gives the same bits: the QR and the GEMM are deterministic."""
    m, n, k = 200, 150, 12
    announce("tape modes", dtype, variant, q)
    A = _dev(gen.spiked_gaussian(m, n, k, 10.0, 5), dtype)
    G = _dev(gen.gaussian(n, n, 6), dtype)
    grads = {}
    for mode in ("all", "v", "none"):
        U, R, V, tape = urv.factor_tape(A, G, q, variant, mode)
        L, dU, dR, dV, dA = urv.truncation_loss(A, U, R, V, k)
        urv.factor_backward(A, G, U, R, V, tape, q, dU, dR, dV, variant, mode, dA=dA, accumulate=True)
        grads[mode] = to_np(dA)
        fwd = (to_np(U), to_np(R), to_np(V))
        if mode == "all":
            fwd0 = fwd
        else:
            assert all(np.array_equal(a, b) for a, b in zip(fwd, fwd0))
    assert np.array_equal(grads["all"], grads["v"]) and np.array_equal(grads["all"], grads["none"])


def test_k_zero_gradient_is_twice_a(urv):
    """k = 0: A_k = 0, L = ||A||^2 and dL/dA = 2A exactly (zero seeds give a
    zero reverse sweep)."""
    m, n = 160, 120
    announce("k = 0")
    A = gen.spiked_gaussian(m, n, 8, 10.0, 9)
    Ad, Gd = to_gpu(A), to_gpu(gen.gaussian(n, n, 10))
    U, R, V, tape = urv.factor_tape(Ad, Gd, 2)
    L, dU, dR, dV, dA = urv.truncation_loss(Ad, U, R, V, 0)
    urv.factor_backward(Ad, Gd, U, R, V, tape, 2, dU, dR, dV, dA=dA, accumulate=True)
    assert np.array_equal(to_np(dA), 2 * A)
    assert abs(L.item() - np.sum(A * A)) <= 1e-13 * np.sum(A * A)


def test_backward_accumulates(urv):
    m, n, q = 140, 100, 1
    announce("accumulate")
    A = to_gpu(gen.spiked_gaussian(m, n, 6, 10.0, 11))
    G = to_gpu(gen.gaussian(n, n, 12))
    U, R, V, tape = urv.factor_tape(A, G, q)
    r = gen.generator(13, 0)
    dU = to_gpu(r.standard_normal((m, n)))
    g = urv.factor_backward(A, G, U, R, V, tape, q, dU=dU)
    base = to_gpu(r.standard_normal((m, n)))
    acc = base.clone()
    urv.factor_backward(A, G, U, R, V, tape, q, dU=dU, dA=acc, accumulate=True)
    np.testing.assert_allclose(to_np(acc), to_np(base) + to_np(g), rtol=0, atol=1e-13 * np.abs(to_np(g)).max())


# ---------------------------------------------------------------- torch.autograd
def test_autograd_function_against_oracle_and_finite_differences(urv):
    import torch

    from paper_1812_06007_amd.autograd import power_urv, truncation_loss

    m, n, q, k = 180, 150, 2, 16
    announce("autograd")
    A_np = gen.spiked_gaussian(m, n, k, 10.0, 21)
    G_np = gen.gaussian(n, n, 22)
    L_ref, g_ref = adjoint.loss_and_grad(A_np, G_np, q, k)
    G = to_gpu(G_np)

    # the library's loss
    A = to_gpu(A_np).requires_grad_(True)
    U, R, V = power_urv(A, G, q)
    L = truncation_loss(A, U, R, V, k)
    L.backward()
    assert abs(L.item() - L_ref) <= 1e-10 * L_ref
    assert _rel(to_np(A.grad), g_ref) <= TOL[("fp64", "chain")]

    # the same loss written with torch operations (FP64 products)
    A2 = to_gpu(A_np).requires_grad_(True)
    U2, R2, V2 = power_urv(A2, G, q)
    E = A2 - (U2[:, :k] @ R2[:k, :]) @ V2.t().contiguous()
    L2 = (E * E).sum()
    L2.backward()
    assert _rel(to_np(A2.grad), g_ref) <= 1e-9

    # central differences along two seeded directions, on the GPU in FP64
    with torch.no_grad():
        for s in (31, 32):
            D = to_gpu(gen.generator(s, 0).standard_normal((m, n)))
            h = 1e-6

            def loss_at(Z):
                Uz, Rz, Vz = power_urv(Z, G, q)
                return truncation_loss(Z, Uz, Rz, Vz, k).item()

            fd = (loss_at(to_gpu(A_np) + h * D) - loss_at(to_gpu(A_np) - h * D)) / (2 * h)
            ana = float((A.grad * D).sum())
            assert abs(fd - ana) <= 1e-6 * abs(ana) + 1e-8 * L_ref


def test_autograd_fp32_half_tape_none(urv):
    import torch

    from paper_1812_06007_amd.autograd import power_urv, truncation_loss

    m, n, q, k = 200, 160, 2, 24
    announce("autograd fp32 half none")
    A_np = gen.spiked_gaussian(m, n, k, 10.0, 41).astype(np.float32).astype(np.float64)
    G_np = gen.gaussian(n, n, 42).astype(np.float32).astype(np.float64)
    _, g_ref = adjoint.loss_and_grad(A_np, G_np, q, k, "half")
    A = to_gpu(A_np).float().requires_grad_(True)
    U, R, V = power_urv(A, to_gpu(G_np).float(), q, "half", "none")
    assert U.dtype == torch.float32
    truncation_loss(A, U, R, V, k).backward()
    assert _rel(to_np(A.grad), g_ref) <= TOL[("fp32", "chain")]


# ---------------------------------------------------------------- the full workload
def test_full_size_fp32_against_fp64_oracle(urv):
    """A 2048 x 2048 FP32: Gaussian N(0, 1/2048) plus a rank-256 spike of 10;
    q = 2, k = 256, FULL, G fixed: the GPU gradient in FP32 against the FP64
    oracle's.  The reverse sweep's share of the gradient (beyond the loss's
    own 2 (A - A_k)) is reported: it is not small here, because q = 2 steps
    without oversampling leave U(:,1:k) well away from the dominant subspace."""
    m = n = 2048
    q, k = 2, 256
    announce("full size fp32", m, n, q, k)
    A_np = gen.spiked_gaussian(m, n, k, 10.0, 1812)
    G_np = gen.gaussian(n, n, 1812)
    A32, G32 = A_np.astype(np.float32).astype(np.float64), G_np.astype(np.float32).astype(np.float64)
    Ad, Gd = to_gpu(A32).float(), to_gpu(G32).float()
    U, R, V, tape = urv.factor_tape(Ad, Gd, q)
    L, dU, dR, dV, dA = urv.truncation_loss(Ad, U, R, V, k)
    E2 = to_np(dA)
    urv.factor_backward(Ad, Gd, U, R, V, tape, q, dU, dR, dV, dA=dA, accumulate=True)
    g = to_np(dA)
    print("[gpu-case] oracle gradient at 2048 (CPU)", flush=True)
    L0, g0 = adjoint.loss_and_grad(A32, G32, q, k)
    print("[gpu-case] rel err", _rel(g, g0), "loss", L.item(), L0, flush=True)
    print("[gpu-case] sweep share", np.linalg.norm(g - E2) / np.linalg.norm(E2), flush=True)
    assert abs(L.item() - L0) <= 1e-4 * L0
    assert _rel(g, g0) <= 2e-4
