"""Parity of the batched factorisation (many FP32 matrices in one persistent
launch) with the FP64 oracle, matrix by matrix, through the C ABI.

Matrix i is PowerURV (Section 3, eqs. power and powerqr, FULL) of A_i with
G_i = fl32 of the Gaussian of seed + i, stream 2; the oracle factors the same
FP32 values of A_i in FP64 from the same G_i.  Bounds (FP32 arithmetic on the
GPU against FP64), with ||A||_F the matrix's Frobenius norm:
- ||R - R_orc||_F <= 1e-4 ||A||_F and max_k |e_k - e_k_orc| <= 1e-4 ||A||_F
  (the FP32 bar of the factorisation; e_k = ||R(k:, k:)||_F, Section 5);
- ||U^T U - I||_F, ||V^T V - I||_F <= max(1e-5, 2 n^1.5 eps32) and
  ||A - U R V^T||_F <= max(1e-6, 2 n eps32) ||A||_F (Householder QR in FP32:
  orthogonality error of order n eps32 in the 2-norm, up to sqrt(n) more in
  the Frobenius norm).
The schedule (workgroup count) never changes the bits of a result; graph
replays reproduce the eager launch bit for bit.
"""
import numpy as np
import pytest

import urv_inputs as gen
from gpu_helpers import announce, to_gpu, to_np

pytestmark = pytest.mark.gpu

SMALL = [(64, 32), (100, 100), (300, 37), (257, 200), (1024, 40), (130, 130), (70, 1), (33, 33),
         (512, 300), (200, 17), (96, 95)]
SEED = 900
EPS32 = float(np.finfo(np.float32).eps)


def _orth_bound(n):
    return max(1e-5, 2.0 * n ** 1.5 * EPS32)


def _recon_bound(n):
    return max(1e-6, 2.0 * n * EPS32)


@pytest.fixture(scope="module")
def urv():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1812_06007_amd import urv as u

    u.lib()
    return u


def _matrices(sizes, base):
    out = []
    for i, (m, n) in enumerate(sizes):
        A = gen.spectral_matrix(m, n, gen.spectrum("geometric6", n), base + i)
        out.append(A.astype(np.float32).astype(np.float64))
    return out


def _oracle_g(orc, n, seed):
    """G of the batched path: FP32 rounding of the oracle's Gaussian (seed, stream 2)."""
    return orc.gaussian(n, n, seed, stream_id=2).astype(np.float32).astype(np.float64)


_ORACLE = {}


def _oracle(orc, sizes, q):
    key = (tuple(sizes), q)
    if key not in _ORACLE:
        res = []
        for i, A in enumerate(_matrices(sizes, SEED)):
            n = A.shape[1]
            U, R, V = orc.urv(A, q, G=_oracle_g(orc, n, SEED + i))
            res.append((U, R, V, orc.metrics(A, U, R, V)))
        _ORACLE[key] = res
    return _ORACLE[key]


def _run(urv, sizes, q, nb=None, grid=None, graph=False, team=1):
    import torch

    ms, ns = [s[0] for s in sizes], [s[1] for s in sizes]
    plan = urv.BatchPlan(ms, ns, q=q, seed=SEED)
    A = [to_gpu(a).float() for a in _matrices(sizes, SEED)]
    U, R, V = urv.batch_outputs(ms, ns)
    plan.set_buffers(A, U, R, V)
    if nb is not None:
        plan.set_config(nb, grid if grid else plan.config()[1], team)
    plan.run(graph=graph)
    torch.cuda.synchronize()
    plan.status()
    return plan, A, U, R, V


def _check_against_oracle(A_np, ref, U, R, V):
    Ur, Rr, Vr, met = ref
    Ug, Rg, Vg = to_np(U), to_np(R), to_np(V)
    n = A_np.shape[1]
    na = np.linalg.norm(A_np)
    assert np.linalg.norm(Rg - Rr) <= 1e-4 * na
    ek = np.array([np.linalg.norm(np.triu(Rg[k:, k:])) for k in range(n + 1)])
    assert np.max(np.abs(ek - met["ek"])) <= 1e-4 * na
    assert np.linalg.norm(Ug.T @ Ug - np.eye(n)) <= _orth_bound(n)
    assert np.linalg.norm(Vg.T @ Vg - np.eye(n)) <= _orth_bound(n)
    assert np.linalg.norm(A_np - Ug @ Rg @ Vg.T) <= _recon_bound(n) * na
    assert np.all(np.diag(Rg) >= 0) and np.all(np.tril(Rg, -1) == 0)


@pytest.mark.parametrize("nb", [16, 32])
@pytest.mark.parametrize("q", [0, 1, 2])
def test_batched_matches_oracle(urv, orc, nb, q):
    announce("batched parity", nb, q)
    ref = _oracle(orc, SMALL, q)
    plan, A, U, R, V = _run(urv, SMALL, q, nb=nb, grid=64)
    for i, A_np in enumerate(_matrices(SMALL, SEED)):
        _check_against_oracle(A_np, ref[i], U[i], R[i], V[i])
    plan.close()


def test_schedule_does_not_change_the_bits(urv):
    """Workgroup counts and teams (GEMM tiles and element ranges split over
    several workgroups with device-wide barriers) give the same bits."""
    announce("batched schedules")
    outs = []
    for grid, team in ((1, 1), (7, 1), (256, 1), (1024, 1), (None, 4), (None, 16), (None, 64)):
        plan, A, U, R, V = _run(urv, SMALL, 1, nb=32, grid=grid, team=team)
        outs.append([to_np(t) for t in U + R + V])
        plan.close()
    for other in outs[1:]:
        assert all(np.array_equal(a, b) for a, b in zip(outs[0], other))


def test_teams_match_oracle(urv, orc):
    announce("batched teams parity")
    ref = _oracle(orc, SMALL, 2)
    plan, A, U, R, V = _run(urv, SMALL, 2, nb=16, team=16)
    for i, A_np in enumerate(_matrices(SMALL, SEED)):
        _check_against_oracle(A_np, ref[i], U[i], R[i], V[i])
    plan.close()


def test_team_grid_beyond_capacity_is_refused(urv):
    announce("batched team capacity check")
    ms, ns = [s[0] for s in SMALL], [s[1] for s in SMALL]
    plan = urv.BatchPlan(ms, ns, q=1, seed=SEED)
    cap = plan.config()[1]
    with pytest.raises(urv.UrvError):
        plan.set_config(32, cap + 1, 4)
    plan.set_config(32, cap + 1, 1)  # a single-workgroup schedule needs no residency
    plan.close()


def test_graph_replays_reproduce_the_eager_launch(urv):
    import torch

    announce("batched graph")
    ms, ns = [s[0] for s in SMALL], [s[1] for s in SMALL]
    plan, A, U, R, V = _run(urv, SMALL, 1, nb=16, team=4)
    eager = [to_np(t) for t in U + R + V]
    scratch = torch.ones(1 << 20, device="cuda")
    for rep in range(3):
        for t in U + R + V:
            t.zero_()
        plan.run(graph=True)
        scratch.mul_(1.0001)  # the program's own work between replays
        torch.cuda.synchronize()
        plan.status()
        assert all(np.array_equal(a, to_np(b)) for a, b in zip(eager, U + R + V)), rep
    # new output buffers: the captured launch reads the descriptors, so it writes there
    U2, R2, V2 = urv.batch_outputs(ms, ns)
    plan.set_buffers(A, U2, R2, V2)
    plan.run(graph=True)
    torch.cuda.synchronize()
    assert all(np.array_equal(a, to_np(b)) for a, b in zip(eager, U2 + R2 + V2))
    plan.close()


def test_autotune_keeps_a_valid_result(urv, orc):
    import torch

    announce("batched autotune")
    ref = _oracle(orc, SMALL, 1)
    plan, A, U, R, V = _run(urv, SMALL, 1)
    ms = plan.autotune()
    assert ms > 0
    nb, grid, team = plan.config()
    assert nb in (16, 32) and team in (1, 2, 4, 8, 16) and grid >= 1
    plan.run(graph=True)
    torch.cuda.synchronize()
    for i, A_np in enumerate(_matrices(SMALL, SEED)):
        _check_against_oracle(A_np, ref[i], U[i], R[i], V[i])
    plan.close()


def test_full_batch_workload(urv, orc):
    """512 matrices, m ~ U[64, 1024], n ~ U[32, m], sigma_j = 10^(-6 (j-1)/(n-1)),
    q = 1, autotuned, through the graph: invariants of every matrix on the GPU
    and the oracle on a sample (the largest, the smallest and two others)."""
    import torch

    announce("batched full workload")
    rng = gen.generator(1812, 6)
    count = 512
    ms = [int(x) for x in rng.integers(64, 1025, size=count)]
    ns = [int(rng.integers(32, m + 1)) for m in ms]
    A = []
    for i, (m, n) in enumerate(zip(ms, ns)):
        A.append(gen.spectral_matrix(m, n, gen.spectrum("geometric6", n), 1812 + i, device="cuda").float()
                 .t().contiguous().t())
    U, R, V = urv.batch_outputs(ms, ns)
    plan = urv.BatchPlan(ms, ns, q=1, seed=1812)
    plan.set_buffers(A, U, R, V)
    plan.autotune()
    plan.run(graph=True)
    torch.cuda.synchronize()
    plan.status()
    worst = {"orthU": 0.0, "orthV": 0.0, "recon": 0.0}  # each as a fraction of its bound
    for i in range(count):
        Ad, Ud, Rd, Vd = (t.double() for t in (A[i], U[i], R[i], V[i]))
        n = ns[i]
        eye = torch.eye(n, dtype=torch.float64, device="cuda")
        worst["orthU"] = max(worst["orthU"], float(torch.linalg.norm(Ud.t() @ Ud - eye)) / _orth_bound(n))
        worst["orthV"] = max(worst["orthV"], float(torch.linalg.norm(Vd.t() @ Vd - eye)) / _orth_bound(n))
        worst["recon"] = max(worst["recon"], float(torch.linalg.norm(Ad - Ud @ Rd @ Vd.t()) /
                                                   torch.linalg.norm(Ad)) / _recon_bound(n))
    print("[gpu-case] worst fraction of the bounds", worst, "config", plan.config(), flush=True)
    assert max(worst.values()) <= 1.0
    costs = [m * n * n for m, n in zip(ms, ns)]
    sample = {int(np.argmax(costs)), int(np.argmin(costs)), 17, 300}
    for i in sorted(sample):
        A_np = to_np(A[i])
        Ur, Rr, Vr = orc.urv(A_np, 1, G=_oracle_g(orc, ns[i], 1812 + i))
        _check_against_oracle(A_np, (Ur, Rr, Vr, orc.metrics(A_np, Ur, Rr, Vr)), U[i], R[i], V[i])
    plan.close()
