"""Benchmark: PowerURV on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 8000] [--q 2] [--variant full]

A step is one whole factorisation A = U R V^T (Gaussian draw, q power steps,
final QR) of the 8000 x 8000 FP64 matrix A = Q1 diag(1/j^2) Q2^T with Haar
Q1, Q2, inputs and workspace resident in HBM.  The printed JSON line carries
TFLOP/s at the standard operation count (LAPACK counts of the products,
factorisations and explicit U and V; the executed count beside it), the
reconstruction error, the MFMA roofline of the dominant kernel (the library's
FP64 launches timed live with HIP events on the streams they run on, during
the timed steps; the A V GEMM alone beside it),
the mixed-precision forms (BF16 / FP16 power steps) against plain FP64 on the
same input and on the 16000 x 8000 noisy exp(-j/800) matrix, the
differentiation workload (forward, truncation loss and reverse sweep of a
2048 x 2048 FP32 matrix with G fixed, against the FP64 oracle's gradient), the
batched workload (512 FP32 matrices of mixed sizes in one persistent launch,
replayed from a graph), and the FP64 CPU oracle timed on a bounded sample of
the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "PowerURV TFLOP/s & time (n=8000,q=2) mixed vs FP64; ||A−URV||/||A||"
FP64_MFMA_PEAK_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_nn_av_8000_traffic.txt")
CLASS_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "powerurv_fp64_8000_q2_traffic.txt")
CSRC = os.path.join(ROOT, "paper_1812_06007_amd", "csrc")
GEMM_SOURCES = [os.path.join(CSRC, f) for f in ("gemm.hip", "common.hpp")]
# the factorisation's launches (their shapes and kernels) follow from these
PIPELINE_SOURCES = [os.path.join(CSRC, f) for f in ("gemm.hip", "common.hpp", "qr.hip", "api.hip")]


def source_hash(paths) -> str:
    """sha256 over the given source files, in order."""
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def gemm_source_hash() -> str:
    """sha256 over the sources the GEMM kernel is built from."""
    return source_hash(GEMM_SOURCES)


def _summary_keys(path: str) -> dict:
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#") and not line.startswith(" "):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv


def class_traffic(cls: str, m: int, n: int, q: int, variant: str):
    """HBM bytes per launch of a launch class of the FP64 factorisation, from the
    committed rocprofv3 PMC summary (FETCH_SIZE + WRITE_SIZE per dispatch,
    copy-calibrated, averaged over the class's dispatches of one factorisation), or
    None when that summary is for another workload or for other sources."""
    try:
        kv = _summary_keys(CLASS_TRAFFIC_FILE)
        if kv.get("pipeline_source_sha256") != source_hash(PIPELINE_SOURCES):
            return None
        if kv.get("workload") != "%dx%d q=%d %s" % (m, n, q, variant):
            return None
        return float(kv["bytes_per_launch." + cls])
    except (OSError, KeyError, ValueError):
        return None


def gemm_traffic(m: int, n: int):
    """HBM bytes per launch of the A V GEMM from the committed rocprofv3 PMC
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when that
    summary is for another shape or for an older gemm.hip."""
    try:
        kv = _summary_keys(TRAFFIC_FILE)
        if kv.get("gemm_source_sha256") != gemm_source_hash() or kv.get("shape") != "%dx%dx%d" % (m, n, n):
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None



def standard_flops(m: int, n: int, q: int, variant: str, orth_g: bool = False) -> float:
    """Standard (LAPACK) operation count of the algorithm as the driver runs it: every
    product with A or A^T 2 m n^2 (2q + 1 of them), every Householder factorisation or
    explicit-Q formation of an m x n matrix 2 m n^2 - 2/3 n^3 (n x n: 4/3 n^3).
    Factorisations: FULL q (X, m x n) + q (A^T W, n x n), HALF q (n x n), NONE one n x n
    (q > 0), plus Qpos(G) when q == 0 or orth_g, plus the final A V = U R; explicit Q:
    V (n x n) and U (m x n).  FULL, q = 2, m = n: 58/3 n^3."""
    m, n = float(m), float(n)
    gemm = (2 * q + 1) * 2 * m * n * n
    f_mn = 2 * m * n * n - 2.0 / 3.0 * n ** 3
    f_nn = 4.0 / 3.0 * n ** 3
    if variant == "full":
        fact = q * (f_mn + f_nn) + f_mn
    elif variant == "half":
        fact = q * f_nn + f_mn
    else:
        fact = (f_nn if q > 0 else 0.0) + f_mn
    if q == 0 or orth_g:
        fact += f_nn
    return gemm + fact + f_nn + f_mn


def executed_flops(m: int, n: int, q: int, variant: str, orth_g: bool = False) -> float:
    """What the driver executes: the standard count, except that U, when m == n, is formed
    by applying the final QR's reflectors to an identity alongside it (Z <- Z Q,
    4 z m n - 2 z n^2 with z the rows of Z: 2 n^3 for n x n) rather than by the structured
    formation (4/3 n^3).  V is formed structurally from its QR's reflectors, beside the
    final QR.  The products A^T W and A V of FULL are applied to A^T and A as targets of
    the QRs at the cost of the products they replace."""
    n_ = float(n)
    extra = 0.0
    if m == n:
        extra += 2.0 * n_ ** 3 - 4.0 / 3.0 * n_ ** 3  # U
    return standard_flops(m, n, q, variant, orth_g) + extra


def paper_flops(m: int, n: int, q: int) -> float:
    """Leading-order count of the paper's Table 1, GEMM term read as 2(2q+1) m n^2."""
    m, n = float(m), float(n)
    return 2 * (2 * q + 1) * m * n * n + (4 * q + 2) * m * n * n - 2.0 / 3.0 * (2 * q + 1) * n ** 3


def cpu_baseline(q: int, variant: str, sample_n: int) -> dict:
    """The FP64 oracle (plain loops, OpenMP over columns) on an n x n sample of the workload."""
    import numpy as np

    import urv_inputs as gen
    from oracle import oracle

    oracle.build()
    A = gen.spectral_matrix(sample_n, sample_n, gen.spectrum("poly2", sample_n), seed=1812)
    t0 = time.perf_counter()
    oracle.urv(A, q, seed=1812, variant=variant)
    dt = time.perf_counter() - t0
    fl = standard_flops(sample_n, sample_n, q, variant)
    cores = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)) or 1)
    return {"value": fl / dt / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "sample": "oracle PowerURV %s q=%d on %dx%d, sigma_j=1/j^2: %.2f s for %.3e flop"
                      % (variant.upper(), q, sample_n, sample_n, dt, fl),
            "seconds": dt}


FP32_MFMA_PEAK_TFLOPS = 157.3


def grad_flops(m: int, n: int, q: int, k: int, variant: str = "full") -> dict:
    """Operation counts of the differentiable FULL/HALF chain (standard counts,
    explicit Q included): the forward pass, the truncation loss with its
    adjoints, and the reverse sweep.  One QR adjoint of an m x n factor costs
    Qb^T Q, Q S (2mn^2 each) and the solve with R^T (mn^2); with an R
    adjoint R Rb^T adds 2n^3."""
    m, n, k = float(m), float(n), float(k)
    fwd = standard_flops(m, n, q, variant)
    loss = 4 * m * n * n + 2 * k * n * n + 8 * m * n * k
    bwd = 5 * m * n * n + 2 * n ** 3 + 4 * m * n * n          # final QR adjoint, Xb V^T, A^T Xb
    per = 5 * n ** 3 + 8 * m * n * n + (5 * m * n * n if variant == "full" else 0.0)
    bwd += q * per - 2 * m * n * n  # no A^T Xb where the sweep ends (V_0 = G, or q = 0)
    return {"forward": fwd, "loss": loss, "backward": bwd, "total": fwd + loss + bwd}


def bench_grad(steps: int, warmup: int, oracle_check: bool) -> dict:
    """The differentiation workload: A 2048 x 2048 FP32 = N(0, 1/2048) + a
    rank-256 spike of 10, G fixed, q = 2 FULL, loss ||A - A_k||_F^2 with
    k = 256; forward (with tape), loss and reverse sweep timed together."""
    import numpy as np
    import torch

    import urv_inputs as gen
    from paper_1812_06007_amd import urv

    m = n = 2048
    q, k = 2, 256
    A_np = gen.spiked_gaussian(m, n, k, 10.0, 1812).astype(np.float32)
    G_np = gen.gaussian(n, n, 1812).astype(np.float32)
    A = torch.from_numpy(np.ascontiguousarray(A_np.T)).cuda().t()
    G = torch.from_numpy(np.ascontiguousarray(G_np.T)).cuda().t()
    ws = torch.empty(urv.grad_workspace_size(m, n, q, torch.float32), dtype=torch.uint8, device=A.device)
    state = {}

    def fwd():
        state["f"] = urv.factor_tape(A, G, q, workspace=ws)

    def step():
        U, R, V, tape = urv.factor_tape(A, G, q, workspace=ws)
        L, dU, dR, dV, dA = urv.truncation_loss(A, U, R, V, k, workspace=ws)
        urv.factor_backward(A, G, U, R, V, tape, q, dU, dR, dV, dA=dA, accumulate=True, workspace=ws)
        state["out"] = (L, dA)

    def timed(fn, reps):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_fwd = timed(fwd, steps)
    ms = timed(step, steps)
    L, dA = state["out"]
    fl = grad_flops(m, n, q, k)
    res = {"workload": "A 2048x2048 FP32 = N(0,1/2048) + rank-256 spike x10, G fixed (seed 1812), q=2 FULL, "
                       "loss ||A - A_k||_F^2, k=256; forward with tape + loss + reverse sweep",
           "dtype": "f32", "ms_forward": ms_fwd, "ms_forward_loss_backward": ms,
           "flops_executed": fl["total"], "tflops": fl["total"] / (ms * 1e-3) / 1e12,
           "frac_fp32_peak": fl["total"] / (ms * 1e-3) / 1e12 / FP32_MFMA_PEAK_TFLOPS,
           "loss": float(L.item())}
    if oracle_check:
        from oracle import adjoint, oracle

        oracle.build()
        t0 = time.perf_counter()
        L0, g0 = adjoint.loss_and_grad(A_np.astype(np.float64), G_np.astype(np.float64), q, k)
        dt = time.perf_counter() - t0
        g = dA.t().contiguous().t().cpu().double().numpy()
        res["grad_rel_err_vs_fp64_oracle"] = float(np.linalg.norm(g - g0) / np.linalg.norm(g0))
        res["loss_rel_err_vs_fp64_oracle"] = abs(res["loss"] - L0) / L0
        cores = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)) or 1)
        res["cpu_baseline"] = {"value": fl["total"] / dt / 1e12, "unit": "TFLOP/s", "cores": cores,
                               "kind": "oracle", "seconds": dt,
                               "sample": "FP64 oracle loss and gradient of the same 2048x2048 workload "
                                         "(C loops for the forward, numpy FP64 for the adjoint)"}
    del ws
    torch.cuda.empty_cache()
    return res


def batched_workload(device):
    """512 FP32 matrices, m ~ U[64, 1024], n ~ U[32, m], sigma_j = 10^(-6 (j-1)/(n-1)),
    drawn on the GPU (Haar factors from QRs of seeded Gaussians)."""
    import urv_inputs as gen

    rng = gen.generator(1812, 6)
    ms = [int(x) for x in rng.integers(64, 1025, size=512)]
    ns = [int(rng.integers(32, m + 1)) for m in ms]
    A = [gen.spectral_matrix(m, n, gen.spectrum("geometric6", n), 1812 + i, device=device).float().t().contiguous().t()
         for i, (m, n) in enumerate(zip(ms, ns))]
    return ms, ns, A


def bench_batched(steps: int, warmup: int, oracle_sample: int) -> dict:
    """The batched workload: one persistent launch per step, replayed from a graph."""
    import numpy as np
    import torch

    from paper_1812_06007_amd import urv

    q = 1
    ms, ns, A = batched_workload("cuda")
    U, R, V = urv.batch_outputs(ms, ns)
    plan = urv.BatchPlan(ms, ns, q=q, seed=1812)
    plan.set_buffers(A, U, R, V)
    tuned_ms = plan.autotune()
    nb, grid, team = plan.config()
    for _ in range(warmup):
        plan.run(graph=True)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan.run(graph=True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / steps
    fl = sum(standard_flops(m, n, q, "full") for m, n in zip(ms, ns))
    # the largest matrix alone, on one workgroup: the floor of a one-workgroup-per-matrix schedule
    big = int(np.argmax([m * n * n for m, n in zip(ms, ns)]))
    one = urv.BatchPlan([ms[big]], [ns[big]], q=q, seed=1812 + big)
    u1, r1, v1 = urv.batch_outputs([ms[big]], [ns[big]])
    one.set_buffers([A[big]], u1, r1, v1)
    one.set_config(nb, 1, 1)
    one.run()
    torch.cuda.synchronize()
    e0.record(stream)
    one.run()
    e1.record(stream)
    torch.cuda.synchronize()
    big_ms = e0.elapsed_time(e1)
    res = {"workload": "512 FP32 matrices, m ~ U[64,1024], n ~ U[32,m], sigma_j = 10^(-6(j-1)/(n-1)), "
                       "G from seed 1812+i, q=1 FULL; one persistent launch per step, replayed from a graph",
           "dtype": "f32", "ms_per_batch": ms_step, "flops_executed": fl,
           "tflops": fl / (ms_step * 1e-3) / 1e12,
           "frac_fp32_peak": fl / (ms_step * 1e-3) / 1e12 / FP32_MFMA_PEAK_TFLOPS,
           "autotuned": {"nb": nb, "workgroups": grid, "team_max": team, "ms": tuned_ms},
           "largest_matrix_alone": {"m": ms[big], "n": ns[big], "ms": big_ms}}
    one.close()
    plan.close()
    if oracle_sample > 0:
        from oracle import oracle

        oracle.build()
        idx = list(range(0, 512, max(1, 512 // oracle_sample)))[:oracle_sample]
        t0 = time.perf_counter()
        for i in idx:
            A_np = A[i].t().contiguous().t().cpu().double().numpy()
            oracle.urv(A_np, q, seed=1812 + i)
        dt = time.perf_counter() - t0
        fl_s = sum(standard_flops(ms[i], ns[i], q, "full") for i in idx)
        cores = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)) or 1)
        res["cpu_baseline"] = {"value": fl_s / dt / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
                               "seconds": dt,
                               "sample": "FP64 oracle on %d of the 512 matrices (every %dth): %.3e flop"
                                         % (len(idx), 512 // oracle_sample, fl_s)}
    return res


def bench_wide(q: int, variant: str, steps: int, warmup: int) -> dict:
    """m < n (a ULV of A^T, transposed): A 4000 x 8000 against the tall
    factorisation of the same A^T (8000 x 4000), same spectrum (1/j^2), FP64."""
    import torch

    import urv_inputs as gen
    from paper_1812_06007_amd import urv

    m, n = 4000, 8000
    dev = torch.device("cuda:0")
    B = gen.spectral_matrix(n, m, gen.spectrum("poly2", m), seed=1812, device=dev)  # tall, n x m
    A = B.contiguous().t()  # its transpose: m x n, column-major (row-major copy of B, transposed view)
    out_w = (urv.empty_colmajor(m, m, device=dev), urv.empty_colmajor(m, m, device=dev),
             urv.empty_colmajor(n, m, device=dev))
    out_t = (urv.empty_colmajor(n, m, device=dev), urv.empty_colmajor(m, m, device=dev),
             urv.empty_colmajor(m, m, device=dev))
    ms_w = time_factor(A, q, variant, "fp64", steps, warmup, out_w)
    ms_t = time_factor(B, q, variant, "fp64", steps, warmup, out_t)
    met = urv.metrics(A, *out_w)
    # the tall problem of A^T, plus the m x m QR of its R with reversed columns, whose reflectors
    # are applied to the tall problem's n x m U (the cost of the n x m x m product)
    fl = standard_flops(n, m, q, variant) + 4.0 / 3.0 * m ** 3 + 2.0 * n * m * m
    return {"workload": "A 4000x8000 = (Q1 diag(1/j^2) Q2^T)^T, FP64 %s q=%d, against the tall 8000x4000 A^T"
                        % (variant.upper(), q),
            "ms": ms_w, "ms_tall_transpose": ms_t, "flops_executed": fl,
            "tflops": fl / (ms_w * 1e-3) / 1e12, "recon": met["recon"], "orthU": met["orthU"],
            "orthV": met["orthV"]}


def time_factor(A, q: int, variant: str, precision: str, steps: int, warmup: int, out) -> float:
    """Mean milliseconds of urv.factor over `steps` runs (HIP events on the current stream)."""
    import torch

    from paper_1812_06007_amd import urv

    m, n = A.shape
    ws = torch.empty(urv.workspace_size(m, n, q, variant, precision), dtype=torch.uint8, device=A.device)
    for _ in range(warmup):
        urv.factor(A, q, seed=1812, variant=variant, precision=precision, workspace=ws, out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        urv.factor(A, q, seed=1812, variant=variant, precision=precision, workspace=ws, out=out, check=False)
    e1.record(stream)
    torch.cuda.synchronize()
    urv.sync_status()
    return e0.elapsed_time(e1) / steps


def compare_precisions(A, q: int, variant: str, ms64: float, met64: dict, steps: int, out64,
                       half_too: bool = True) -> dict:
    """The mixed-precision forms against the FP64 run (time, reconstruction,
    orthogonality, rank-k errors and the diagonal of R) on the same A and G,
    for the variant timed and, with half_too, for HALF as well (one QR per
    power step: at q = 2 the FULL mixed form runs five QRs, three of them FP32,
    like the five FP64 ones)."""
    import numpy as np
    import torch

    from paper_1812_06007_amd import urv

    m, n = A.shape
    na = met64["normA"]
    ek64 = met64["ek"]
    d64 = torch.diagonal(out64[1]).abs().cpu().numpy()
    keep = ek64[:-1] > 1e-3 * na  # rank-k errors that rise above FP32-level noise
    res = {"fp64": {"ms": ms64, "recon": met64["recon"], "orthU": met64["orthU"], "orthV": met64["orthV"]}}
    runs = [(variant, prec, prec) for prec in ("mixed_bf16", "mixed_fp16")]
    if half_too and variant != "half":
        out = (urv.empty_colmajor(m, n, device=A.device), urv.empty_colmajor(n, n, device=A.device),
               urv.empty_colmajor(n, n, device=A.device))
        ms = time_factor(A, q, "half", "fp64", steps, 1, out)
        met = urv.metrics(A, *out)
        res["fp64_half"] = {"ms": ms, "recon": met["recon"], "orthU": met["orthU"], "orthV": met["orthV"],
                            "speedup_vs_fp64": ms64 / ms}
        del out
        runs += [("half", prec, prec + "_half") for prec in ("mixed_bf16", "mixed_fp16")]
    for var, prec, key in runs:
        out = (urv.empty_colmajor(m, n, device=A.device), urv.empty_colmajor(n, n, device=A.device),
               urv.empty_colmajor(n, n, device=A.device))
        ms = time_factor(A, q, var, prec, steps, 1, out)
        met = urv.metrics(A, *out)
        ek = met["ek"]
        ratio = ek[:-1][keep] / ek64[:-1][keep]
        d = torch.diagonal(out[1]).abs().cpu().numpy()
        res[key] = {"ms": ms, "speedup_vs_fp64": ms64 / ms, "recon": met["recon"], "orthU": met["orthU"],
                     "orthV": met["orthV"],
                     "ek_ratio_max": float(ratio.max()) if ratio.size else None,
                     "ek_ratio_at_k_n8": float(ek[n // 8] / ek64[n // 8]) if ek64[n // 8] > 0 else None,
                     "diagR_maxdiff_rel_normA": float(np.max(np.abs(d - d64)) / na)}
        if var == "half" and "fp64_half" in res:
            res[key]["speedup_vs_fp64_half"] = res["fp64_half"]["ms"] / ms
        del out
    return res


KERNEL_NAMES = {
    "panel": "cqr_panel_kernel<double> (128-column QR panel; applies the previous block first)",
    "gemm_nn": "gemm_kernel<double,NN> (every FP64 NN launch: A V and the trailing updates)",
    "gemm_tn": "gemm_kernel<double,TN> (every FP64 TN launch: Y^T C of the updates)",
    "gemm_nt": "gemm_kernel<double,NT> (every FP64 NT launch: the reflectors applied to targets)",
    "gemm_tt": "gemm_kernel<double,TT>",
}


def live_roofline(classes: dict, steps: int, workload: tuple) -> dict:
    """The dominant kernel of the timed steps (most summed time among the library's FP64
    launch classes, timed live with HIP events on the streams they run on): its algorithmic
    flops per launch over its mean launch time, against the FP64 MFMA peak; its HBM bytes
    per launch from the committed counter summary (None if that is stale)."""
    cls = max(classes, key=lambda c: classes[c]["ms"])
    v = classes[cls]
    n = max(v["launches"], 1)
    launch_ms = v["ms"] / n
    achieved = v["flops"] / n / (launch_ms * 1e-3) / 1e12 if launch_ms > 0 else 0.0
    return {"bound": "mfma", "kernel": KERNEL_NAMES[cls], "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP64_MFMA_PEAK_TFLOPS, "traffic": class_traffic(cls, *workload),
            "launch_ms": launch_ms, "flop_per_launch": v["flops"] / n, "launches_per_step": v["launches"] / steps,
            "ms_per_step": v["ms"] / steps}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=8000)
    ap.add_argument("--m", type=int, default=0, help="rows (default n)")
    ap.add_argument("--q", type=int, default=2)
    ap.add_argument("--variant", default="full", choices=["full", "half", "none"])
    ap.add_argument("--cpu-sample", type=int, default=3600, help="n of the oracle sample (0: skip)")
    ap.add_argument("--gemm-reps", type=int, default=5)
    ap.add_argument("--mixed-steps", type=int, default=3, help="timed steps per mixed comparison (0: skip)")
    ap.add_argument("--wide-steps", type=int, default=3,
                    help="timed steps of the m < n workload, 4000x8000 (0: skip)")
    ap.add_argument("--grad-steps", type=int, default=5,
                    help="timed steps of the differentiation workload (0: skip)")
    ap.add_argument("--grad-only", action="store_true",
                    help="run only the differentiation workload (for profiling) and exit")
    ap.add_argument("--batched-steps", type=int, default=5,
                    help="timed launches of the batched workload (0: skip)")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched workload (for profiling) and exit")
    ap.add_argument("--gemm-only", action="store_true",
                    help="run only the A V GEMM launches (for counter collection) and exit")
    ap.add_argument("--factor-only", action="store_true",
                    help="run only two factorisations of a Gaussian A of the bench's shape (for counter "
                         "collection: no input construction through torch) and exit")
    ap.add_argument("--no-live-timing", action="store_true",
                    help="do not bracket the library's launches with HIP events during the timed steps")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only plain 1 GiB device copies (counter calibration) and exit")
    ap.add_argument("--gemm-source-hash", action="store_true",
                    help="print the hash the traffic summary is keyed on and exit")
    ap.add_argument("--pipeline-source-hash", action="store_true",
                    help="print the hash the per-class traffic summary is keyed on and exit")
    args = ap.parse_args()
    if args.gemm_source_hash:
        print(gemm_source_hash())
        return 0
    if args.pipeline_source_hash:
        print(source_hash(PIPELINE_SOURCES))
        return 0

    if args.gpus != 1:
        print("bench.py: only one GPU is supported (--gpus 1); a layout over several GPUs is designed "
              "but not implemented", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import urv_inputs as gen
    from paper_1812_06007_amd import urv

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    n = args.n
    m = args.m or n
    q = args.q
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] 3 copies of 1 GiB done", file=sys.stderr, flush=True)
        return 0

    if args.batched_only:
        print("[bench] batched workload only", file=sys.stderr, flush=True)
        print(json.dumps(bench_batched(max(args.batched_steps, 1), args.warmup, 0)))
        return 0

    if args.grad_only:
        print("[bench] differentiation workload only", file=sys.stderr, flush=True)
        print(json.dumps(bench_grad(max(args.grad_steps, 1), args.warmup, False)))
        return 0

    if args.factor_only:
        # the factorisation itself, on an input that needs no QR of torch's to build
        A = urv.gaussian(m, n, seed=1812, stream_id=5)
        U, R, V = urv.empty_colmajor(m, n, device=dev), urv.empty_colmajor(n, n, device=dev), \
            urv.empty_colmajor(n, n, device=dev)
        ws = torch.empty(urv.workspace_size(m, n, q, args.variant), dtype=torch.uint8, device=dev)
        for _ in range(2):
            urv.factor(A, q, seed=1812, variant=args.variant, workspace=ws, out=(U, R, V))
        torch.cuda.synchronize()
        print("[bench] 2 factorisations (%s, %dx%d, q=%d) done" % (args.variant, m, n, q), file=sys.stderr, flush=True)
        return 0

    if args.gemm_only:
        # any A of the shape will do for the counters; torch's own QR is kept out of the profiled run
        A = urv.gaussian(m, n, seed=1812, stream_id=5)
        X = urv.empty_colmajor(m, n, device=dev)
        Vg = urv.gaussian(n, n, seed=1812)
        for _ in range(args.gemm_reps):
            urv.dgemm(A, Vg, C=X)
        torch.cuda.synchronize()
        print("[bench] %d launches of the %dx%dx%d FP64 GEMM done" % (args.gemm_reps, m, n, n),
              file=sys.stderr, flush=True)
        return 0

    print("[bench] generating A %dx%d (sigma_j = 1/j^2) on the GPU" % (m, n), file=sys.stderr, flush=True)
    sigma = gen.spectrum("poly2", n)
    A = gen.spectral_matrix(m, n, sigma, seed=1812, device=dev)
    U = urv.empty_colmajor(m, n, device=dev)
    R = urv.empty_colmajor(n, n, device=dev)
    V = urv.empty_colmajor(n, n, device=dev)
    ws = torch.empty(urv.workspace_size(m, n, q, args.variant), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def step():
        # asynchronous: the expired-wait status is read once after the timed steps
        urv.factor(A, q, seed=1812, variant=args.variant, workspace=ws, out=(U, R, V), check=False)

    print("[bench] warmup %d" % args.warmup, file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    print("[bench] timing %d steps" % args.steps, file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps - 1)]
    e0.record(stream)
    for i in range(args.steps):
        step()
        if i + 1 < args.steps:
            marks[i].record(stream)  # per-step boundaries, for the spread of the step times
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    bounds = [e0] + marks + [e1]
    step_ms = sorted(bounds[i].elapsed_time(bounds[i + 1]) for i in range(args.steps))
    urv.sync_status()  # raises if a panel's device-side wait expired in the timed steps
    classes = None
    if not args.no_live_timing:
        # The same steps again with every FP64 launch of the library bracketed by HIP events
        # on the stream it runs on (the host-side event records slow a step by a few per
        # cent, so `value` comes from the steps above): per-class time, launches, flops.
        print("[bench] %d steps with launch timing" % args.steps, file=sys.stderr, flush=True)
        urv.timing(True)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        urv.timing(False)
        urv.sync_status()
        classes = {c: urv.timing_read(c) for c in urv.TIMED_CLASSES}

    met = urv.metrics(A, U, R, V)
    fl_std = standard_flops(m, n, q, args.variant)
    fl = executed_flops(m, n, q, args.variant)
    tflops = fl_std / (ms * 1e-3) / 1e12

    # Dominant kernel: the FP64 MFMA GEMM X = A V (2 m n^2 flop per launch), timed alone on the
    # same stream with HIP events, same shapes and leading dimensions as inside the step.
    X = urv.empty_colmajor(m, n, device=dev)
    urv.dgemm(A, V, C=X)
    torch.cuda.synchronize()
    g0 = torch.cuda.Event(enable_timing=True)
    g1 = torch.cuda.Event(enable_timing=True)
    g0.record(stream)
    for _ in range(args.gemm_reps):
        urv.dgemm(A, V, C=X)
    g1.record(stream)
    torch.cuda.synchronize()
    gemm_ms = g0.elapsed_time(g1) / args.gemm_reps
    gemm_tf = 2.0 * m * n * n / (gemm_ms * 1e-3) / 1e12
    del X

    mixed = None
    if args.mixed_steps > 0:
        mixed = {"n8000": compare_precisions(A, q, args.variant, ms, met, args.mixed_steps, (U, R, V)),
                 "c3": None}
        del ws
        print("[bench] mixed vs FP64 on the 16000x8000 noisy exp(-j/800) matrix", file=sys.stderr, flush=True)
        m3, n3 = 16000, 8000
        A3 = gen.noisy_spectral_matrix(m3, n3, gen.spectrum("exp800", n3), seed=1812, noise_var=1e-6,
                                       device=dev).float().double()
        out3 = (urv.empty_colmajor(m3, n3, device=dev), urv.empty_colmajor(n3, n3, device=dev),
                urv.empty_colmajor(n3, n3, device=dev))
        ms3 = time_factor(A3, q, args.variant, "fp64", max(1, args.mixed_steps - 1), 1, out3)
        met3 = urv.metrics(A3, *out3)
        mixed["c3"] = compare_precisions(A3, q, args.variant, ms3, met3, max(1, args.mixed_steps - 1), out3)
        mixed["c3"]["workload"] = ("A 16000x8000 = Q1 diag(exp(-j/800)) Q2^T + N(0, 1e-6) noise, "
                                   "rounded to FP32 values")
        del A3, out3
        torch.cuda.empty_cache()

    wide = None
    if args.wide_steps > 0:
        print("[bench] m < n: 4000x8000 against its tall transpose", file=sys.stderr, flush=True)
        wide = bench_wide(q, args.variant, args.wide_steps, 1)
        torch.cuda.empty_cache()

    grad = None
    if args.grad_steps > 0:
        print("[bench] differentiation workload (2048x2048 FP32, q=2, k=256)", file=sys.stderr, flush=True)
        grad = bench_grad(args.grad_steps, args.warmup, args.cpu_sample > 0)

    batched = None
    if args.batched_steps > 0:
        print("[bench] batched workload (512 FP32 matrices up to 1024 x 1024, q=1)", file=sys.stderr, flush=True)
        batched = bench_batched(args.batched_steps, args.warmup, 16 if args.cpu_sample > 0 else 0)

    cpu = None
    if args.cpu_sample > 0:
        print("[bench] oracle CPU baseline on a %dx%d sample" % (args.cpu_sample, args.cpu_sample),
              file=sys.stderr, flush=True)
        cpu = cpu_baseline(q, args.variant, args.cpu_sample)

    out = {
        "metric": METRIC,
        "value": tflops,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "PowerURV FP64 %s, A %dx%d = Q1 diag(1/j^2) Q2^T (Haar Q1, Q2), q=%d, G from seed 1812"
                               % (args.variant.upper(), m, n, q),
                   "m": m, "n": n, "q": q, "variant": args.variant, "precision": "fp64"},
        "flops_standard": fl_std,
        "flops_executed": fl,
        "tflops_executed": fl / (ms * 1e-3) / 1e12,
        "flops_paper_table1": paper_flops(m, n, q),
        "tflops_at_paper_count": paper_flops(m, n, q) / (ms * 1e-3) / 1e12,
        "frac_fp64_peak": tflops / FP64_MFMA_PEAK_TFLOPS,
        "recon": met["recon"],
        "orthU": met["orthU"],
        "orthV": met["orthV"],
        "wall_s_timed": wall,
        "step_ms": {"median": step_ms[len(step_ms) // 2] if len(step_ms) % 2 else
                    0.5 * (step_ms[len(step_ms) // 2 - 1] + step_ms[len(step_ms) // 2]),
                    "min": step_ms[0], "max": step_ms[-1]},
        "roofline": live_roofline(classes, args.steps, (m, n, q, args.variant)) if classes else None,
        "roofline_classes": None if not classes else
        {c: dict(v, frac=(v["flops"] / (v["ms"] * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS) if v["ms"] else None,
                 ms_per_step=v["ms"] / args.steps) for c, v in classes.items()},
        "gemm_av": {"bound": "mfma", "kernel": "gemm_kernel<double,NN,128x128,4x4 waves> (X = A V alone)",
                    "achieved": gemm_tf, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": gemm_tf / FP64_MFMA_PEAK_TFLOPS, "traffic": gemm_traffic(m, n),
                    "launch_ms": gemm_ms, "flop_per_launch": 2.0 * m * n * n},
        "mixed_vs_fp64": mixed,
        "m_lt_n": wide,
        "differentiation": grad,
        "batched": batched,
        "cpu_baseline": None if cpu is None else {k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample")},
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
