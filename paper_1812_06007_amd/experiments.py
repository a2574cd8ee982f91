"""The accuracy experiments of Section 5 on the GPU path, synthetic inputs.

    python -m paper_1812_06007_amd.experiments [--q 0 1 2] [--seed 1812]

Matrices 1-3 of Section 5 are A = U D V^T (200 x 160) with Haar U, V and
prescribed diagonals: fast (geometric, spread over n since the printed
(10^-20)^(k-1) underflows), slow (1/k) and S-shaped decay (the tanh read
with 80 in place of n).  Matrix 4 (a boundary integral operator) has no data
here and is left out, as are the comparison methods (QLP, CPQR).  For each
matrix and q the factorisation runs through the library (FP64 FULL; Matrix 2
also without the stabilising re-orthonormalisations, as the paper runs it),
and the rank-k errors e_k = ||A - U(:,1:k) R(1:k,:) V^T||_F = ||R22||_F
(Section 5, eq. blocks) are compared with the optimal ones, which the
prescribed spectrum gives in closed form: sqrt(sum_{j>k} sigma_j^2).  The
singular values of R11 and R22 against sigma_k and sigma_{k+1} (the
rank-revealing bounds of Section 1, shown in the figure of Section 3) are
reported too; those small SVDs are analysis on the host, not part of the path.

The section relating PowerURV to the RSVD is reproduced by `rsvd_comparison`:
Matrix 2, l = 60, q = 0 and 1, both methods from the same G.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

MATRICES = {"matrix1": "fast decay", "matrix2": "slow decay", "matrix3": "S-shaped decay"}


def run(q_values=(0, 1, 2), m: int = 200, n: int = 160, seed: int = 1812, device="cuda") -> dict:
    """Rank-k error ratios and R11/R22 singular value ratios for Matrices 1-3."""
    import torch

    import urv_inputs as gen

    from . import urv

    out = {}
    for name in MATRICES:
        sigma = gen.spectrum(name, n)
        A_np = gen.spectral_matrix(m, n, sigma, seed)
        A = torch.from_numpy(np.ascontiguousarray(A_np.T)).to(device).t()
        opt = np.sqrt(np.concatenate([np.cumsum((sigma ** 2)[::-1])[::-1], [0.0]]))  # opt[k], k = 0..n
        normA = float(np.linalg.norm(A_np))
        keep = opt[1:n] > 1e-13 * normA  # k = 1..n-1 above the FP64 noise floor
        variants = ["full", "none"] if name == "matrix2" else ["full"]
        for variant in variants:
            for q in q_values:
                U, R, V = urv.factor(A, q, seed=seed, variant=variant)
                met = urv.metrics(A, U, R, V)
                ek = met["ek"]
                ratio = ek[1:n][keep] / opt[1:n][keep]
                Rh = R.cpu().numpy()
                ks = [k for k in (10, 20, 40, 80) if k < n and opt[k] > 1e-13 * normA]
                r11 = {k: float(np.linalg.svd(Rh[:k, :k], compute_uv=False)[-1] / sigma[k - 1]) for k in ks}
                r22 = {k: float(np.linalg.svd(Rh[k:, k:], compute_uv=False)[0] / sigma[k]) for k in ks}
                # the figure of Section 3 over every k: sigma_min(R11) against sigma_k and
                # sigma_max(R22) against sigma_{k+1}, where sigma_k is above the FP64 noise floor
                kall = [k for k in range(1, n) if sigma[k - 1] > 1e-13 * sigma[0]]
                p11 = np.array([np.linalg.svd(Rh[:k, :k], compute_uv=False)[-1] / sigma[k - 1] for k in kall])
                p22 = np.array([np.linalg.svd(Rh[k:, k:], compute_uv=False)[0] / sigma[k] for k in kall])
                out["%s/%s/q%d" % (name, variant, q)] = {
                    "matrix": name, "decay": MATRICES[name], "variant": variant, "q": q,
                    "recon": float(met["recon"]), "ek": ek.tolist(), "opt": opt.tolist(),
                    "ratio_max": float(ratio.max()), "ratio_median": float(np.median(ratio)),
                    "sigma_min_R11_over_sigma_k": r11, "norm_R22_over_sigma_k1": r22,
                    "profile_k": kall, "profile_R11": p11.tolist(), "profile_R22": p22.tolist(),
                    "profile_R11_median": float(np.median(p11)), "profile_R22_median": float(np.median(p22))}
    return out


def rsvd_comparison(q_values=(0, 1), l: int = 60, m: int = 200, n: int = 160, seed: int = 1812,
                    device="cuda") -> dict:
    """PowerURV against the RSVD on Matrix 2 with l = 60 (the section relating
    the two; its figures for q = 0 and q = 1).

    The RSVD starts from the first l columns of the same G: Y = A (A^T A)^q G(:, 1:l)
    by the library's GEMMs, Q = Qpos(Y) by its QR, Q^T A = W S Vr^T (an l x n SVD,
    analysis on the host, as the paper's deterministic SVD step), U_rsvd = Q W.
    Reported for k = 1..l: ||A - U_k U_k^T A||_F and ||A - A V_k V_k^T||_F for both
    methods (U_k, V_k the first k columns).  The section's Lemma makes the two
    U-errors equal at k = l (the leading l columns of U and U_rsvd span the same
    space); below l the RSVD, which applies A once more, is closer to the optimum."""
    import torch

    import urv_inputs as gen

    from . import urv

    sigma = gen.spectrum("matrix2", n)
    A_np = gen.spectral_matrix(m, n, sigma, seed)
    A = torch.from_numpy(np.ascontiguousarray(A_np.T)).to(device).t()
    G = urv.gaussian(n, n, seed=seed, device=device)
    normA = float(np.linalg.norm(A_np))
    opt = np.sqrt(np.concatenate([np.cumsum((sigma ** 2)[::-1])[::-1], [0.0]]))
    out = {}
    for q in q_values:
        U, R, V = urv.factor(A, q, G=G)
        Z = G[:, :l].contiguous().t().contiguous().t()
        for _ in range(q):
            Z = urv.dgemm(A, urv.dgemm(A, Z), transA=True)  # A^T (A Z)
        Q, _ = urv.qr_pos(urv.dgemm(A, Z), want_r=False)
        B = urv.dgemm(Q, A, transA=True)                    # Q^T A, l x n
        Wr, _, Vrt = np.linalg.svd(B.cpu().numpy())
        Ur = Q.cpu().numpy() @ Wr[:, :l]
        Vr = Vrt[:l].T
        Uh, Vh = U.cpu().numpy(), V.cpu().numpy()

        def left(Bk, k):
            return float(np.linalg.norm(A_np - Bk[:, :k] @ (Bk[:, :k].T @ A_np)))

        def right(Bk, k):
            return float(np.linalg.norm(A_np - (A_np @ Bk[:, :k]) @ Bk[:, :k].T))

        ks = range(1, l + 1)
        eu = np.array([left(Uh, k) for k in ks])
        er = np.array([left(Ur, k) for k in ks])
        fu = np.array([right(Vh, k) for k in ks])
        fr = np.array([right(Vr, k) for k in ks])
        out["q%d" % q] = {
            "q": q, "l": l, "normA": normA, "opt": opt[1:l + 1].tolist(),
            "powerurv_left": eu.tolist(), "rsvd_left": er.tolist(),
            "powerurv_right": fu.tolist(), "rsvd_right": fr.tolist(),
            "lemma_gap_at_l": abs(eu[-1] - er[-1]) / normA,
            "projector_gap_at_l": float(np.linalg.norm(Uh[:, :l] @ (Uh[:, :l].T @ A_np) - Ur @ (Ur.T @ A_np))) / normA,
            "left_ratio_median_k_lt_l": float(np.median(er[:-1] / eu[:-1])),
            "right_ratio_median_k_lt_l": float(np.median(fr[:-1] / fu[:-1])),
        }
    return out


def rsvd_table(res: dict) -> str:
    lines = ["| q | k = l: PowerURV / RSVD / optimum (left errors, /||A||) | projectors at l | median RSVD/PowerURV, k < l: left, right |",
             "|---|---|---|---|"]
    for key in sorted(res):
        r = res[key]
        na = r["normA"]
        lines.append("| %d | %.6f / %.6f / %.6f | %.1e | %.3f, %.3f |" % (
            r["q"], r["powerurv_left"][-1] / na, r["rsvd_left"][-1] / na, r["opt"][-1] / na,
            r["projector_gap_at_l"], r["left_ratio_median_k_lt_l"], r["right_ratio_median_k_lt_l"]))
    return "\n".join(lines)


def table(res: dict) -> str:
    lines = ["| matrix | variant | q | max_k e_k / e_k^opt | median | sigma_min(R11)/sigma_k at k = 10, 20, 40, 80 "
             "| median over k: sigma_min(R11)/sigma_k, sigma_max(R22)/sigma_{k+1} |",
             "|---|---|---|---|---|---|---|"]
    for key in sorted(res):
        r = res[key]
        r11 = ", ".join("%.3f" % v for v in r["sigma_min_R11_over_sigma_k"].values())
        lines.append("| %s (%s) | %s | %d | %.3f | %.3f | %s | %.3f, %.3f |" % (
            r["matrix"], r["decay"], r["variant"].upper(), r["q"], r["ratio_max"], r["ratio_median"], r11,
            r["profile_R11_median"], r["profile_R22_median"]))
    return "\n".join(lines)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--q", type=int, nargs="+", default=[0, 1, 2])
    ap.add_argument("--seed", type=int, default=1812)
    ap.add_argument("--json", action="store_true", help="print the full results as JSON")
    args = ap.parse_args()
    res = run(tuple(args.q), seed=args.seed)
    rs = rsvd_comparison(seed=args.seed)
    print(json.dumps({"section5": res, "rsvd": rs}) if args.json else table(res) + "\n\n" + rsvd_table(rs))
    return 0


if __name__ == "__main__":
    sys.exit(main())
