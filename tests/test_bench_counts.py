"""The benchmark's flop accounting and its one-GPU contract (CPU only).

`value` is standard flops / time, so the counts are pinned here against hand
counts written as the list of operations the driver (run_factor) performs,
with the standard LAPACK counts of each: a product with A or A^T 2mn^2; a
Householder QR of an m x n matrix 2mn^2 - (2/3)n^3, and the same for forming
its explicit Q; n x n: (4/3)n^3.  The executed count differs where U, when
m == n, is formed by applying the final QR's reflectors to an identity (2n^3
for n x n); V is formed structurally.  The paper's Table 1 count (leading order, GEMM term 2(2q+1)mn^2)
is pinned too."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _ops(m, n):
    prod = 2.0 * m * n * n
    qr_mn = 2.0 * m * n * n - 2.0 * n ** 3 / 3.0
    qr_nn = 4.0 * n ** 3 / 3.0
    return prod, qr_mn, qr_nn


def _calls(m, n, q, variant):
    """The driver's operations in order (run_factor, final_qr)."""
    prod, qr_mn, qr_nn = _ops(m, n)
    calls = []
    if variant == "none":
        calls += [prod, prod] * q                     # (A^T A)^q G
        calls += [qr_nn] if q > 0 else [qr_nn]        # V = Qpos((A^T A)^q G), or Qpos(G) when q == 0
        calls += [prod]                               # X = A V
    else:
        calls += [qr_nn, prod] if q == 0 else [prod]  # q == 0: V = Qpos(G), X = A V; else X = A G
        for _ in range(q):
            if variant == "full":
                calls += [qr_mn, prod]                # W = Qpos(X), A^T W
            else:
                calls += [prod]                       # A^T X
            calls += [qr_nn, prod]                    # V = Qpos(.), X = A V
    calls += [qr_nn]                                  # V formed
    calls += [qr_mn, qr_mn]                           # A V = U R, U formed
    return calls


@pytest.mark.parametrize("m,n", [(8000, 8000), (16000, 8000), (400, 400), (1200, 600)])
@pytest.mark.parametrize("q", [0, 1, 2, 3])
@pytest.mark.parametrize("variant", ["full", "half", "none"])
def test_standard_flops_by_call_list(bench, m, n, q, variant):
    assert bench.standard_flops(m, n, q, variant) == pytest.approx(sum(_calls(m, n, q, variant)), rel=1e-12)


def test_standard_flops_of_the_bench_config(bench):
    n = 8000.0
    assert bench.standard_flops(8000, 8000, 2, "full") == pytest.approx(58.0 / 3.0 * n ** 3, rel=1e-12)
    assert bench.standard_flops(8000, 8000, 2, "half") == pytest.approx(50.0 / 3.0 * n ** 3, rel=1e-12)
    assert bench.standard_flops(8000, 8000, 2, "full") == pytest.approx(9.898666666666667e12, rel=1e-12)


@pytest.mark.parametrize("m,n,extra", [(8000, 8000, 2.0 - 4.0 / 3.0), (16000, 8000, 0.0)])
def test_executed_flops_identity_targets(bench, m, n, extra):
    """U, when m == n, is formed as the reflectors applied to an identity: 2 n^3 instead
    of 4/3 n^3; V always by the structured formation."""
    for variant in ("full", "half"):
        got = bench.executed_flops(m, n, 2, variant) - bench.standard_flops(m, n, 2, variant)
        assert got == pytest.approx(extra * n ** 3, rel=1e-12, abs=1.0)
    assert bench.executed_flops(8000, 8000, 2, "full") == pytest.approx(60.0 / 3.0 * 8000.0 ** 3, rel=1e-12)


@pytest.mark.parametrize("q,expected", [(0, 1.7066666666666667e12), (1, 5.12e12), (2, 8.533333333333333e12)])
def test_paper_table1_count(bench, q, expected):
    assert bench.paper_flops(8000, 8000, q) == pytest.approx(expected, rel=1e-12)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_class_traffic_follows_the_committed_summary(bench, tmp_path, monkeypatch):
    """roofline.traffic comes from the committed PMC summary only while the factorisation's
    sources hash to the value recorded there, and only for the workload it was taken on."""
    src = tmp_path / "summary.txt"
    h = bench.source_hash(bench.PIPELINE_SOURCES)
    src.write_text("workload: 8000x8000 q=2 full\npipeline_source_sha256: %s\nbytes_per_launch.gemm_nn: 123\n" % h)
    monkeypatch.setattr(bench, "CLASS_TRAFFIC_FILE", str(src))
    assert bench.class_traffic("gemm_nn", 8000, 8000, 2, "full") == 123.0
    assert bench.class_traffic("gemm_nn", 8000, 8000, 2, "half") is None
    assert bench.class_traffic("gemm_tn", 8000, 8000, 2, "full") is None
    src.write_text("workload: 8000x8000 q=2 full\npipeline_source_sha256: %s\nbytes_per_launch.gemm_nn: 123\n" % ("0" * 64))
    assert bench.class_traffic("gemm_nn", 8000, 8000, 2, "full") is None

