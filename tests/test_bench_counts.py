"""The benchmark's flop accounting and its one-GPU contract (CPU only).

`value` is executed flops / time, so the counts are pinned here against
independent figures: the standard LAPACK operation counts written out for
the benchmark's shapes (GEMM 2mn^2; QR with explicit Q of an m x n matrix
2(2mn^2 - (2/3)n^3); an n x n QR with Q (8/3)n^3), and the paper's Table 1
count (leading order, GEMM term 2(2q+1)mn^2)."""
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


@pytest.mark.parametrize("m,n,q,variant,expected", [
    (8000, 8000, 2, "full", 1.1946666666666667e13),   # 5 GEMMs 5.12e12 + 3 m x n QRs 4.096e12 + 2 n x n 2.731e12
    (8000, 8000, 2, "half", 9.216e12),
    (8000, 8000, 1, "full", 7.168e12),
    (8000, 8000, 1, "half", 5.802666666666667e12),
    (8000, 8000, 0, "full", 3.754666666666667e12),     # A G, QR of A V, and Qpos(G)
    (400, 400, 2, "full", 1.4933333333333333e9),
    (400, 400, 2, "half", 1.152e9),
    (4000, 4000, 2, "full", 1.4933333333333333e12),    # the Kahan case
])
def test_executed_flops(bench, m, n, q, variant, expected):
    assert bench.executed_flops(m, n, q, variant) == pytest.approx(expected, rel=1e-12)


def test_executed_flops_by_hand(bench):
    m, n, q = 16000, 8000, 2
    gemm = 5 * 2 * m * n * n
    qr_mn = 2 * (2 * m * n * n - 2 * n ** 3 / 3)
    qr_nn = 8 * n ** 3 / 3
    assert bench.executed_flops(m, n, q, "full") == pytest.approx(gemm + 3 * qr_mn + 2 * qr_nn, rel=1e-12)
    assert bench.executed_flops(m, n, q, "half") == pytest.approx(gemm + qr_mn + 2 * qr_nn, rel=1e-12)


@pytest.mark.parametrize("q,expected", [(0, 1.7066666666666667e12), (1, 5.12e12), (2, 8.533333333333333e12)])
def test_paper_table1_count(bench, q, expected):
    assert bench.paper_flops(8000, 8000, q) == pytest.approx(expected, rel=1e-12)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
