"""Planted mistakes: each mutant copy of the oracle must fail the pin suite.

A plausible slip anywhere in the oracle (a dropped term, a wrong sign, index
or operand, a skipped step of the method) has to be caught by the pins in
test_oracle_rng / test_oracle_linalg / test_oracle_urv.  Each mutant is
the oracle source with one textual change, compiled on the CPU into a
temporary library and loaded by a fresh pytest process.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "urv_oracle.c")
PIN_FILES = ["tests/test_oracle_rng.py", "tests/test_oracle_linalg.py", "tests/test_oracle_urv.py"]

# (name, original text, planted text)
MUTANTS = [
    ("philox key bump", "k1 += PHILOX_W1;", "k1 += PHILOX_W0;"),
    ("philox stream word dropped", "{(uint64_t)b, (uint64_t)stream_id, 0, 0}", "{(uint64_t)b, 0, 0, 0}"),
    ("box-muller cos/sin swapped", "z[2 * pair] = radius * cos(angle);", "z[2 * pair] = radius * sin(angle);"),
    ("gemm operand transposed", "double b = op_at(B, ldb, transB, k, j);", "double b = op_at(B, ldb, !transB, k, j);"),
    ("gemm beta term dropped", "v + beta * C[i + j * ldc]", "v"),
    ("householder tau sign", "tau[j] = (beta - alpha) / beta;", "tau[j] = (beta + alpha) / beta;"),
    ("reflector drops v(0) term", "double s = y[j];", "double s = 0.0;"),
    ("reflector update skips a row", "for (int64_t i = j + 1; i < m; ++i) y[i] -= w * vcol[i];",
     "for (int64_t i = j + 2; i < m; ++i) y[i] -= w * vcol[i];"),
    ("R sign normalisation dropped", "double d = (X[i + i * ldx] < 0.0) ? -1.0 : 1.0;", "double d = 1.0;"),
    ("Q sign normalisation dropped", "if (X[c + c * ldx] < 0.0)", "if (0)"),
    ("power step count off by one", "for (int32_t t = 0; t < q; ++t)", "for (int32_t t = 1; t < q; ++t)"),
    ("FULL skips re-orthonormalisation of A V",
     "orc_gemm(1, 0, n, n, m, 1.0, A, lda, W, m, 0.0, Vw, n);        /* Y = A^T W */",
     "orc_gemm(1, 0, n, n, m, 1.0, A, lda, X, m, 0.0, Vw, n);        /* Y = A^T W */"),
    ("final product uses A^T", "orc_gemm(0, 0, mt, nt, nt, 1.0, At, ldat, Vw, nt, 0.0, X, mt);    /* X = A V */",
     "orc_gemm(1, 0, mt, nt, nt, 1.0, At, ldat, Vw, nt, 0.0, X, mt);    /* X = A V */"),
    ("wide: columns of A V not reversed", "memcpy(S + j * mt, X + (p - 1 - j) * mt,", "memcpy(S + j * mt, X + j * mt,"),
    ("wide: R not transposed", "R[i + j * ldr] = Rp[(p - 1 - j) + (p - 1 - i) * p];",
     "R[i + j * ldr] = Rp[(p - 1 - i) + (p - 1 - j) * p];"),
    ("wide: V not reversed", "memcpy(V + j * ldv, Up + (p - 1 - j) * mt,", "memcpy(V + j * ldv, Up + j * mt,"),
    ("q = 0 start not orthonormalised", "if (q == 0 || orth_g) orthonormalize_square", "if (orth_g) orthonormalize_square"),
    ("rank-k error drops the diagonal", "for (int64_t j = k; j < p; ++j) row +=", "for (int64_t j = k + 1; j < p; ++j) row +="),
    ("jacobi rotation sign", "ap[i] = c * x - s * y;", "ap[i] = c * x + s * y;"),
    ("recon not divided by ||A||", "out[0] = frob(E, m, n, m) / normA;", "out[0] = frob(E, m, n, m);"),
    ("recon with V instead of V^T", "orc_gemm(0, 1, m, n, p, -1.0, UR, m, V, ldv, 1.0, E, m);",
     "orc_gemm(0, 0, m, n, p, -1.0, UR, m, V, ldv, 1.0, E, m);"),
    ("orthU without the identity", "Gm[i + i * p] -= 1.0;\n  out[1] = frob", "Gm[i + i * p] -= 0.0;\n  out[1] = frob"),
    ("orthV measured on U", "orc_gemm(1, 0, p, p, n, 1.0, V, ldv, V, ldv, 0.0, Gm, p);",
     "orc_gemm(1, 0, p, p, n, 1.0, U, ldu, U, ldu, 0.0, Gm, p);"),
]


def _run_mutant(mutant, workdir):
    name, old, new = mutant
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor must occur exactly once: %r" % old
    idx = MUTANTS.index(mutant)
    msrc = os.path.join(workdir, "mutant%d.c" % idx)
    with open(msrc, "w") as f:
        f.write(src.replace(old, new))
    lib = os.path.join(workdir, "mutant%d.so" % idx)
    from oracle import oracle as o

    o.compile_library(msrc, lib)
    env = dict(os.environ, URV_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    proc = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PIN_FILES],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, proc.returncode, proc.stdout[-2000:]


def test_every_planted_mistake_is_caught():
    with tempfile.TemporaryDirectory() as d:
        with ThreadPoolExecutor(max_workers=4) as ex:
            results = list(ex.map(lambda m: _run_mutant(m, d), MUTANTS))
    survivors = [(name, out) for name, rc, out in results if rc == 0]
    assert not survivors, "mutants not caught by the pins: %s" % [s[0] for s in survivors]
    # a failing run must be a test failure (1), not a collection/usage error
    for name, rc, out in results:
        assert rc == 1, (name, rc, out)


def test_unmutated_copy_passes(tmp_path):
    """Control: the same procedure on an unchanged copy passes the pins."""
    from oracle import oracle as o

    lib = str(tmp_path / "copy.so")
    o.compile_library(SRC, lib)
    env = dict(os.environ, URV_ORACLE_LIB=lib, OMP_NUM_THREADS="4")
    proc = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           "tests/test_oracle_linalg.py"], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=600)
    assert proc.returncode == 0, proc.stdout[-2000:]
