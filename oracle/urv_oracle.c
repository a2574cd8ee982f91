/*
 * urv_oracle.c -- TEST INFRASTRUCTURE ONLY: plain, slow FP64 CPU reference of
 * PowerURV (Gopal & Martinsson, arXiv:1812.06007).  Not part of the product
 * path; only tests, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * Every routine is written for a reader to check against the paper by eye:
 * unblocked Householder QR, triple-loop products, the driver in the order of
 * eqs. (power) and (powerqr).  OpenMP only splits independent columns; each
 * scalar result is one sequential sum, so results do not depend on the thread
 * count.  Build with -O2 -ffp-contract=off (no fused multiply-add, no
 * fast-math) so that every product and sum is rounded as written.
 */
#include "urv_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static int g_descending = 0;

void orc_set_sum_order(int descending) { g_descending = descending ? 1 : 0; }

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon et al., "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11): ten rounds of two 64x64->128 multiplications; the key is bumped by
 * the Weyl constants before every round but the first. */
#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL /* golden ratio */
#define PHILOX_W1 0xBB67AE8584CAA73BULL /* sqrt(3) - 1 */

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * x0;
    unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    x0 = hi1 ^ x1 ^ k0;
    x1 = lo1;
    x2 = hi0 ^ x3 ^ k1;
    x3 = lo0;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* u in (0,1): the top 53 bits, offset by half a unit so 0 is never hit. */
static double to_unit(uint64_t w) { return ((double)(w >> 11) + 0.5) * 0x1p-53; }

void orc_gaussian(double* G, int64_t rows, int64_t cols, int64_t ld,
                  uint64_t seed, uint32_t stream_id) {
  if (rows <= 0 || cols <= 0) return;
  const int64_t total = rows * cols;
  const int64_t nblocks = (total + 3) / 4;
  const double two_pi = 6.28318530717958647692528676655900577; /* 2 pi */
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nblocks; ++b) {
    uint64_t ctr[4] = {(uint64_t)b, (uint64_t)stream_id, 0, 0};
    uint64_t key[2] = {seed, 0};
    uint64_t w[4];
    orc_philox4x64_10(ctr, key, w);
    double z[4];
    for (int pair = 0; pair < 2; ++pair) {
      double ua = to_unit(w[2 * pair]);
      double ub = to_unit(w[2 * pair + 1]);
      double radius = sqrt(-2.0 * log(ua));
      double angle = two_pi * ub;
      z[2 * pair] = radius * cos(angle);
      z[2 * pair + 1] = radius * sin(angle);
    }
    for (int lane = 0; lane < 4; ++lane) {
      int64_t l = 4 * b + lane;
      if (l < total) {
        int64_t i = l % rows, j = l / rows;
        G[i + j * ld] = z[lane];
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Matrix products: plain sums over k. */
static double op_at(const double* X, int64_t ld, int trans, int64_t r, int64_t c) {
  return trans ? X[c + r * ld] : X[r + c * ld];
}

void orc_gemm(int transA, int transB, int64_t M, int64_t N, int64_t K,
              double alpha, const double* A, int64_t lda,
              const double* B, int64_t ldb, double beta, double* C, int64_t ldc) {
  if (M <= 0 || N <= 0) return;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < N; ++j) {
    double* acc = (double*)calloc((size_t)M, sizeof(double));
    if (!acc) abort();
    if (!transA) {
      /* column form: acc(:) += A(:,k) * opB(k,j), k in the chosen order */
      for (int64_t t = 0; t < K; ++t) {
        int64_t k = g_descending ? K - 1 - t : t;
        double b = op_at(B, ldb, transB, k, j);
        const double* a = A + k * lda;
        for (int64_t i = 0; i < M; ++i) acc[i] += a[i] * b;
      }
    } else {
      /* dot-product form: acc(i) = sum_k A(k,i) * opB(k,j) */
      for (int64_t i = 0; i < M; ++i) {
        double s = 0.0;
        const double* a = A + i * lda;
        for (int64_t t = 0; t < K; ++t) {
          int64_t k = g_descending ? K - 1 - t : t;
          s += a[k] * op_at(B, ldb, transB, k, j);
        }
        acc[i] = s;
      }
    }
    for (int64_t i = 0; i < M; ++i) {
      double v = alpha * acc[i];
      C[i + j * ldc] = (beta == 0.0) ? v : v + beta * C[i + j * ldc];
    }
    free(acc);
  }
}

/* ------------------------------------------------------------------------ */
/* Householder QR, one column at a time (Golub & Van Loan, Matrix Computations,
 * Householder QR; Trefethen & Bau, Lecture 10).
 *
 * Column j: x = X(j:m-1, j), alpha = x(0), sigma2 = sum_{i>0} x(i)^2.
 *   sigma2 == 0: tau = 0 (H = I; input already triangular there stays exact).
 *   else: beta = -sgn(alpha) * sqrt(alpha^2 + sigma2), sgn(0) = +1,
 *         v = x / (alpha - beta) with v(0) = 1, tau = (beta - alpha) / beta,
 *         so that (I - tau v v^T) x = beta e_1.
 * v(1:) is stored below the diagonal of X, beta on the diagonal. */

static double sum_sq_below(const double* col, int64_t from, int64_t to) {
  double s = 0.0;
  for (int64_t t = from; t < to; ++t) {
    int64_t i = g_descending ? to - 1 - (t - from) : t;
    s += col[i] * col[i];
  }
  return s;
}

/* y(j:m-1) <- (I - tau v v^T) y(j:m-1), v(0) = 1 implicit, v(1:) = vcol(j+1:). */
static void apply_reflector(const double* vcol, double tau, int64_t j, int64_t m, double* y) {
  if (tau == 0.0) return;
  double s = y[j];
  for (int64_t t = j + 1; t < m; ++t) {
    int64_t i = g_descending ? m - 1 - (t - j - 1) : t;
    s += vcol[i] * y[i];
  }
  double w = tau * s;
  y[j] -= w;
  for (int64_t i = j + 1; i < m; ++i) y[i] -= w * vcol[i];
}

int orc_qr_pos(double* X, int64_t m, int64_t n, int64_t ldx,
               double* Q, int64_t ldq, double* R, int64_t ldr) {
  if (n < 0 || m < n || ldx < (m > 1 ? m : 1)) return -1;
  if (n == 0) return 0;
  double* tau = (double*)malloc((size_t)n * sizeof(double));
  if (!tau) return -1;

  for (int64_t j = 0; j < n; ++j) {
    double* x = X + j * ldx;
    double alpha = x[j];
    double sigma2 = sum_sq_below(x, j + 1, m);
    if (sigma2 == 0.0) {
      tau[j] = 0.0;
    } else {
      double norm = sqrt(alpha * alpha + sigma2);
      double beta = (alpha >= 0.0) ? -norm : norm;
      double denom = alpha - beta;
      for (int64_t i = j + 1; i < m; ++i) x[i] = x[i] / denom;
      tau[j] = (beta - alpha) / beta;
      x[j] = beta;
    }
#pragma omp parallel for schedule(static)
    for (int64_t c = j + 1; c < n; ++c) apply_reflector(x, tau[j], j, m, X + c * ldx);
  }

  /* D = diag(sgn R(j,j)), sgn(0) = +1: R <- D R, Q <- Q D. */
  if (R) {
    for (int64_t c = 0; c < n; ++c)
      for (int64_t i = 0; i < n; ++i) {
        double d = (X[i + i * ldx] < 0.0) ? -1.0 : 1.0;
        R[i + c * ldr] = (i <= c) ? d * X[i + c * ldx] : 0.0;
      }
  }
  if (Q) {
    /* Q = H_0 H_1 ... H_{n-1} [I_n; 0], accumulated from the last reflector
     * back to the first; H_j only touches rows j.. of columns j.. at its turn. */
    for (int64_t c = 0; c < n; ++c)
      for (int64_t i = 0; i < m; ++i) Q[i + c * ldq] = (i == c) ? 1.0 : 0.0;
    for (int64_t j = n - 1; j >= 0; --j) {
      const double* v = X + j * ldx;
#pragma omp parallel for schedule(static)
      for (int64_t c = j; c < n; ++c) apply_reflector(v, tau[j], j, m, Q + c * ldq);
    }
    for (int64_t c = 0; c < n; ++c) {
      if (X[c + c * ldx] < 0.0)
        for (int64_t i = 0; i < m; ++i) Q[i + c * ldq] = -Q[i + c * ldq];
    }
  }
  free(tau);
  return 0;
}

/* ------------------------------------------------------------------------ */
static double* alloc_mat(int64_t rows, int64_t cols) {
  return (double*)malloc((size_t)(rows > 0 ? rows : 1) * (size_t)(cols > 0 ? cols : 1) * sizeof(double));
}

static void copy_mat(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows, int64_t cols) {
  for (int64_t j = 0; j < cols; ++j) memcpy(dst + j * ldd, src + j * lds, (size_t)rows * sizeof(double));
}

/* V <- Qpos(V) for an n x n V (packed). Work: scratch n x n. */
static int orthonormalize_square(double* V, int64_t n, double* scratch) {
  memcpy(scratch, V, (size_t)n * n * sizeof(double));
  return orc_qr_pos(scratch, n, n, n, V, n, NULL, 0);
}

/* The power steps of eq. (power) for a tall A (m x n, m >= n): Vw (n x n,
 * packed) = V after q steps from G (or the Gaussian of seed, stream 2).
 * X and W (m x n) and S (m x n) are scratch. */
static void power_steps(const double* A, int64_t m, int64_t n, int64_t lda, int32_t q,
                        uint64_t seed, const double* G, int64_t ldg, int32_t variant,
                        int32_t orth_g, double* Vw, double* X, double* W, double* S) {
  /* Starting matrix: the Gaussian G of eq. (power). */
  if (G) copy_mat(G, ldg, Vw, n, n, n);
  else orc_gaussian(Vw, n, n, n, seed, 2u);
  if (q == 0 || orth_g) orthonormalize_square(Vw, n, S);

  for (int32_t t = 0; t < q; ++t) {
    orc_gemm(0, 0, m, n, n, 1.0, A, lda, Vw, n, 0.0, X, m);          /* X = A V   */
    if (variant == ORC_FULL) {
      memcpy(S, X, (size_t)m * n * sizeof(double));
      orc_qr_pos(S, m, n, m, W, m, NULL, 0);                         /* W = Qpos(X) */
      orc_gemm(1, 0, n, n, m, 1.0, A, lda, W, m, 0.0, Vw, n);        /* Y = A^T W */
      orthonormalize_square(Vw, n, S);                               /* V = Qpos(Y) */
    } else if (variant == ORC_HALF) {
      orc_gemm(1, 0, n, n, m, 1.0, A, lda, X, m, 0.0, Vw, n);        /* Y = A^T X */
      orthonormalize_square(Vw, n, S);
    } else {
      orc_gemm(1, 0, n, n, m, 1.0, A, lda, X, m, 0.0, Vw, n);        /* V = A^T A V */
    }
  }
  if (variant == ORC_NONE && q > 0) orthonormalize_square(Vw, n, S); /* (A^T A)^q G = V Z */
}

int orc_urv(const double* A, int64_t m, int64_t n, int64_t lda, int32_t q,
            uint64_t seed, const double* G, int64_t ldg, int32_t variant,
            int32_t orth_g, double* U, int64_t ldu, double* R, int64_t ldr,
            double* V, int64_t ldv) {
  if (m < 0 || n < 0 || q < 0 || variant < 0 || variant > 2) return -1;
  const int64_t p = m < n ? m : n;
  if (p == 0) return 0;
  if (lda < m || ldu < m || ldr < p || ldv < n || (G && ldg < p)) return -1;

  /* m < n (Section 1): a ULV of B = A^T, transposed.  The rows and columns of
   * the tall problem are (mt, nt) = (n, m). */
  const int wide = m < n;
  const int64_t mt = wide ? n : m, nt = p;
  double* B = NULL;
  if (wide) {
    B = alloc_mat(n, m);
    if (!B) return -1;
    for (int64_t j = 0; j < m; ++j)
      for (int64_t i = 0; i < n; ++i) B[i + j * n] = A[j + i * lda];
  }
  const double* At = wide ? B : A;
  const int64_t ldat = wide ? n : lda;

  double* Vw = alloc_mat(nt, nt);  /* current V, packed nt x nt */
  double* X = alloc_mat(mt, nt);   /* A V, packed mt x nt */
  double* W = alloc_mat(mt, nt);   /* Qpos(A V), packed */
  double* S = alloc_mat(mt, nt);   /* scratch for QR */
  double* Up = alloc_mat(mt, nt);
  double* Rp = alloc_mat(nt, nt);
  if (!Vw || !X || !W || !S || !Up || !Rp) {
    free(B); free(Vw); free(X); free(W); free(S); free(Up); free(Rp);
    return -1;
  }
  power_steps(At, mt, nt, ldat, q, seed, G, ldg, variant, orth_g, Vw, X, W, S);
  orc_gemm(0, 0, mt, nt, nt, 1.0, At, ldat, Vw, nt, 0.0, X, mt);    /* X = A V */
  if (!wide) {
    /* eq. (powerqr): A V = U R. */
    orc_qr_pos(X, mt, nt, mt, Up, mt, Rp, nt);
    copy_mat(Up, mt, U, ldu, m, n);
    copy_mat(Rp, nt, R, ldr, n, n);
    copy_mat(Vw, nt, V, ldv, n, n);
  } else {
    /* B V = X, and X J = Q R' with J the reversal of the p columns, so
     * B = (Q J)(J R' J) V^T with J R' J lower triangular (a ULV of B) and
     * A = B^T = V (J R' J)^T (Q J)^T: U = V (m x m), R = J R'^T J (upper,
     * R(i,j) = R'(p-1-j, p-1-i)), V = Q J (n x m). */
    for (int64_t j = 0; j < p; ++j) memcpy(S + j * mt, X + (p - 1 - j) * mt, (size_t)mt * sizeof(double));
    orc_qr_pos(S, mt, p, mt, Up, mt, Rp, p);
    copy_mat(Vw, p, U, ldu, m, m);
    for (int64_t j = 0; j < p; ++j)
      for (int64_t i = 0; i < p; ++i) R[i + j * ldr] = Rp[(p - 1 - j) + (p - 1 - i) * p];
    for (int64_t j = 0; j < p; ++j) memcpy(V + j * ldv, Up + (p - 1 - j) * mt, (size_t)mt * sizeof(double));
  }
  free(B); free(Up); free(Rp);
  free(Vw); free(X); free(W); free(S);
  return 0;
}

/* ------------------------------------------------------------------------ */
static double frob(const double* X, int64_t rows, int64_t cols, int64_t ld) {
  double s = 0.0;
  for (int64_t j = 0; j < cols; ++j)
    for (int64_t i = 0; i < rows; ++i) s += X[i + j * ld] * X[i + j * ld];
  return sqrt(s);
}

int orc_metrics(const double* A, int64_t m, int64_t n, int64_t lda,
                const double* U, int64_t ldu, const double* R, int64_t ldr,
                const double* V, int64_t ldv, double out[4], double* ek) {
  const int64_t p = m < n ? m : n;  /* U m x p, R p x p, V n x p */
  if (p <= 0) return -1;
  double* UR = alloc_mat(m, p);
  double* E = alloc_mat(m, n);
  double* Gm = alloc_mat(p, p);
  if (!UR || !E || !Gm) { free(UR); free(E); free(Gm); return -1; }

  /* recon: A - (U R) V^T */
  orc_gemm(0, 0, m, p, p, 1.0, U, ldu, R, ldr, 0.0, UR, m);
  copy_mat(A, lda, E, m, m, n);
  orc_gemm(0, 1, m, n, p, -1.0, UR, m, V, ldv, 1.0, E, m);
  double normA = frob(A, m, n, lda);
  out[0] = frob(E, m, n, m) / normA;
  out[3] = normA;

  orc_gemm(1, 0, p, p, m, 1.0, U, ldu, U, ldu, 0.0, Gm, p);
  for (int64_t i = 0; i < p; ++i) Gm[i + i * p] -= 1.0;
  out[1] = frob(Gm, p, p, p);
  orc_gemm(1, 0, p, p, n, 1.0, V, ldv, V, ldv, 0.0, Gm, p);
  for (int64_t i = 0; i < p; ++i) Gm[i + i * p] -= 1.0;
  out[2] = frob(Gm, p, p, p);

  if (ek) {
    /* ek[k]^2 = sum over rows i >= k of sum_{j >= i} R(i,j)^2 (the trailing
     * block R22 of eq. blocks, which is upper triangular). */
    double acc = 0.0;
    ek[p] = 0.0;
    for (int64_t k = p - 1; k >= 0; --k) {
      double row = 0.0;
      for (int64_t j = k; j < p; ++j) row += R[k + j * ldr] * R[k + j * ldr];
      acc += row;
      ek[k] = sqrt(acc);
    }
  }
  free(UR); free(E); free(Gm);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* One-sided Jacobi (Hestenes 1958): rotate column pairs of a copy of A until
 * they are numerically orthogonal; the column norms are then the singular
 * values. */
static int cmp_desc(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x < y) - (x > y);
}

int orc_jacobi_svd(const double* A, int64_t m, int64_t n, int64_t lda,
                   double* sigma, int32_t max_sweeps) {
  if (n <= 0 || m < n || lda < m) return -1;
  double* W = alloc_mat(m, n);
  if (!W) return -1;
  copy_mat(A, lda, W, m, m, n);
  const double eps = 0x1p-52;
  int sweeps = 0, converged = 0;
  while (!converged && sweeps < max_sweeps) {
    converged = 1;
    ++sweeps;
    for (int64_t p = 0; p < n - 1; ++p) {
      for (int64_t r = p + 1; r < n; ++r) {
        double* ap = W + p * m;
        double* ar = W + r * m;
        double alpha = 0.0, beta = 0.0, gamma = 0.0;
        for (int64_t i = 0; i < m; ++i) {
          alpha += ap[i] * ap[i];
          beta += ar[i] * ar[i];
          gamma += ap[i] * ar[i];
        }
        if (gamma == 0.0 || fabs(gamma) <= eps * sqrt(alpha) * sqrt(beta)) continue;
        converged = 0;
        double zeta = (beta - alpha) / (2.0 * gamma);
        double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double c = 1.0 / sqrt(1.0 + t * t);
        double s = c * t;
        for (int64_t i = 0; i < m; ++i) {
          double x = ap[i], y = ar[i];
          ap[i] = c * x - s * y;
          ar[i] = s * x + c * y;
        }
      }
    }
  }
  for (int64_t j = 0; j < n; ++j) sigma[j] = frob(W + j * m, m, 1, m);
  qsort(sigma, (size_t)n, sizeof(double), cmp_desc);
  free(W);
  return converged ? sweeps : -1;
}
