/*
 * urv_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU reference for the PowerURV factorization of
 * Gopal & Martinsson, "The PowerURV algorithm for computing rank-revealing
 * full factorizations" (arXiv:1812.06007).  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code,
 * header or constant table with the GPU library (include/urv.h); both sides
 * implement the Gaussian generator separately from its published definition.
 *
 * Conventions: column-major, element (i,j) of a matrix with leading dimension
 * ld is p[i + j*ld]; host pointers; every routine is deterministic for any
 * OpenMP thread count (each dot product is summed in one fixed order).
 */
#ifndef URV_ORACLE_H
#define URV_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Variants of the power iteration (Section 3, paragraph after eq. powerqr). */
enum { ORC_FULL = 0, ORC_HALF = 1, ORC_NONE = 2 };

/* Summation order of every inner product: 0 ascending (default), 1 descending.
 * Used only to measure the oracle's own rounding spread. */
void orc_set_sum_order(int descending);

/* Philox4x64 with 10 rounds (Salmon, Moraes, Dror & Shaw, SC'11). */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Gaussian matrix (Section 3: "Gaussian random matrix G is drawn").
 * Element (i,j) has linear index l = i + j*rows; it is lane l%4 of Philox
 * block b = l/4 with counter (b, stream_id, 0, 0) and key (seed, 0).  The four
 * words w of a block give u = ((w>>11)+0.5)*2^-53 and two Box-Muller pairs
 * (u0,u1) -> sqrt(-2 ln u0) * (cos 2 pi u1, sin 2 pi u1), likewise (u2,u3). */
void orc_gaussian(double* G, int64_t rows, int64_t cols, int64_t ld,
                  uint64_t seed, uint32_t stream_id);

/* C = alpha*op(A)*op(B) + beta*C, op(X) = X or X^T (trans != 0).  C is M x N,
 * op(A) is M x K, op(B) is K x N.  Each entry is one sum over k, in the order
 * set by orc_set_sum_order.  beta == 0 never reads C. */
void orc_gemm(int transA, int transB, int64_t M, int64_t N, int64_t K,
              double alpha, const double* A, int64_t lda,
              const double* B, int64_t ldb, double beta, double* C, int64_t ldc);

/* Unpivoted Householder QR with explicit Q and positive diagonal of R
 * (DDH-URV description in Section 2.2 and its footnote on Haar matrices).
 * X (m x n, m >= n) is overwritten with the reflectors.  Q (m x n) and R
 * (n x n, strictly lower part set to 0) may be NULL when not wanted.
 * Returns 0, or -1 on bad arguments / allocation failure. */
int orc_qr_pos(double* X, int64_t m, int64_t n, int64_t ldx,
               double* Q, int64_t ldq, double* R, int64_t ldr);

/* PowerURV (Section 3, eqs. power and powerqr): A = U R V^T.
 * A m x n is read only; p = min(m, n).  G: p x p starting matrix, or NULL to
 * draw it with orc_gaussian(seed, stream 2).  q >= 0 power steps; variant
 * ORC_FULL re-orthonormalises after every product with A or A^T, ORC_HALF once
 * per A^T A step, ORC_NONE only at the end.  q == 0 or orth_g != 0 starts from
 * V = Qpos(G) (q == 0 is DDH-URV, Section 2.2).  Outputs U (m x p), R (p x p
 * upper, strictly lower part 0), V (n x p).  m < n (Section 1): the tall
 * method runs on B = A^T (n x m) up to X = B V; X with its columns reversed
 * (J) is factored, X J = Q R', and A = V (J R' J)^T (Q J)^T is returned:
 * U = V, R = J R'^T J, V = Q J.  Returns 0 or -1. */
int orc_urv(const double* A, int64_t m, int64_t n, int64_t lda, int32_t q,
            uint64_t seed, const double* G, int64_t ldg, int32_t variant,
            int32_t orth_g, double* U, int64_t ldu, double* R, int64_t ldr,
            double* V, int64_t ldv);

/* Checks of a factorisation (rank-k errors of Section 5, eq. blocks), with
 * p = min(m, n), U m x p, R p x p, V n x p:
 * out[0] = ||A - U R V^T||_F / ||A||_F, out[1] = ||U^T U - I||_F,
 * out[2] = ||V^T V - I||_F, out[3] = ||A||_F; ek (length p+1, may be NULL):
 * ek[k] = ||R(k:p-1, k:p-1)||_F over the upper triangle (0-based). */
int orc_metrics(const double* A, int64_t m, int64_t n, int64_t lda,
                const double* U, int64_t ldu, const double* R, int64_t ldr,
                const double* V, int64_t ldv, double out[4], double* ek);

/* Singular values of A (m x n, m >= n) by one-sided (Hestenes) Jacobi,
 * cyclic sweeps until no pair has |a_p^T a_q| > eps*||a_p||*||a_q||.
 * sigma (length n) is sorted non-increasing.  Returns the number of sweeps,
 * or -1 if max_sweeps was reached / bad arguments. */
int orc_jacobi_svd(const double* A, int64_t m, int64_t n, int64_t lda,
                   double* sigma, int32_t max_sweeps);

#ifdef __cplusplus
}
#endif
#endif
