/*
 * urv.h -- C ABI of liburv, a gfx950 (MI355X) implementation of the PowerURV
 * rank-revealing factorisation A = U R V^T of Gopal & Martinsson, "The
 * PowerURV algorithm for computing rank-revealing full factorizations"
 * (arXiv:1812.06007).
 *
 * Layout: every matrix is column-major; element (i,j) of a matrix with
 * leading dimension ld lives at p[i + j*ld].  All matrix pointers are DEVICE
 * pointers (memory from hipMalloc or a torch CUDA tensor) unless a comment
 * says host.  The caller allocates and owns every buffer it passes; no
 * pointer is kept after a call returns.  Calls taking a stream are
 * asynchronous on that stream (NULL = the default stream): buffers must stay
 * valid until the stream reaches the end of the call's work.
 *
 * Errors: every entry point returns an int status (urv_status).  Argument
 * checks run on the host before any device work, so a call that returns
 * URV_EINVAL has written nothing.  HIP failures return URV_EDEVICE; the text
 * of the last failure on the calling thread is in urv_last_error().
 * Non-finite inputs propagate (NaN in, NaN out) unless urv_factor_ex is asked
 * to check them (URV_CHECK_FINITE).  The QR's panels wait on each other on the
 * device with a bounded spin; an expired wait poisons the outputs with NaN and
 * raises a per-device status word, which the blocking urv_factor reports and
 * asynchronous callers read with urv_sync_status.
 */
#ifndef URV_H
#define URV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  URV_OK = 0,
  URV_EINVAL = -1,   /* bad argument: null pointer, size, leading dimension, enum, workspace */
  URV_ENOMEM = -2,   /* device allocation failed */
  URV_EDEVICE = -3,  /* HIP runtime error, or a device-side bounded wait expired */
  URV_ENOTSUP = -4,  /* valid but unsupported combination */
  URV_ENONFINITE = -5 /* URV_CHECK_FINITE found a NaN or an infinity in A (nothing written) */
} urv_status;

/* When the power iteration re-orthonormalises (Section 3, paragraph after
 * eq. powerqr: re-orthonormalise after each application of A or A^T). */
typedef enum {
  URV_REORTH_FULL = 0, /* Qpos after every product with A and with A^T (default) */
  URV_REORTH_HALF = 1, /* one Qpos per A^T A step */
  URV_REORTH_NONE = 2  /* (A^T A)^q G then a single Qpos; only for small q and mild spectra */
} urv_variant;

/* Arithmetic of the factorisation.  U, R, V are FP64 in every mode of
 * urv_factor_ex (A is FP64, or FP32 with URV_A_FP32).  URV_FP32 is taken only
 * by the derivative entry points below: urv_factor_ex returns URV_EINVAL for
 * it, since its outputs are FP64 buffers and an all-FP32 factorisation would
 * leave A = U R V^T at about 1e-6 -- the mixed modes already run the power
 * iteration in 16/32 bits and keep the FP64 tail that makes the result exact
 * to FP64 rounding. */
typedef enum {
  URV_FP64 = 0,       /* everything in FP64 */
  URV_FP32 = 1,       /* everything in FP32 (derivative entry points only) */
  URV_MIXED_BF16 = 2, /* power-step products on BF16 MFMA with FP32 accumulation, QR of the
                         power iterates in FP32 except the last V = Qpos(Y), which is taken
                         in FP64, as is the final A V = U R */
  URV_MIXED_FP16 = 3  /* as above with FP16 operands */
} urv_precision;

/* Bits of urv_opts.flags. */
#define URV_CHECK_FINITE 1 /* scan A first; NaN or infinity -> URV_ENONFINITE (the call then waits for the scan) */
#define URV_A_FP32 2       /* A points to FP32 values (the 16-bit casts of the mixed modes read them directly;
                              the FP64 steps use their exact FP64 value) */

typedef struct {
  int32_t variant;    /* urv_variant */
  int32_t precision;  /* urv_precision */
  int32_t orth_g;     /* nonzero: start the power iteration from Qpos(G) instead of G */
  int32_t flags;      /* URV_CHECK_FINITE | URV_A_FP32; other bits must be 0 */
  int64_t lda, ldu, ldr, ldv; /* leading dimensions; 0 selects the packed value (m, m, p, n), p = min(m, n) */
  const double* G;    /* optional p x p starting matrix (device); NULL draws it from seed */
  int64_t ldg;        /* leading dimension of G; 0 = p */
  void* stream;       /* hipStream_t; NULL = default stream */
  void* workspace;    /* optional device workspace; NULL = the library allocates on the stream */
  size_t workspace_bytes;
} urv_opts;

/* Fills opts with the defaults: FULL, FP64, packed leading dimensions, drawn G,
 * default stream, library-allocated workspace. */
void urv_opts_init(urv_opts* opts);

/*
 * PowerURV (Section 3, eqs. power and powerqr).  A is m x n (read only;
 * FP64, or FP32 with URV_A_FP32 in opts->flags); p = min(m, n).  A Gaussian p x p G (eq. power) is drawn from seed (see
 * urv_gaussian, stream id 2) unless opts->G is given.  Then q >= 0 power
 * steps are taken on V (V starts as G, or Qpos(G) when q == 0 -- the DDH-URV
 * case of Section 2.2 -- or when orth_g is set), and the final step factors
 * A V = U R.  Qpos is an unpivoted blocked Householder QR whose R has a
 * non-negative diagonal.
 * Outputs: U m x p with orthonormal columns, R p x p upper triangular (its
 * strictly lower part is written as 0), V n x p with orthonormal columns;
 * A = U R V^T.  m < n (Section 1: a ULV of A^T, transposed): the method runs
 * on B = A^T up to X = B V_B; X with its columns reversed (J) is factored,
 * X J = Q R', and U = V_B (m x m), R = J R'^T J, V = Q J (n x m).
 * min(m, n) == 0 is a no-op returning URV_OK.  q < 0, ld < rows (ldr < p,
 * ldv < n, ldg < p), unknown enums, null pointers or a too-small workspace
 * give URV_EINVAL; max(m, n) beyond the panel kernel's rows, URV_ENOTSUP.
 * With URV_CHECK_FINITE, a NaN or infinity in A gives URV_ENONFINITE and no
 * output is written.  Asynchronous on opts->stream (except for that scan);
 * an expired device-side wait is reported by urv_sync_status.  In the FP16
 * mode each 16-bit operand is scaled by a power of two from its largest
 * magnitude before the cast (exact, and Qpos is unchanged by it), so entries
 * beyond FP16's range do not overflow.
 */
int urv_factor_ex(const void* A, int64_t m, int64_t n, int32_t q, uint64_t seed,
                  double* U, double* R, double* V, const urv_opts* opts);

/* Launch timing, for measurement (not in the paper).  urv_timing(1) clears the
 * counts and starts bracketing the library's FP64 launches of each class with
 * HIP events on the stream each runs on; urv_timing(0) stops.  After the
 * caller has synchronised, urv_timing_read gives (HOST pointers) the summed
 * elapsed milliseconds, the number of launches and their algorithmic flops:
 * class 0 the QR panel kernel (Householder QR of its mp x jb panel, plus the
 * previous block's two products 4 (mp + 128) 128 jb when it applies them),
 * classes 1..4 the FP64 GEMM tiles NN, TN, NT, TT (2 M N K each).  Unknown
 * class or null pointers: URV_EINVAL.  The registry is process-wide. */
int urv_timing(int32_t enable);
int urv_timing_read(int32_t cls, double* ms, int64_t* launches, double* flops);

/* Waits for the stream, then reports whether any factorisation or QR queued
 * on the current device since the last report had a panel's bounded
 * device-side wait expire (URV_EDEVICE, outputs of that call NaN) or not
 * (URV_OK), and clears that state.  The state is per device, shared by every
 * stream and thread.  Allocates nothing. */
int urv_sync_status(void* stream);

/* urv_factor_ex with default options (FULL, FP64, packed, default stream);
 * returns after the device work has finished. */
int urv_factor(const double* A, int64_t m, int64_t n, int32_t q, uint64_t seed,
               double* U, double* R, double* V);

/* Bytes of device workspace urv_factor_ex needs for these arguments (opts may
 * be NULL for the defaults).  0 when min(m, n) == 0. */
size_t urv_workspace_size(int64_t m, int64_t n, int32_t q, const urv_opts* opts);

/*
 * The Gaussian matrix of eq. power (Section 3).  Element (i,j) is number
 * l = i + j*rows of a counter-based stream: Philox4x64-10 (Salmon et al.,
 * SC'11) with key (seed, 0) and counter (l/4, stream_id, 0, 0) gives four
 * 64-bit words w; u = ((w >> 11) + 0.5) * 2^-53 in (0,1); Box-Muller maps
 * (u0,u1) to sqrt(-2 ln u0) (cos 2 pi u1, sin 2 pi u1) and likewise (u2,u3);
 * element l takes output l % 4.  G: rows x cols with leading dimension ld,
 * FP64 (precision URV_FP64) or FP32 (any other value: the FP32 rounding of
 * the FP64 value).  urv_factor_ex draws its G with stream_id 2.
 */
int urv_gaussian(void* G, int64_t rows, int64_t cols, int64_t ld, uint64_t seed,
                 uint32_t stream_id, int32_t precision, void* stream);

/*
 * C = alpha * op(A) * op(B) + beta * C in FP64 on MFMA (the products A V and
 * A^T W of Section 3 and the block-reflector updates of Section 2.2).
 * op(X) = X when trans == 0, X^T otherwise; C is M x N, op(A) M x K,
 * op(B) K x N.  beta == 0 never reads C.  C must not overlap A or B.
 * Sums over k are split in a fixed order: results are bitwise reproducible.
 */
int urv_dgemm(int32_t transA, int32_t transB, int64_t M, int64_t N, int64_t K,
              double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
              double beta, double* C, int64_t ldc, void* stream);

/*
 * urv_dgemm for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, arithmetic and bitwise results, but the split-K partial
 * sums live in a static 32 MiB device buffer that the library holds on every
 * GPU it runs on until the process ends; this call allocates nothing.  Shapes
 * whose partial sums would exceed 32 MiB return URV_EINVAL (message in
 * urv_last_error) before any device work.  Every call on one GPU shares that
 * buffer: calls that overlap on one GPU (different streams, or host threads,
 * without ordering between them) race and give wrong results.
 */
int urv_dgemm_noalloc(int32_t transA, int32_t transB, int64_t M, int64_t N, int64_t K,
                      double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                      double beta, double* C, int64_t ldc, void* stream);

/*
 * Qpos: unpivoted blocked Householder QR of X (m x n, m >= n) with the
 * diagonal of R made non-negative (the Q-factors of Section 2.2 and eqs.
 * power / powerqr; the footnote on Haar matrices fixes the sign).  X is
 * overwritten.  Q (m x n, explicit) and R (n x n, strictly lower part
 * written as 0) may each be NULL when not wanted.  Asynchronous on stream;
 * the workspace is allocated on the stream by the library.
 */
int urv_qr_pos(double* X, int64_t m, int64_t n, int64_t ldx, double* Q, int64_t ldq,
               double* R, int64_t ldr, void* stream);

/* urv_qr_pos in FP32 (the QR of the power iterates in the mixed-precision
 * form): same layout, ownership and errors, FP32 matrices. */
int urv_qr_pos_f32(float* X, int64_t m, int64_t n, int64_t ldx, float* Q, int64_t ldq,
                   float* R, int64_t ldr, void* stream);

/*
 * Checks of a factorisation, in FP64 on the device (rank-k errors of
 * Section 5 and the partition of eq. blocks), with p = min(m, n), U m x p,
 * R p x p, V n x p.  Blocking.  out (HOST, 4
 * doubles): ||A - U R V^T||_F / ||A||_F, ||U^T U - I||_F, ||V^T V - I||_F,
 * ||A||_F.  ek (HOST, p+1 doubles, may be NULL): ek[k] = ||R(k:p-1,k:p-1)||_F
 * over the upper triangle, the Frobenius error of the rank-k truncation
 * U(:,1:k) R(1:k,:) V^T when A = U R V^T.  Packed leading dimensions.
 */
int urv_metrics(const double* A, int64_t m, int64_t n, const double* U, const double* R,
                const double* V, double* out, double* ek, void* stream);

/* ------------------------------------------------------------------------
 * Derivative of the factorisation with G held fixed (not in the paper).
 *
 * The forward chain is that of Section 3 (eqs. power and powerqr) from a
 * given n x n starting matrix G: V_0 = G; for t = 1..q, X_t = A V_{t-1},
 * (W_t, Rw_t) = Qpos(X_t), Y_t = A^T W_t, (V_t, Rv_t) = Qpos(Y_t) (HALF:
 * Y_t = A^T X_t); then A V_q = U R and V = V_q.  q == 0 takes V = Qpos(G), a
 * constant.  The reverse sweep applies the adjoint of each product and of each
 * QR (for X = Q R with m >= n and diag(R) != 0: Xb = (Qb + Q S) R^{-T}, S
 * the symmetric matrix from the lower triangle of R Rb^T - Qb^T Q, after
 * Walter & Lehmann 2018 and Seeger et al. 2017) in the opposite order.
 *
 * All matrices are packed column-major device arrays (ld = rows) of the type
 * opts->precision selects: double (URV_FP64) or float (URV_FP32).  The
 * derivative exists where every QR of the chain has full column rank; where a
 * diagonal entry of an R is zero the outputs are not finite, except the last
 * entry of a square QR's R: there the last column of Xb is Q Rb(:,n) exactly
 * ((I - Q Q^T) Qb vanishes for square Q), with no division.  Every call is
 * asynchronous on opts->stream; a device-side wait of a QR that expired leaves
 * NaN in the outputs.  Argument errors return URV_EINVAL before any launch;
 * m beyond the QR panel's row limit returns URV_ENOTSUP.
 * ---------------------------------------------------------------------- */

/* What the tape between urv_factor_tape and urv_factor_backward keeps. */
typedef enum {
  URV_TAPE_ALL = 0,  /* every Q and R of the power steps: the reverse sweep recomputes nothing */
  URV_TAPE_V = 1,    /* the V_t only: each power step is recomputed from its V_{t-1} */
  URV_TAPE_NONE = 2  /* nothing: each V_{t-1} is recomputed from G as well (q(q+1)/2 steps) */
} urv_tape_mode;

typedef struct {
  int32_t precision;   /* URV_FP64 or URV_FP32 */
  int32_t variant;     /* URV_REORTH_FULL or URV_REORTH_HALF */
  int32_t tape_mode;   /* urv_tape_mode; forward and backward must use the same value */
  int32_t accumulate;  /* urv_factor_backward: nonzero adds to dA instead of overwriting it */
  void* stream;        /* hipStream_t; NULL = default stream */
  void* workspace;     /* optional device scratch of urv_grad_workspace_size bytes; NULL = the
                          library allocates on the stream */
  size_t workspace_bytes;
} urv_grad_opts;

/* Defaults: FP64, FULL, URV_TAPE_ALL, overwrite, default stream, library workspace. */
void urv_grad_opts_init(urv_grad_opts* opts);

/* Bytes of the tape for these arguments (0 for q == 0, URV_TAPE_NONE or bad arguments). */
size_t urv_tape_bytes(int64_t m, int64_t n, int32_t q, const urv_grad_opts* opts);

/* Bytes of scratch a derivative entry point needs (0 for n == 0 or bad arguments). */
size_t urv_grad_workspace_size(int64_t m, int64_t n, int32_t q, const urv_grad_opts* opts);

/*
 * Forward pass: U (m x n), R (n x n, strictly lower part 0), V (n x n) of the
 * chain above from A (m x n, m >= n, read only) and G (n x n, read only), and
 * the tape (urv_tape_bytes, caller-owned, opaque) that urv_factor_backward
 * reads.  The tape must stay unmodified, together with A, G, U, R and V,
 * until the backward call has run.
 */
int urv_factor_tape(const void* A, int64_t m, int64_t n, int32_t q, const void* G, void* U, void* R,
                    void* V, void* tape, const urv_grad_opts* opts);

/*
 * Reverse pass: dA (m x n) = dL/dA for a loss L(U, R, V) whose adjoints are
 * dU (m x n), dR (n x n; only its upper triangle is read in effect) and dV
 * (n x n); each may be NULL for zero.  A, G, U, R, V and the tape are those of
 * the forward call.  With opts->accumulate the result is added to dA.
 */
int urv_factor_backward(const void* A, int64_t m, int64_t n, int32_t q, const void* G, const void* U,
                        const void* R, const void* V, const void* tape, const void* dU, const void* dR,
                        const void* dV, void* dA, const urv_grad_opts* opts);

/*
 * Adjoint of one QR X = Q R (Q m x n, R n x n upper, m >= n): dX = (dQ + Q S) R^{-T}
 * with S from the lower triangle of R dR^T - dQ^T Q.  dQ or dR may be NULL
 * (zero).  For m == n the last column of dX is Q dR(:,n) (no division by
 * R(n,n), which may then be zero).  precision URV_FP64 or URV_FP32;
 * asynchronous on stream.
 */
int urv_qr_adjoint(const void* Q, const void* R, int64_t m, int64_t n, const void* dQ, const void* dR,
                   void* dX, int32_t precision, void* stream);

/*
 * The rank-k truncation loss L = ||A - A_k||_F^2 with A_k = U(:,1:k) R(1:k,:) V^T
 * (its square root is the rank-k error of Section 5 when A = U R V^T), and
 * its adjoints: dU, dR, dV (each may be NULL: not formed) and dA = 2 (A - A_k),
 * the loss's own term in A (required).  loss (DEVICE, one double, may be
 * NULL) receives L summed in FP64 in a fixed order.  0 <= k <= n.
 */
int urv_truncation_loss(const void* A, int64_t m, int64_t n, const void* U, const void* R, const void* V,
                        int64_t k, double* loss, void* dU, void* dR, void* dV, void* dA,
                        const urv_grad_opts* opts);

/* ------------------------------------------------------------------------
 * Batched factorisation: many independent FP32 matrices (1 <= n <= m <= 1024,
 * sizes may all differ) factored by one persistent kernel launch.  Matrix i
 * runs PowerURV (Section 3, eqs. power and powerqr, FULL re-orthonormalisation)
 * with its own Gaussian G drawn as in urv_gaussian (FP32 rounding) under seed
 * + i, stream id 2, and q power steps; diag(R) >= 0 as in urv_qr_pos.
 * One workgroup factors one matrix at a time, taking matrices largest first
 * from a device-side queue.  Matrices are packed column-major FP32 device
 * arrays: A_i m_i x n_i (ld m_i, read only), U_i m_i x n_i, R_i n_i x n_i
 * (zero below the diagonal), V_i n_i x n_i.
 * ---------------------------------------------------------------------- */
typedef struct urv_batch_plan urv_batch_plan; /* opaque */

/* Plan for `count` matrices with HOST arrays m[count], n[count]: validates
 * the sizes (URV_EINVAL; URV_ENOTSUP above 1024 rows), allocates the device
 * scratch of every matrix and the queue (this call allocates; the run calls do
 * not), and orders the queue by m n^2, largest first.  Blocking. */
int urv_batch_create(int64_t count, const int64_t* m, const int64_t* n, int32_t q, uint64_t seed,
                     urv_batch_plan** plan);

/* Sets the matrices: HOST arrays of count DEVICE pointers.  Blocking (copies
 * the descriptors to the device).  May be called again with other buffers of
 * the same sizes; a captured graph stays valid. */
int urv_batch_set_buffers(urv_batch_plan* plan, const float* const* A, float* const* U, float* const* R,
                          float* const* V);

/* Panel width nb (16 or 32), number of persistent workgroups (1..65536) and
 * largest team (1..64).  With team_max > 1 a matrix whose cost m n^2 exceeds
 * the average load of one workgroup is factored by a team of up to team_max
 * workgroups (GEMM tiles and element ranges split over the members, the panels
 * on one member, device-wide barriers between the phases); teams need every
 * workgroup resident at once, so grid must not exceed the device's capacity
 * for the kernel (URV_EINVAL otherwise).  Results do not depend on grid or
 * team_max, bit for bit.  Not while a run of the plan is in flight.
 * urv_batch_create selects nb 32, the device's capacity and team_max 1;
 * urv_batch_autotune chooses by timing. */
int urv_batch_set_config(urv_batch_plan* plan, int32_t nb, int32_t grid, int32_t team_max);
int urv_batch_get_config(const urv_batch_plan* plan, int32_t* nb, int32_t* grid, int32_t* team_max);

/* Times every (nb, team_max) candidate, with the grid at the device's
 * capacity, on the plan's matrices (running the whole batch twice each on
 * stream, blocking) and keeps the fastest; *best_ms (HOST, may be NULL)
 * receives its time.  The outputs hold a valid result. */
int urv_batch_autotune(urv_batch_plan* plan, void* stream, double* best_ms);

/* One persistent launch on stream (asynchronous; no allocation, no host-side
 * clearing).  Two runs of one plan must not overlap. */
int urv_batch_run(urv_batch_plan* plan, void* stream);

/* urv_batch_run through a graph: the launch is captured into a graph on the
 * first call (and after a configuration change), then the graph is launched
 * on stream. */
int urv_batch_run_graph(urv_batch_plan* plan, void* stream);

/* Blocking: URV_EDEVICE if a team barrier's bounded wait expired in a run so
 * far (its outputs are then invalid), else URV_OK. */
int urv_batch_status(urv_batch_plan* plan, void* stream);

/* Frees the plan's device memory and graph (after the stream work that uses it). */
void urv_batch_destroy(urv_batch_plan* plan);

/* The largest row count of the tall problem (max(m, n) for urv_factor_ex, m for
 * urv_qr_pos and the derivative calls) that the QR panel supports; larger
 * inputs return URV_ENOTSUP. */
int64_t urv_max_rows(void);

/* Static text for a status code. */
const char* urv_strerror(int code);

/* Detail text of the last error on the calling thread ("" if none). */
const char* urv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* URV_H */
