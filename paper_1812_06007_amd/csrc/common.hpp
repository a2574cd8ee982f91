// Internal declarations shared by the liburv translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <mutex>
#include <string>

#include "urv.h"

namespace urv {

// ---------------------------------------------------------------- errors
// Thread-local detail text for urv_last_error().
void set_last_error(const std::string& msg);
void clear_last_error();

// Status from a HIP call; records the HIP message.
int hip_status(hipError_t e, const char* what);

#define URV_HIP(call)                                          \
  do {                                                         \
    hipError_t urv_e_ = (call);                                \
    if (urv_e_ != hipSuccess) return ::urv::hip_status(urv_e_, #call); \
  } while (0)

#define URV_TRY(expr)            \
  do {                           \
    int urv_rc_ = (expr);        \
    if (urv_rc_ != URV_OK) return urv_rc_; \
  } while (0)

// Launch check after <<<>>>.
#define URV_LAUNCHED(what) URV_HIP(hipGetLastError())

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// The dispatcher deals the workgroups of a launch to the 8 XCDs of MI355X
// round-robin (workgroup b runs on XCD b % 8), and each XCD has its own L2.
// Returns the logical tile index of workgroup b such that every XCD works
// through one contiguous range of the tile sequence (a bijection on
// [0, ntiles) for any ntiles), so neighbouring tiles share an L2.
__device__ inline int xcd_tile_order(int b, int ntiles) {
  const int q = ntiles >> 3, r = ntiles & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------- launch timing
// Host-side registry of HIP event pairs around the FP64 launches the bench
// reports (off unless urv_timing(1) is called): each class accumulates the
// elapsed time, the launch count and the algorithmic flops of its launches.
enum TimedKernel { kTimedPanel = 0, kTimedGemmNN, kTimedGemmTN, kTimedGemmNT, kTimedGemmTT, kTimedClasses };
// Records the start event on s; -1 when timing is off.
int timing_begin(hipStream_t s);
// Records the end event on s for the launch opened by token.
void timing_end(int token, int cls, double flops, hipStream_t s);
int timing_enable(bool on);
int timing_read(int cls, double* ms, int64_t* launches, double* flops);

// ---------------------------------------------------------------- workspace
// Bump allocator over one caller- or library-provided device block.
// With base == nullptr it only measures (used = bytes needed).
struct Arena {
  char* base = nullptr;
  size_t size = 0;
  size_t used = 0;
  bool overflow = false;
  template <class T>
  T* take(size_t count) {
    const size_t off = align_up(used, 256);
    const size_t bytes = align_up(count * sizeof(T), 256);
    used = off + bytes;
    if (base == nullptr) return nullptr;
    if (used > size) {
      overflow = true;
      return nullptr;
    }
    return reinterpret_cast<T*>(base + off);
  }
};

// ---------------------------------------------------------------- kernels
// Gaussian fill, see urv_gaussian.  out_f32 selects FP32 output.
int launch_gaussian(void* G, int64_t rows, int64_t cols, int64_t ld, uint64_t seed,
                    uint32_t stream_id, bool out_f32, hipStream_t s);

// FP64 / FP32 GEMM on MFMA.  work: device scratch for split-K partial sums
// (may be null: then no split-K is used); work_elems its capacity in elements.
template <class T>
int gemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, T alpha, const T* A, int64_t lda,
         const T* B, int64_t ldb, T beta, T* C, int64_t ldc, T* work, size_t work_elems,
         hipStream_t s);
inline int dgemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                 const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                 double* C, int64_t ldc, double* work, size_t work_elems, hipStream_t s) {
  return gemm<double>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, work, work_elems, s);
}
// Scratch elements gemm may use for the given shape (0 if it never splits K).
size_t gemm_work_elems(int64_t M, int64_t N, int64_t K);
// op(A) op(B) as `splits` partial sums over consecutive k chunks, each M x N
// packed (ld M) one after the other in `partial`, to be added in order by the
// consumer.  *splits is at least 1 and at most work_elems / (M N).
template <class T>
int gemm_partials(bool ta, bool tb, int64_t M, int64_t N, int64_t K, const T* A, int64_t lda, const T* B,
                  int64_t ldb, T* partial, size_t work_elems, int* splits, hipStream_t s);
// Scratch elements gemm_partials uses for this shape when given enough.
size_t gemm_partials_elems(int64_t M, int64_t N, int64_t K);
inline size_t dgemm_work_elems(int64_t M, int64_t N, int64_t K) { return gemm_work_elems(M, N, K); }

// 2-D copies / fills.
int copy_matrix(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                int64_t cols, hipStream_t s);

// ---------------------------------------------------------------- QR
constexpr int kPanelNB = 64;  // block width of the Householder QR
// Tallest matrix (rows of the tall problem) the QR accepts: the panel's
// workgroups must all be resident at once, and this is the largest height the
// tests factor and compare with the oracle.
constexpr int64_t kMaxRows = 64 * 256;

template <class T>
struct QrWorkT {
  T* Y = nullptr;           // m x n explicit unit-lower reflector blocks (ld = m)
  T* Tm = nullptr;          // 2 kPanelNB x n: T of each 128-column block (ld = 2 kPanelNB)
  T* tau = nullptr;         // n
  T* W1 = nullptr;          // 2 kPanelNB x n, bulk trailing updates (fourth stream)
  T* W2 = nullptr;          // 2 kPanelNB x n
  uint64_t* xch = nullptr;  // panel exchange slots (tagged partial sums, pivot rows)
  size_t xch_words = 0;
  uint64_t* jxch = nullptr; // exchange of the panel join: P x 4096 partial sums, then 4096 sums
  size_t jxch_words = 0;
  uint64_t* txch = nullptr; // exchange of the tall-skinny panel: R factors, U^-1 and T
  size_t txch_words = 0;
  unsigned* sync = nullptr; // panel error flag area
  T* gemm_work = nullptr;   // split-K partial sums of the bulk trailing updates
  size_t gemm_work_elems = 0;
  // updates of the next two column blocks (caller's stream)
  T* W1n = nullptr;         // 2 kPanelNB x 2 kPanelNB
  T* W2n = nullptr;         // 2 kPanelNB x 2 kPanelNB
  T* Tq = nullptr;          // 4 kPanelNB x 4 kPanelNB: joined T of the block pair the updates apply
  T* gemm_work_n = nullptr;
  size_t gemm_work_n_elems = 0;
  // scratch of the block factorisations, which run on a second stream
  T* W1b = nullptr;         // kPanelNB x kPanelNB
  T* W2b = nullptr;         // kPanelNB x kPanelNB
  T* gemm_work_b = nullptr;
  size_t gemm_work_b_elems = 0;
  // scratch of the reflectors applied to targets (third stream)
  int64_t target_rows = 0;  // largest target row count the workspace covers
  T* W1f = nullptr;         // target_rows x 4 kPanelNB
  T* W2f = nullptr;         // target_rows x 4 kPanelNB
  T* Tp = nullptr;          // 4 kPanelNB x n: T of pairs of 128-column blocks, for the targets
  T* gemm_work_f = nullptr;
  size_t gemm_work_f_elems = 0;
};
using QrWork = QrWorkT<double>;

// Workspace of qr_pos for an m x n matrix and targets of up to target_rows rows.
template <class T>
size_t qr_work_bytes(int64_t m, int64_t n, int64_t target_rows = 0);
template <class T>
void qr_work_carve(Arena& a, int64_t m, int64_t n, QrWorkT<T>& w, int64_t target_rows = 0);
// Device flag set by a panel whose bounded device-wide wait expired.  qr_pos
// does not clear it: a caller clears it once before a whole computation.
template <class T>
unsigned* qr_error_flag(const QrWorkT<T>& w, int64_t n);
template <class T>
int qr_clear_error_flag(const QrWorkT<T>& w, int64_t n, hipStream_t s);

// Streams of the current device for the QR pipeline beside the caller's,
// created on first use and kept for the life of the process (non-blocking,
// default priority), with their events.  Work is enqueued on them only while
// *mu is held, so calls from several host threads keep their event records and
// waits paired.
struct SideStream {
  hipStream_t stream = nullptr;   // block factorisations
  hipStream_t stream3 = nullptr;  // reflectors applied to the targets of a QR
  hipStream_t stream4 = nullptr;  // bulk of the trailing updates
  hipEvent_t ev_next = nullptr;
  hipEvent_t ev_fact = nullptr;   // block factored (even blocks)
  hipEvent_t ev_fact2 = nullptr;  // block factored (odd blocks)
  hipEvent_t ev_tgt = nullptr;
  hipEvent_t ev_near = nullptr;
  hipEvent_t ev_bulk = nullptr;
  hipEvent_t ev_pair = nullptr;
  hipEvent_t ev_defer = nullptr;       // caller's stream -> stream3: work deferred beside the next QR
  hipEvent_t ev_defer_done = nullptr;  // stream3 -> caller's stream
  std::mutex* mu = nullptr;
};
int side_stream(SideStream* out);

// A matrix Z (rows x m, ld ldz) to be multiplied on the right by the Q factor
// of a QR of an m x n matrix: on return Z(:, 0:n) = Z Q, where
// Q = H_1 ... H_n [D; 0] is the Q of qr_pos; columns n..m-1 are scratch.
template <class T>
struct QrTarget {
  T* Z = nullptr;
  int64_t rows = 0;
  int64_t ldz = 0;
};

// dst(:, j) = src(:, cols - 1 - j).
int reverse_cols(const double* src, int64_t lds, int64_t rows, int64_t cols, double* dst, int64_t ldd,
                 hipStream_t s);
// dst(i, j) = src(p - 1 - j, p - 1 - i) for p x p (J src^T J, J the reversal).
int transpose_reverse(const double* src, int64_t lds, int64_t p, double* dst, int64_t ldd, hipStream_t s);

// dst (cols x rows, ldd) = src^T for src rows x cols.
int transpose_matrix(const double* src, int64_t lds, int64_t rows, int64_t cols, double* dst, int64_t ldd,
                     hipStream_t s);
template <class T>
int set_identity(T* Z, int64_t rows, int64_t cols, int64_t ld, hipStream_t s);
// Z(:, j) *= sign(X(j, j)) for j < n (sign(0) = +1).
template <class T>
int scale_cols_sign(T* Z, int64_t rows, int64_t n, int64_t ldz, const T* X, int64_t ldx, hipStream_t s);

// X (m x n, ldx) overwritten; Q (m x n) / R (n x n) optional.  T = double or float.
// Targets (optional) get Z <- Z Q as above, applied block by block while the
// factorisation proceeds.
template <class T>
int qr_pos(T* X, int64_t m, int64_t n, int64_t ldx, T* Q, int64_t ldq, T* R, int64_t ldr,
           const QrWorkT<T>& w, hipStream_t s, const QrTarget<T>* targets = nullptr, int ntargets = 0);

// Q = H_1 ... H_n [D; 0] (m x n, ld ldq), D = diag(sign(X(c,c))), from the reflectors
// that the last qr_pos on w left there (X is that call's factored matrix): the blocks
// applied backward, 2 m n^2 - 2/3 n^3 flops.  With pairs, 256-column pairs of blocks are
// applied with the joined T that the call's target products formed (only valid after a
// qr_pos with targets).  On stream s; w's scratch must be free.
template <class T>
int form_q(const T* X, int64_t ldx, int64_t m, int64_t n, T* Q, int64_t ldq, const QrWorkT<T>& w, hipStream_t s,
           bool pairs);

// ---------------------------------------------------------------- mixed precision
// Leading dimension of a 16-bit operand with `rows` rows (multiple of 32).
int64_t lowp_ld(int64_t rows);
// C (FP32, M x N) = alpha A^T B + beta C for 16-bit (BF16 if bf16, else FP16) A (K x M) and
// B (K x N), column-major, leading dimensions multiples of 32 with zero padding below K.
int gemm_lowp(bool bf16, int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
              const void* B, int64_t ldb, float beta, float* C, int64_t ldc, hipStream_t s);
// dst (ldd x cols, 16-bit, RNE) = c src (rows x cols), zero in rows [rows, ldd).  c = 1
// without amax; with amax (device word from absmax), the power of two that brings
// max |src| into [2^13, 2^14) (exact; Qpos is unchanged by positive scaling).
template <class S>
int to_lowp(bool bf16, const S* src, int64_t lds, int64_t rows, int64_t cols, void* dst, int64_t ldd,
            hipStream_t s, const unsigned* amax = nullptr);
// dst (ldd x rows, 16-bit) = c src^T for src rows x cols, zero in rows [cols, ldd).
template <class S>
int to_lowp_transposed(bool bf16, const S* src, int64_t lds, int64_t rows, int64_t cols, void* dst, int64_t ldd,
                       hipStream_t s, const unsigned* amax = nullptr);
// *amax (device) = bits of max |src| as FP32.
template <class S>
int absmax(const S* src, int64_t lds, int64_t rows, int64_t cols, unsigned* amax, hipStream_t s);
template <class S, class D>
int convert(const S* src, int64_t lds, int64_t rows, int64_t cols, D* dst, int64_t ldd, hipStream_t s);
int copy_matrix_f32(const float* src, int64_t lds, float* dst, int64_t ldd, int64_t rows, int64_t cols,
                    hipStream_t s);

// ---------------------------------------------------------------- metrics
int metrics(const double* A, int64_t m, int64_t n, const double* U, const double* R,
            const double* V, double* out_host, double* ek_host, hipStream_t s);

}  // namespace urv
