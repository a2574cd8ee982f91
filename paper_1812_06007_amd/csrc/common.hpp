// Internal declarations shared by the liburv translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
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
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

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

// FP64 GEMM.  work: device scratch for split-K partial sums (may be null:
// then no split-K is used); work_elems its capacity in doubles.
int dgemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
          int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
          double* work, size_t work_elems, hipStream_t s);
// Scratch doubles dgemm may use for the given shape (0 if it never splits K).
size_t dgemm_work_elems(int64_t M, int64_t N, int64_t K);

// 2-D copies / fills.
int copy_matrix(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                int64_t cols, hipStream_t s);

// ---------------------------------------------------------------- QR
constexpr int kPanelNB = 64;  // block width of the Householder QR

struct QrWork {
  double* Y = nullptr;      // m x n explicit unit-lower reflector blocks (ld = m)
  double* T = nullptr;      // kPanelNB x n: T of each block (ld = kPanelNB)
  double* tau = nullptr;    // n
  double* W1 = nullptr;     // kPanelNB x n
  double* W2 = nullptr;     // kPanelNB x n
  uint64_t* xch = nullptr;  // panel exchange slots (tagged partial sums, pivot rows)
  size_t xch_words = 0;
  unsigned* sync = nullptr; // panel barrier counters (one per block) + error flag
  double* gemm_work = nullptr;
  size_t gemm_work_elems = 0;
};

size_t qr_work_bytes(int64_t m, int64_t n);
void qr_work_carve(Arena& a, int64_t m, int64_t n, QrWork& w);
// Device flag set by a panel whose bounded device-wide wait expired.
unsigned* qr_error_flag(const QrWork& w, int64_t n);

// X (m x n, ldx) overwritten; Q (m x n) / R (n x n) optional.
int qr_pos(double* X, int64_t m, int64_t n, int64_t ldx, double* Q, int64_t ldq, double* R,
           int64_t ldr, const QrWork& w, hipStream_t s);

// ---------------------------------------------------------------- metrics
int metrics(const double* A, int64_t m, int64_t n, const double* U, const double* R,
            const double* V, double* out_host, double* ek_host, hipStream_t s);

}  // namespace urv
