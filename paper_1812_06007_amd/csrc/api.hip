// C ABI of liburv (include/urv.h) and the PowerURV driver of Section 3:
//
//   G (n x n Gaussian, eq. power)          -> V  (V = Qpos(G) when q == 0: DDH-URV)
//   q times:  X = A V;  FULL: W = Qpos(X), V = Qpos(A^T W)
//                       HALF: V = Qpos(A^T X);  NONE: V = A^T X
//   NONE, q > 0: V = Qpos(V)                 ((A^T A)^q G = V Z, eq. power)
//   X = A V;  (U, R) = Qpos(X)               (eq. powerqr)
//
// Every step is a kernel launch on the caller's stream; the host only
// validates arguments, carves the workspace and sequences launches.
#include "common.hpp"

#include <cstring>

namespace urv {

namespace {
thread_local std::string g_last_error;

struct FactorWork {
  double* X = nullptr;   // m x n (ld m): A V, factored in place
  double* Xs = nullptr;  // n x n (ld n): A^T W, factored in place
  double* gemm_work = nullptr;
  size_t gemm_work_elems = 0;
  QrWork qr;
};

size_t driver_gemm_work(int64_t m, int64_t n) {
  return std::max(dgemm_work_elems(m, n, n), dgemm_work_elems(n, n, m));
}

void carve_factor(Arena& a, int64_t m, int64_t n, FactorWork& w) {
  w.X = a.take<double>(static_cast<size_t>(m) * n);
  w.Xs = a.take<double>(static_cast<size_t>(n) * n);
  w.gemm_work_elems = driver_gemm_work(m, n);
  w.gemm_work = a.take<double>(w.gemm_work_elems);
  qr_work_carve(a, m, n, w.qr);
}

size_t factor_bytes(int64_t m, int64_t n) {
  Arena a;
  FactorWork w;
  carve_factor(a, m, n, w);
  return a.used;
}

constexpr int64_t kMaxRows = 240 * 256;  // rows the panel kernel's co-resident grid covers

int validate_factor(const double* A, int64_t m, int64_t n, int32_t q, const double* U,
                    const double* R, const double* V, const urv_opts& o) {
  if (n < 0 || m < n || q < 0) {
    set_last_error("urv_factor: need 0 <= n <= m and q >= 0");
    return URV_EINVAL;
  }
  if (o.variant < URV_REORTH_FULL || o.variant > URV_REORTH_NONE) {
    set_last_error("urv_factor: unknown variant");
    return URV_EINVAL;
  }
  if (o.precision != URV_FP64 && o.precision != URV_MIXED_BF16 && o.precision != URV_MIXED_FP16) {
    set_last_error("urv_factor: unknown precision");
    return URV_EINVAL;
  }
  if (o.reserved != 0) {
    set_last_error("urv_factor: reserved field must be 0");
    return URV_EINVAL;
  }
  if (n == 0) return URV_OK;
  if (!A || !U || !R || !V) {
    set_last_error("urv_factor: null matrix pointer");
    return URV_EINVAL;
  }
  const int64_t lda = o.lda ? o.lda : m, ldu = o.ldu ? o.ldu : m;
  const int64_t ldr = o.ldr ? o.ldr : n, ldv = o.ldv ? o.ldv : n, ldg = o.ldg ? o.ldg : n;
  if (lda < m || ldu < m || ldr < n || ldv < n || ldg < n || o.lda < 0 || o.ldu < 0 ||
      o.ldr < 0 || o.ldv < 0 || o.ldg < 0) {
    set_last_error("urv_factor: leading dimension smaller than the row count");
    return URV_EINVAL;
  }
  if (o.workspace == nullptr && o.workspace_bytes != 0) {
    set_last_error("urv_factor: workspace_bytes given without a workspace");
    return URV_EINVAL;
  }
  if (o.workspace != nullptr && o.workspace_bytes < factor_bytes(m, n)) {
    set_last_error("urv_factor: workspace too small (see urv_workspace_size)");
    return URV_EINVAL;
  }
  if (m > kMaxRows) {
    set_last_error("urv_factor: more rows than the panel kernel supports");
    return URV_ENOTSUP;
  }
  if (o.precision != URV_FP64) {
    set_last_error("urv_factor: mixed precision is not available in this build");
    return URV_ENOTSUP;
  }
  return URV_OK;
}

int run_factor(const double* A, int64_t m, int64_t n, int32_t q, uint64_t seed, double* U,
               double* R, double* V, const urv_opts& o, const FactorWork& w, hipStream_t s) {
  const int64_t lda = o.lda ? o.lda : m, ldu = o.ldu ? o.ldu : m;
  const int64_t ldr = o.ldr ? o.ldr : n, ldv = o.ldv ? o.ldv : n, ldg = o.ldg ? o.ldg : n;
  const bool full = o.variant == URV_REORTH_FULL, none = o.variant == URV_REORTH_NONE;

  // Starting matrix G of eq. (power).
  if (o.G)
    URV_TRY(copy_matrix(o.G, ldg, V, ldv, n, n, s));
  else
    URV_TRY(launch_gaussian(V, n, n, ldv, seed, 2u, false, s));
  if (q == 0 || o.orth_g) {
    URV_TRY(copy_matrix(V, ldv, w.Xs, n, n, n, s));
    URV_TRY(qr_pos(w.Xs, n, n, n, V, ldv, nullptr, 0, w.qr, s));
  }
  for (int32_t t = 0; t < q; ++t) {
    URV_TRY(dgemm(false, false, m, n, n, 1.0, A, lda, V, ldv, 0.0, w.X, m, w.gemm_work,
                  w.gemm_work_elems, s));                                   // X = A V
    if (full) {
      URV_TRY(qr_pos(w.X, m, n, m, U, ldu, nullptr, 0, w.qr, s));          // W = Qpos(X), in U
      URV_TRY(dgemm(true, false, n, n, m, 1.0, A, lda, U, ldu, 0.0, w.Xs, n, w.gemm_work,
                    w.gemm_work_elems, s));                                 // A^T W
      URV_TRY(qr_pos(w.Xs, n, n, n, V, ldv, nullptr, 0, w.qr, s));         // V = Qpos(A^T W)
    } else if (none) {
      URV_TRY(dgemm(true, false, n, n, m, 1.0, A, lda, w.X, m, 0.0, V, ldv, w.gemm_work,
                    w.gemm_work_elems, s));                                 // V = A^T A V
    } else {
      URV_TRY(dgemm(true, false, n, n, m, 1.0, A, lda, w.X, m, 0.0, w.Xs, n, w.gemm_work,
                    w.gemm_work_elems, s));                                 // A^T X
      URV_TRY(qr_pos(w.Xs, n, n, n, V, ldv, nullptr, 0, w.qr, s));         // V = Qpos(A^T X)
    }
  }
  if (none && q > 0) {
    URV_TRY(copy_matrix(V, ldv, w.Xs, n, n, n, s));
    URV_TRY(qr_pos(w.Xs, n, n, n, V, ldv, nullptr, 0, w.qr, s));
  }
  URV_TRY(dgemm(false, false, m, n, n, 1.0, A, lda, V, ldv, 0.0, w.X, m, w.gemm_work,
                w.gemm_work_elems, s));                                     // X = A V
  URV_TRY(qr_pos(w.X, m, n, m, U, ldu, R, ldr, w.qr, s));                  // A V = U R
  return URV_OK;
}

// Runs the factorisation; when check_flag, waits for the stream and reports a
// panel wait that expired on the device.
int factor_impl(const double* A, int64_t m, int64_t n, int32_t q, uint64_t seed, double* U,
                double* R, double* V, const urv_opts& o, bool check_flag) {
  clear_last_error();
  URV_TRY(validate_factor(A, m, n, q, U, R, V, o));
  if (n == 0) return URV_OK;
  hipStream_t s = static_cast<hipStream_t>(o.stream);
  const size_t need = factor_bytes(m, n);
  Arena a;
  bool owned = false;
  if (o.workspace) {
    a.base = static_cast<char*>(o.workspace);
    a.size = o.workspace_bytes;
  } else {
    void* p = nullptr;
    const hipError_t e = hipMallocAsync(&p, need, s);
    if (e != hipSuccess) {
      hipGetLastError();
      set_last_error(std::string("urv_factor: workspace allocation failed: ") + hipGetErrorString(e));
      return URV_ENOMEM;
    }
    a.base = static_cast<char*>(p);
    a.size = need;
    owned = true;
  }
  FactorWork w;
  carve_factor(a, m, n, w);
  int rc = a.overflow ? URV_EINVAL : run_factor(A, m, n, q, seed, U, R, V, o, w, s);
  if (rc == URV_OK && check_flag) {
    unsigned flag = 0;
    if (hipMemcpyAsync(&flag, qr_error_flag(w.qr, n), sizeof(flag), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = hip_status(hipGetLastError(), "urv_factor: synchronize");
      if (rc == URV_OK) rc = URV_EDEVICE;
    } else if (flag != 0) {
      set_last_error("urv_factor: a panel's device-wide wait expired");
      rc = URV_EDEVICE;
    }
  }
  if (owned) hipFreeAsync(a.base, s);
  return rc;
}

}  // namespace

void set_last_error(const std::string& msg) { g_last_error = msg; }
void clear_last_error() { g_last_error.clear(); }

int hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return URV_OK;
  set_last_error(std::string(what) + ": " + hipGetErrorString(e));
  return (e == hipErrorOutOfMemory) ? URV_ENOMEM : URV_EDEVICE;
}

}  // namespace urv

using namespace urv;

extern "C" {

void urv_opts_init(urv_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->variant = URV_REORTH_FULL;
  o->precision = URV_FP64;
}

int urv_factor_ex(const double* A, int64_t m, int64_t n, int32_t q, uint64_t seed, double* U,
                  double* R, double* V, const urv_opts* opts) {
  urv_opts o;
  urv_opts_init(&o);
  if (opts) o = *opts;
  return factor_impl(A, m, n, q, seed, U, R, V, o, false);
}

int urv_factor(const double* A, int64_t m, int64_t n, int32_t q, uint64_t seed, double* U,
               double* R, double* V) {
  urv_opts o;
  urv_opts_init(&o);
  return factor_impl(A, m, n, q, seed, U, R, V, o, true);
}

size_t urv_workspace_size(int64_t m, int64_t n, int32_t q, const urv_opts* opts) {
  (void)q;
  (void)opts;
  if (n <= 0 || m < n) return 0;
  return factor_bytes(m, n);
}

int urv_gaussian(void* G, int64_t rows, int64_t cols, int64_t ld, uint64_t seed,
                 uint32_t stream_id, int32_t precision, void* stream) {
  clear_last_error();
  if (rows < 0 || cols < 0 || (rows > 0 && ld < rows)) {
    set_last_error("urv_gaussian: bad size or leading dimension");
    return URV_EINVAL;
  }
  if (rows == 0 || cols == 0) return URV_OK;
  if (!G) {
    set_last_error("urv_gaussian: null pointer");
    return URV_EINVAL;
  }
  return launch_gaussian(G, rows, cols, ld, seed, stream_id, precision != URV_FP64,
                         static_cast<hipStream_t>(stream));
}

int urv_dgemm(int32_t transA, int32_t transB, int64_t M, int64_t N, int64_t K, double alpha,
              const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
              int64_t ldc, void* stream) {
  clear_last_error();
  if (M < 0 || N < 0 || K < 0) {
    set_last_error("urv_dgemm: negative size");
    return URV_EINVAL;
  }
  const int64_t arows = transA ? K : M, brows = transB ? N : K;
  if (lda < std::max<int64_t>(arows, 1) || ldb < std::max<int64_t>(brows, 1) ||
      ldc < std::max<int64_t>(M, 1)) {
    set_last_error("urv_dgemm: leading dimension smaller than the row count");
    return URV_EINVAL;
  }
  if (M == 0 || N == 0) return URV_OK;
  if (!C || (K > 0 && alpha != 0.0 && (!A || !B))) {
    set_last_error("urv_dgemm: null pointer");
    return URV_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t we = dgemm_work_elems(M, N, K);
  double* work = nullptr;
  if (we) URV_HIP(hipMallocAsync(reinterpret_cast<void**>(&work), we * sizeof(double), s));
  const int rc = dgemm(transA != 0, transB != 0, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                       work, we, s);
  if (work) hipFreeAsync(work, s);
  return rc;
}

int urv_qr_pos(double* X, int64_t m, int64_t n, int64_t ldx, double* Q, int64_t ldq, double* R,
               int64_t ldr, void* stream) {
  clear_last_error();
  if (n < 0 || m < n) {
    set_last_error("urv_qr_pos: need 0 <= n <= m");
    return URV_EINVAL;
  }
  if (n == 0) return URV_OK;
  if (!X || ldx < m || (Q && ldq < m) || (R && ldr < n)) {
    set_last_error("urv_qr_pos: null pointer or leading dimension smaller than the row count");
    return URV_EINVAL;
  }
  if (m > kMaxRows) {
    set_last_error("urv_qr_pos: more rows than the panel kernel supports");
    return URV_ENOTSUP;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t need = qr_work_bytes(m, n);
  void* p = nullptr;
  URV_HIP(hipMallocAsync(&p, need, s));
  Arena a;
  a.base = static_cast<char*>(p);
  a.size = need;
  QrWork w;
  qr_work_carve(a, m, n, w);
  const int rc = qr_pos(X, m, n, ldx, Q, ldq, R, ldr, w, s);
  hipFreeAsync(p, s);
  return rc;
}

int urv_metrics(const double* A, int64_t m, int64_t n, const double* U, const double* R,
                const double* V, double* out, double* ek, void* stream) {
  clear_last_error();
  if (n <= 0 || m < n || !A || !U || !R || !V || !out) {
    set_last_error("urv_metrics: need 0 < n <= m and non-null pointers");
    return URV_EINVAL;
  }
  return metrics(A, m, n, U, R, V, out, ek, static_cast<hipStream_t>(stream));
}

const char* urv_strerror(int code) {
  switch (code) {
    case URV_OK: return "success";
    case URV_EINVAL: return "invalid argument";
    case URV_ENOMEM: return "device memory allocation failed";
    case URV_EDEVICE: return "device (HIP) error";
    case URV_ENOTSUP: return "unsupported argument combination";
    default: return "unknown status";
  }
}

const char* urv_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
