// C ABI of liburv (include/urv.h) and the PowerURV driver of Section 3:
//
//   G (n x n Gaussian, eq. power)          -> V  (V = Qpos(G) when q == 0: DDH-URV)
//   q times:  X = A V;  FULL: W = Qpos(X), V = Qpos(A^T W)
//                       HALF: V = Qpos(A^T X);  NONE: V = A^T X
//   NONE, q > 0: V = Qpos(V)                 ((A^T A)^q G = V Z, eq. power)
//   X = A V;  (U, R) = Qpos(X)               (eq. powerqr)
//
// Mixed precision (not in the paper): the power-step products run on BF16 or
// FP16 matrix cores with FP32 accumulation and the QRs of the iterates in
// FP32; V is then re-orthonormalised once in FP64 (an FP32 QR leaves
// ||V^T V - I|| near 1e-6, which would bound the reconstruction error), and the
// final A V = U R is FP64, so A = U R V^T holds to FP64 accuracy.
//
// Every step is a kernel launch on the caller's stream; the host only
// validates arguments, carves the workspace and sequences launches.
#include "common.hpp"

#include <cstring>

namespace urv {

namespace {
thread_local std::string g_last_error;

struct MixedWork {
  void* A16 = nullptr;   // A rounded to 16 bits, m x n, ld lda16
  void* At16 = nullptr;  // A^T rounded to 16 bits, n x m, ld ldat16
  void* B16 = nullptr;   // second operand of a 16-bit product (V, W or X)
  int64_t lda16 = 0, ldat16 = 0;
  float* V32 = nullptr;  // n x n
  float* X32 = nullptr;  // m x n
  float* W32 = nullptr;  // m x n
  float* Y32 = nullptr;  // n x n
  unsigned* amax = nullptr;  // max |x| words of the FP16 casts (A, V, right-hand side)
  QrWorkT<float> qr;
};

struct FactorWork {
  double* X = nullptr;   // m x n (ld m): A V, factored in place
  double* Xs = nullptr;  // n x n (ld n): A^T W, factored in place
  double* At = nullptr;  // n x m (ld n): A^T, turned into A^T W by the reflectors of W
  double* gemm_work = nullptr;
  size_t gemm_work_elems = 0;
  QrWork qr;
  QrWork qr2;  // the final QR's, while V is formed from the reflectors left in qr
  bool mixed = false;
  MixedWork mx;
};

// Whether the square FP32 QRs of the mixed form take their explicit Q as the reflectors
// applied to I alongside the factorisation (2n^3, on the targets' stream, beside the chain)
// rather than backward after it (4/3 n^3, after the chain; URV_MIXED_ITARGET=0, for tuning).
// Measured on MI355X at n = 8000, q = 2, BF16: FULL 193.0-193.3 ms against 210.0-210.4.
bool mixed_identity_target() {
  const char* e = std::getenv("URV_MIXED_ITARGET");
  return !(e && std::atoi(e) == 0);
}

// Qpos of the square or tall FP32 matrix X (rows x n, ld rows, overwritten) into Q (ld rows).
int qpos_f32(float* X, int64_t rows, int64_t n, float* Q, const QrWorkT<float>& w, hipStream_t s) {
  if (rows == n && mixed_identity_target()) {
    URV_TRY(set_identity<float>(Q, rows, n, rows, s));
    const QrTarget<float> t{Q, rows, rows};
    return qr_pos<float>(X, rows, n, rows, nullptr, 0, nullptr, 0, w, s, &t, 1);
  }
  return qr_pos<float>(X, rows, n, rows, Q, rows, nullptr, 0, w, s);
}

// Whether the explicit V is formed from its QR's reflectors beside the final QR
// (URV_DEFER_V=0: as a product with I alongside its QR, for tuning).
bool defer_v() {
  const char* e = std::getenv("URV_DEFER_V");
  return !(e && std::atoi(e) == 0);
}

size_t driver_gemm_work(int64_t m, int64_t n) {
  return std::max(dgemm_work_elems(m, n, n), dgemm_work_elems(n, n, m));
}

void carve_factor(Arena& a, int64_t m, int64_t n, bool mixed, FactorWork& w) {
  w.X = a.take<double>(static_cast<size_t>(m) * n);
  w.Xs = a.take<double>(static_cast<size_t>(n) * n);
  w.At = a.take<double>(static_cast<size_t>(n) * m);
  w.gemm_work_elems = driver_gemm_work(m, n);
  w.gemm_work = a.take<double>(w.gemm_work_elems);
  qr_work_carve(a, m, n, w.qr, m);
  qr_work_carve(a, m, n, w.qr2, m);
  w.mixed = mixed;
  if (!mixed) return;
  MixedWork& x = w.mx;
  x.lda16 = lowp_ld(m);
  x.ldat16 = lowp_ld(n);
  x.A16 = a.take<uint16_t>(static_cast<size_t>(x.lda16) * n);
  x.At16 = a.take<uint16_t>(static_cast<size_t>(x.ldat16) * m);
  x.B16 = a.take<uint16_t>(static_cast<size_t>(std::max(x.lda16, x.ldat16)) * n);
  x.V32 = a.take<float>(static_cast<size_t>(n) * n);
  x.X32 = a.take<float>(static_cast<size_t>(m) * n);
  x.W32 = a.take<float>(static_cast<size_t>(m) * n);
  x.Y32 = a.take<float>(static_cast<size_t>(n) * n);
  x.amax = a.take<unsigned>(4);
  qr_work_carve(a, m, n, x.qr, n);  // targets of n rows: the square QRs' explicit Q formed from I
}

size_t factor_bytes(int64_t m, int64_t n, bool mixed) {
  Arena a;
  FactorWork w;
  carve_factor(a, m, n, mixed, w);
  return a.used;
}

// m < n: the tall problem of B = A^T (n x m) and the buffers of the transposed
// ULV (Section 1).
struct WideWork {
  double* B = nullptr;   // n x m: A^T
  double* Ut = nullptr;  // n x m: U of B's factorisation
  double* T = nullptr;   // n x m
  double* Rt = nullptr;  // m x m: R of B's factorisation
  double* RJ = nullptr;  // m x m: Rt with its columns reversed
  double* Q2 = nullptr;  // m x m
  double* R2 = nullptr;  // m x m
  double* gw = nullptr;
  size_t gw_elems = 0;
};

void carve_wide(Arena& a, int64_t m, int64_t n, WideWork& x) {
  const size_t nm = static_cast<size_t>(n) * m, mm = static_cast<size_t>(m) * m;
  x.B = a.take<double>(nm);
  x.Ut = a.take<double>(nm);
  x.T = a.take<double>(nm);
  x.Rt = a.take<double>(mm);
  x.RJ = a.take<double>(mm);
  x.Q2 = a.take<double>(mm);
  x.R2 = a.take<double>(mm);
  x.gw_elems = dgemm_work_elems(n, m, m);
  x.gw = a.take<double>(x.gw_elems);
}

// The parts of the workspace beyond the factorisation's own: the FP64 copy of
// an FP32 A, and the word of the finiteness scan.
struct ExtraWork {
  double* A64 = nullptr;       // m x n (ld m), with URV_A_FP32
  unsigned* nonfinite = nullptr;
};

void carve_extra(Arena& a, int64_t m, int64_t n, bool a32, ExtraWork& e) {
  if (a32) e.A64 = a.take<double>(static_cast<size_t>(m) * n);
  e.nonfinite = a.take<unsigned>(1);
}

// Workspace of urv_factor_ex for any shape.
size_t work_bytes(int64_t m, int64_t n, bool mixed, bool a32) {
  Arena a;
  FactorWork w;
  if (m >= n) {
    carve_factor(a, m, n, mixed, w);
  } else {
    carve_factor(a, n, m, mixed, w);
    WideWork x;
    carve_wide(a, m, n, x);
  }
  ExtraWork e;
  carve_extra(a, m, n, a32, e);
  return a.used;
}

// *flag = 1 if src (rows x cols) holds a NaN or an infinity.  *flag must be 0 before.
template <class S>
__global__ __launch_bounds__(256) void nonfinite_kernel(const S* __restrict__ src, int64_t lds, int64_t rows,
                                                        int64_t cols, unsigned* __restrict__ flag) {
  int bad = 0;
  const int64_t total = rows * cols;
  for (int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const S v = src[idx % rows + (idx / rows) * lds];
    bad |= !(v - v == v - v) ? 1 : 0;  // inf - inf and NaN - NaN are NaN
  }
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(flag, 1u);
}

__global__ void set_u32_kernel(unsigned* p, unsigned v) { *p = v; }

// Folds the error flags of a factorisation or QR into the device's status word.
__global__ void fold_status_kernel(unsigned* status, const unsigned* f1, const unsigned* f2, const unsigned* f3) {
  if ((f1 && *f1) || (f2 && *f2) || (f3 && *f3)) atomicOr(status, 1u);
}

// Per-device statics: the split-K scratch of urv_dgemm_noalloc and the status word
// that urv_sync_status reads (file-scope device arrays, one copy on every GPU the
// library runs on; host code uses the addresses hipGetSymbolAddress gives).
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __attribute__((aligned(256))) double scratch[kStaticScratchBytes / sizeof(double)];
static __device__ __attribute__((aligned(256))) unsigned status_word[64];
constexpr int kMaxDevices = 64;
struct DeviceStatics {
  double* scratch = nullptr;
  unsigned* status = nullptr;
};
std::mutex statics_mu;
DeviceStatics statics[kMaxDevices];

// The current device's statics, looked up once per device.
int device_statics(DeviceStatics* out) {
  int dev = 0;
  URV_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_last_error("liburv: device index beyond the library's table");
    return URV_ENOTSUP;
  }
  std::lock_guard<std::mutex> lock(statics_mu);
  DeviceStatics& d = statics[dev];
  if (!d.scratch) {
    void* p = nullptr;
    void* q = nullptr;
    URV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    URV_HIP(hipGetSymbolAddress(&q, HIP_SYMBOL(status_word)));
    d.scratch = static_cast<double*>(p);
    d.status = static_cast<unsigned*>(q);
  }
  *out = d;
  return URV_OK;
}

// Queues the fold of up to two error flags into the device's status word.
int fold_status(const unsigned* f1, const unsigned* f2, hipStream_t s, const unsigned* f3 = nullptr) {
  DeviceStatics d;
  URV_TRY(device_statics(&d));
  fold_status_kernel<<<1, 1, 0, s>>>(d.status, f1, f2, f3);
  URV_LAUNCHED("fold_status_kernel");
  return URV_OK;
}

// Waits for s, then reads and clears the device's status word.
int sync_status(hipStream_t s, const char* who) {
  DeviceStatics d;
  URV_TRY(device_statics(&d));
  URV_HIP(hipStreamSynchronize(s));
  unsigned v = 0;
  URV_HIP(hipMemcpy(&v, d.status, sizeof(v), hipMemcpyDeviceToHost));
  if (v == 0) return URV_OK;
  const unsigned zero = 0;
  URV_HIP(hipMemcpy(d.status, &zero, sizeof(zero), hipMemcpyHostToDevice));
  set_last_error(std::string(who) + ": a panel's device-wide wait expired");
  return URV_EDEVICE;
}


int validate_factor(const void* A, int64_t m, int64_t n, int32_t q, const double* U,
                    const double* R, const double* V, const urv_opts& o) {
  if (n < 0 || m < 0 || q < 0) {
    set_last_error("urv_factor: need m, n >= 0 and q >= 0");
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
  if ((o.flags & ~(URV_CHECK_FINITE | URV_A_FP32)) != 0) {
    set_last_error("urv_factor: unknown bits in flags");
    return URV_EINVAL;
  }
  const int64_t p = std::min(m, n);
  if (p == 0) return URV_OK;
  if (!A || !U || !R || !V) {
    set_last_error("urv_factor: null matrix pointer");
    return URV_EINVAL;
  }
  const int64_t lda = o.lda ? o.lda : m, ldu = o.ldu ? o.ldu : m;
  const int64_t ldr = o.ldr ? o.ldr : p, ldv = o.ldv ? o.ldv : n, ldg = o.ldg ? o.ldg : p;
  if (lda < m || ldu < m || ldr < p || ldv < n || ldg < p || o.lda < 0 || o.ldu < 0 ||
      o.ldr < 0 || o.ldv < 0 || o.ldg < 0) {
    set_last_error("urv_factor: leading dimension smaller than the row count");
    return URV_EINVAL;
  }
  if (o.workspace == nullptr && o.workspace_bytes != 0) {
    set_last_error("urv_factor: workspace_bytes given without a workspace");
    return URV_EINVAL;
  }
  if (o.workspace != nullptr &&
      o.workspace_bytes < work_bytes(m, n, o.precision != URV_FP64 && q > 0, (o.flags & URV_A_FP32) != 0)) {
    set_last_error("urv_factor: workspace too small (see urv_workspace_size)");
    return URV_EINVAL;
  }
  if (std::max(m, n) > kMaxRows) {
    set_last_error("urv_factor: more rows than the panel kernel supports");
    return URV_ENOTSUP;
  }
  return URV_OK;
}

// V = Qpos(Y) for Y n x n (ld n, overwritten), delivered as X = A V in w.X
// and, when wanted, explicitly in V: the reflectors of Y are applied to a copy
// of A (and to I) block by block while Y is being factored.
int qpos_times_a(const double* A, int64_t lda, int64_t m, int64_t n, double* Y, double* V, int64_t ldv,
                 bool want_v, const FactorWork& w, hipStream_t s) {
  QrTarget<double> t[2];
  int nt = 0;
  URV_TRY(copy_matrix(A, lda, w.X, m, m, n, s));
  t[nt++] = QrTarget<double>{w.X, m, m};
  const bool defer = want_v && defer_v();
  if (want_v && !defer) {
    URV_TRY(set_identity<double>(V, n, n, ldv, s));
    t[nt++] = QrTarget<double>{V, n, ldv};
  }
  URV_TRY(qr_pos<double>(Y, n, n, n, nullptr, 0, nullptr, 0, w.qr, s, t, nt));
  if (!defer) return URV_OK;
  // V from the reflectors, applied backward to [D; 0] (4/3 n^3 instead of the 2 n^3 of a
  // target), on the targets' stream beside the final QR, which runs on w.qr2; final_qr
  // joins it.  Y (the factored matrix, for D) and w.qr stay untouched until then.
  SideStream side;
  URV_TRY(side_stream(&side));
  std::lock_guard<std::mutex> lock(*side.mu);
  URV_HIP(hipEventRecord(side.ev_defer, s));
  URV_HIP(hipStreamWaitEvent(side.stream3, side.ev_defer, 0));
  return form_q<double>(Y, n, n, n, V, ldv, w.qr, side.stream3, true);
}

// The final step of eq. (powerqr): A V = U R with X = A V in w.X.
int final_qr(int64_t m, int64_t n, double* U, int64_t ldu, double* R, int64_t ldr, const FactorWork& w,
             hipStream_t s) {
  const bool defer = defer_v();
  const QrWork& wq = defer ? w.qr2 : w.qr;
  if (m == n) {  // U formed from I alongside the factorisation
    URV_TRY(set_identity<double>(U, m, n, ldu, s));
    const QrTarget<double> t{U, m, ldu};
    URV_TRY(qr_pos<double>(w.X, m, n, m, nullptr, 0, R, ldr, wq, s, &t, 1));
  } else {
    URV_TRY(qr_pos<double>(w.X, m, n, m, U, ldu, R, ldr, wq, s));
  }
  if (!defer) return URV_OK;
  // the V formed beside this QR (if any) is part of the result
  SideStream side;
  URV_TRY(side_stream(&side));
  std::lock_guard<std::mutex> lock(*side.mu);
  URV_HIP(hipEventRecord(side.ev_defer_done, side.stream3));
  URV_HIP(hipStreamWaitEvent(s, side.ev_defer_done, 0));
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
  if (none) {
    // (A^T A)^q G (or (A^T A)^q Qpos(G)), then one Qpos
    if (o.orth_g && q > 0) {
      URV_TRY(copy_matrix(V, ldv, w.Xs, n, n, n, s));
      URV_TRY(qr_pos<double>(w.Xs, n, n, n, V, ldv, nullptr, 0, w.qr, s));
    }
    for (int32_t t = 0; t < q; ++t) {
      URV_TRY(dgemm(false, false, m, n, n, 1.0, A, lda, V, ldv, 0.0, w.X, m, w.gemm_work,
                    w.gemm_work_elems, s));                                 // X = A V
      URV_TRY(dgemm(true, false, n, n, m, 1.0, A, lda, w.X, m, 0.0, V, ldv, w.gemm_work,
                    w.gemm_work_elems, s));                                 // V = A^T A V
    }
    URV_TRY(copy_matrix(V, ldv, w.Xs, n, n, n, s));
    URV_TRY(qpos_times_a(A, lda, m, n, w.Xs, V, ldv, true, w, s));          // V = Qpos, X = A V
    return final_qr(m, n, U, ldu, R, ldr, w, s);
  }
  if (q == 0 || o.orth_g) {
    URV_TRY(copy_matrix(V, ldv, w.Xs, n, n, n, s));
    URV_TRY(qpos_times_a(A, lda, m, n, w.Xs, V, ldv, q == 0, w, s));       // V = Qpos(G), X = A V
  } else {
    URV_TRY(dgemm(false, false, m, n, n, 1.0, A, lda, V, ldv, 0.0, w.X, m, w.gemm_work,
                  w.gemm_work_elems, s));                                   // X = A G
  }
  for (int32_t t = 0; t < q; ++t) {
    const bool last = t == q - 1;
    double* Y = w.Xs;
    if (full) {
      // W = Qpos(X) is needed only as A^T W: its reflectors are applied to A^T
      URV_TRY(transpose_matrix(A, lda, m, n, w.At, n, s));
      const QrTarget<double> tt{w.At, n, n};
      URV_TRY(qr_pos<double>(w.X, m, n, m, nullptr, 0, nullptr, 0, w.qr, s, &tt, 1));
      Y = w.At;                                                             // A^T W, n x n
    } else {
      URV_TRY(dgemm(true, false, n, n, m, 1.0, A, lda, w.X, m, 0.0, w.Xs, n, w.gemm_work,
                    w.gemm_work_elems, s));                                 // A^T X
    }
    URV_TRY(qpos_times_a(A, lda, m, n, Y, V, ldv, last, w, s));             // V = Qpos(Y), X = A V
  }
  return final_qr(m, n, U, ldu, R, ldr, w, s);
}

// The power iteration in 16-bit products / FP32 QRs, then the FP64 tail.
// A (FP64, ld lda) feeds the FP64 tail; the 16-bit casts read A32 (FP32, ld lda32)
// when the caller's matrix is FP32, else A.  FP16 casts scale their source by a
// power of two from its largest magnitude (FP16 overflows at 65504); BF16 has
// FP32's range and casts unscaled.
int run_factor_mixed(const double* A, int64_t lda, const float* A32, int64_t lda32, int64_t m, int64_t n,
                     int32_t q, uint64_t seed, double* U, double* R, double* V, const urv_opts& o,
                     const FactorWork& w, hipStream_t s) {
  const int64_t ldu = o.ldu ? o.ldu : m;
  const int64_t ldr = o.ldr ? o.ldr : n, ldv = o.ldv ? o.ldv : n, ldg = o.ldg ? o.ldg : n;
  const bool full = o.variant == URV_REORTH_FULL, none = o.variant == URV_REORTH_NONE;
  const bool bf16 = o.precision == URV_MIXED_BF16;
  const MixedWork& x = w.mx;
  const int64_t ldv16 = lowp_ld(n);
  unsigned* const amaxA = bf16 ? nullptr : x.amax;
  unsigned* const amaxB = bf16 ? nullptr : x.amax + 1;

  if (A32) {
    if (amaxA) URV_TRY(absmax<float>(A32, lda32, m, n, amaxA, s));
    URV_TRY(to_lowp<float>(bf16, A32, lda32, m, n, x.A16, x.lda16, s, amaxA));            // A^T W operand
    URV_TRY(to_lowp_transposed<float>(bf16, A32, lda32, m, n, x.At16, x.ldat16, s, amaxA)); // A V operand
  } else {
    if (amaxA) URV_TRY(absmax<double>(A, lda, m, n, amaxA, s));
    URV_TRY(to_lowp<double>(bf16, A, lda, m, n, x.A16, x.lda16, s, amaxA));
    URV_TRY(to_lowp_transposed<double>(bf16, A, lda, m, n, x.At16, x.ldat16, s, amaxA));
  }
  if (o.G)
    URV_TRY((convert<double, float>(o.G, ldg, n, n, x.V32, n, s)));
  else
    URV_TRY(launch_gaussian(x.V32, n, n, n, seed, 2u, true, s));
  if (o.orth_g) {
    URV_TRY(copy_matrix_f32(x.V32, n, x.Y32, n, n, n, s));
    URV_TRY(qpos_f32(x.Y32, n, n, x.V32, x.qr, s));
  }
  for (int32_t t = 0; t < q; ++t) {
    if (amaxB) URV_TRY(absmax<float>(x.V32, n, n, n, amaxB, s));
    URV_TRY(to_lowp<float>(bf16, x.V32, n, n, n, x.B16, ldv16, s, amaxB));
    URV_TRY(gemm_lowp(bf16, m, n, n, 1.f, x.At16, x.ldat16, x.B16, ldv16, 0.f, x.X32, m, s));  // X = A V
    const float* rhs = x.X32;
    if (full) {
      URV_TRY(qpos_f32(x.X32, m, n, x.W32, x.qr, s));                                      // W = Qpos(X)
      rhs = x.W32;
    }
    if (amaxB) URV_TRY(absmax<float>(rhs, m, m, n, amaxB, s));
    URV_TRY(to_lowp<float>(bf16, rhs, m, m, n, x.B16, x.lda16, s, amaxB));
    float* out = none ? x.V32 : x.Y32;
    URV_TRY(gemm_lowp(bf16, n, n, m, 1.f, x.A16, x.lda16, x.B16, x.lda16, 0.f, out, n, s));   // A^T W
    // V = Qpos(Y), in FP32 except after the last step: there the FP64 QR below takes Y
    // itself, since Qpos(Qpos(Y)) = Qpos(Y)
    if (!none && t + 1 < q) URV_TRY(qpos_f32(x.Y32, n, n, x.V32, x.qr, s));
  }
  // The last V = Qpos(.) in FP64 (delivering X = A V alongside): of Y after a power step
  // (FULL, HALF), of (A^T A)^q G (NONE), or of the starting V when q = 0; then the FP64
  // tail A V = U R.
  const float* vsrc = (q > 0 && !none) ? x.Y32 : x.V32;
  URV_TRY((convert<float, double>(vsrc, n, n, n, w.Xs, n, s)));
  URV_TRY(qpos_times_a(A, lda, m, n, w.Xs, V, ldv, true, w, s));
  return final_qr(m, n, U, ldu, R, ldr, w, s);
}

// m < n (Section 1): the ULV of B = A^T, transposed.  B = Ut Rt V_B^T is the
// tall factorisation; X = B V_B = Ut Rt, and X J (J the column reversal) =
// Ut (Rt J) = (Ut Q2) R2 with Rt J = Q2 R2.  So B = (Ut Q2 J)(J R2 J) V_B^T,
// J R2 J lower triangular, and A = V_B (J R2^T J) (Ut Q2 J)^T: U = V_B,
// R = J R2^T J, V = Ut Q2 J.
int run_wide(const double* A, int64_t m, int64_t n, int32_t q, uint64_t seed, double* U, double* R, double* V,
             const urv_opts& o, const FactorWork& w, const WideWork& x, bool mixed, hipStream_t s) {
  const int64_t lda = o.lda ? o.lda : m, ldu = o.ldu ? o.ldu : m;
  const int64_t ldr = o.ldr ? o.ldr : m, ldv = o.ldv ? o.ldv : n;
  URV_TRY(transpose_matrix(A, lda, m, n, x.B, n, s));                       // B = A^T
  urv_opts ob = o;
  ob.lda = n;
  ob.ldu = n;
  ob.ldr = m;
  ob.ldv = ldu;
  URV_TRY(mixed ? run_factor_mixed(x.B, n, nullptr, 0, n, m, q, seed, x.Ut, x.Rt, U, ob, w, s)
                : run_factor(x.B, n, m, q, seed, x.Ut, x.Rt, U, ob, w, s));  // U = V_B
  URV_TRY(reverse_cols(x.Rt, m, m, m, x.RJ, m, s));
  const char* wt = std::getenv("URV_WIDE_TARGET");
  if (!(wt && std::atoi(wt) == 0)) {
    // Rt J = Q2 R2 with Q2's reflectors applied to Ut as they come: Ut <- Ut Q2, beside the
    // chain, and Q2 never formed (URV_WIDE_TARGET=0: Q2 formed, then the product, for
    // tuning).  Measured on MI355X at 4000 x 8000, FP64 FULL q = 2: 113.0-113.1 ms
    // against 119.1-119.3.
    const QrTarget<double> t{x.Ut, n, n};
    URV_TRY(qr_pos<double>(x.RJ, m, m, m, nullptr, 0, x.R2, m, w.qr, s, &t, 1));
    URV_TRY(reverse_cols(x.Ut, n, n, m, V, ldv, s));                        // V = Ut Q2 J
    return transpose_reverse(x.R2, m, m, R, ldr, s);                        // R = J R2^T J
  }
  URV_TRY(qr_pos<double>(x.RJ, m, m, m, x.Q2, m, x.R2, m, w.qr, s));     // Rt J = Q2 R2
  URV_TRY(dgemm(false, false, n, m, m, 1.0, x.Ut, n, x.Q2, m, 0.0, x.T, n, x.gw, x.gw_elems, s));
  URV_TRY(reverse_cols(x.T, n, n, m, V, ldv, s));                           // V = Ut Q2 J
  return transpose_reverse(x.R2, m, m, R, ldr, s);                           // R = J R2^T J
}

// Runs the factorisation, then folds the panels' error flags into the device's
// status word; when blocking, waits for the stream and reports (and clears) it.
int factor_impl(const void* A, int64_t m, int64_t n, int32_t q, uint64_t seed, double* U, double* R, double* V,
                const urv_opts& o, bool blocking) {
  clear_last_error();
  URV_TRY(validate_factor(A, m, n, q, U, R, V, o));
  if (std::min(m, n) == 0) return URV_OK;
  hipStream_t s = static_cast<hipStream_t>(o.stream);
  const bool mixed = o.precision != URV_FP64 && q > 0;
  const bool a32 = (o.flags & URV_A_FP32) != 0;
  const bool wide = m < n;
  const int64_t mt = wide ? n : m, nt = wide ? m : n;  // the tall problem
  const int64_t lda = o.lda ? o.lda : m;
  const size_t need = work_bytes(m, n, mixed, a32);
  Arena a;
  bool owned = false;
  if (o.workspace) {
    a.base = static_cast<char*>(o.workspace);
    a.size = o.workspace_bytes;
  } else {
    void* p = nullptr;
    const hipError_t e = hipMallocAsync(&p, need, s);
    if (e != hipSuccess) {
      (void)hipGetLastError();  // clear the sticky error; the failure is reported below
      set_last_error(std::string("urv_factor: workspace allocation failed: ") + hipGetErrorString(e));
      return URV_ENOMEM;
    }
    a.base = static_cast<char*>(p);
    a.size = need;
    owned = true;
  }
  FactorWork w;
  carve_factor(a, mt, nt, mixed, w);
  WideWork x;
  if (wide) carve_wide(a, m, n, x);
  ExtraWork ex;
  carve_extra(a, m, n, a32, ex);
  int rc = a.overflow ? URV_EINVAL : URV_OK;
  if (rc == URV_OK && (o.flags & URV_CHECK_FINITE)) {
    // scan A before any other work; the answer needs the host
    set_u32_kernel<<<1, 1, 0, s>>>(ex.nonfinite, 0u);
    rc = hip_status(hipGetLastError(), "set_u32_kernel");
    const unsigned blocks = static_cast<unsigned>(std::min<int64_t>(ceil_div(m * n, 256), 2048));
    if (rc == URV_OK) {
      if (a32)
        nonfinite_kernel<float><<<blocks, 256, 0, s>>>(static_cast<const float*>(A), lda, m, n, ex.nonfinite);
      else
        nonfinite_kernel<double><<<blocks, 256, 0, s>>>(static_cast<const double*>(A), lda, m, n, ex.nonfinite);
      rc = hip_status(hipGetLastError(), "nonfinite_kernel");
    }
    unsigned bad = 0;
    if (rc == URV_OK) rc = hip_status(hipMemcpyAsync(&bad, ex.nonfinite, sizeof(bad), hipMemcpyDeviceToHost, s),
                                      "urv_factor: finiteness scan");
    if (rc == URV_OK) rc = hip_status(hipStreamSynchronize(s), "urv_factor: finiteness scan");
    if (rc == URV_OK && bad) {
      set_last_error("urv_factor: A holds a NaN or an infinity");
      rc = URV_ENONFINITE;
    }
  }
  // an FP32 A: its FP64 value for every FP64 step (exact)
  const double* A64 = static_cast<const double*>(A);
  urv_opts o64 = o;
  if (rc == URV_OK && a32) {
    rc = convert<float, double>(static_cast<const float*>(A), lda, m, n, ex.A64, m, s);
    A64 = ex.A64;
    o64.lda = m;
  }
  if (rc == URV_OK) rc = qr_clear_error_flag(w.qr, nt, s);
  if (rc == URV_OK && w.qr2.Y) rc = qr_clear_error_flag(w.qr2, nt, s);
  if (rc == URV_OK && mixed) rc = qr_clear_error_flag(w.mx.qr, nt, s);
  if (rc == URV_OK) {
    if (wide)
      rc = run_wide(A64, m, n, q, seed, U, R, V, o64, w, x, mixed, s);
    else if (mixed)
      rc = run_factor_mixed(A64, o64.lda ? o64.lda : m, a32 ? static_cast<const float*>(A) : nullptr, lda, m, n, q,
                            seed, U, R, V, o64, w, s);
    else
      rc = run_factor(A64, m, n, q, seed, U, R, V, o64, w, s);
  }
  if (rc == URV_OK)
    rc = fold_status(qr_error_flag(w.qr, nt), mixed ? qr_error_flag(w.mx.qr, nt) : nullptr, s,
                     w.qr2.Y ? qr_error_flag(w.qr2, nt) : nullptr);
  if (rc == URV_OK && blocking) rc = sync_status(s, "urv_factor");
  if (owned) {
    const hipError_t e = hipFreeAsync(a.base, s);
    if (e != hipSuccess && rc == URV_OK) rc = hip_status(e, "urv_factor");
  }
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

namespace urv {
namespace {
template <class T>
int qr_entry(T* X, int64_t m, int64_t n, int64_t ldx, T* Q, int64_t ldq, T* R, int64_t ldr,
             void* stream) {
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
  const size_t need = qr_work_bytes<T>(m, n);
  void* p = nullptr;
  URV_HIP(hipMallocAsync(&p, need, s));
  Arena a;
  a.base = static_cast<char*>(p);
  a.size = need;
  QrWorkT<T> w;
  qr_work_carve(a, m, n, w);
  int rc = qr_clear_error_flag(w, n, s);
  if (rc == URV_OK) rc = qr_pos<T>(X, m, n, ldx, Q, ldq, R, ldr, w, s);
  if (rc == URV_OK) rc = fold_status(qr_error_flag(w, n), nullptr, s);
  const hipError_t e = hipFreeAsync(p, s);
  if (e != hipSuccess && rc == URV_OK) rc = hip_status(e, "urv_qr_pos");
  return rc;
}
// Argument checks shared by urv_dgemm and urv_dgemm_noalloc.
int dgemm_args(const char* who, int64_t M, int64_t N, int64_t K, int32_t transA, int32_t transB, double alpha,
               const double* A, int64_t lda, const double* B, int64_t ldb, const double* C, int64_t ldc) {
  if (M < 0 || N < 0 || K < 0) {
    set_last_error(std::string(who) + ": negative size");
    return URV_EINVAL;
  }
  const int64_t arows = transA ? K : M, brows = transB ? N : K;
  if (lda < std::max<int64_t>(arows, 1) || ldb < std::max<int64_t>(brows, 1) ||
      ldc < std::max<int64_t>(M, 1)) {
    set_last_error(std::string(who) + ": leading dimension smaller than the row count");
    return URV_EINVAL;
  }
  if (M > 0 && N > 0 && (!C || (K > 0 && alpha != 0.0 && (!A || !B)))) {
    set_last_error(std::string(who) + ": null pointer");
    return URV_EINVAL;
  }
  return URV_OK;
}
}  // namespace
}  // namespace urv

using namespace urv;

extern "C" {

void urv_opts_init(urv_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->variant = URV_REORTH_FULL;
  o->precision = URV_FP64;
}

int urv_factor_ex(const void* A, int64_t m, int64_t n, int32_t q, uint64_t seed, double* U,
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
  if (m <= 0 || n <= 0 || q < 0) return 0;
  const bool mixed = opts && opts->precision != URV_FP64 && q > 0;
  return work_bytes(m, n, mixed, opts && (opts->flags & URV_A_FP32) != 0);
}

int urv_timing(int32_t enable) { return timing_enable(enable != 0); }

int urv_timing_read(int32_t cls, double* ms, int64_t* launches, double* flops) {
  clear_last_error();
  return timing_read(cls, ms, launches, flops);
}

int urv_sync_status(void* stream) {
  clear_last_error();
  return sync_status(static_cast<hipStream_t>(stream), "urv_sync_status");
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
  URV_TRY(dgemm_args("urv_dgemm", M, N, K, transA, transB, alpha, A, lda, B, ldb, C, ldc));
  if (M == 0 || N == 0) return URV_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t we = dgemm_work_elems(M, N, K);
  double* work = nullptr;
  if (we) URV_HIP(hipMallocAsync(reinterpret_cast<void**>(&work), we * sizeof(double), s));
  int rc = dgemm(transA != 0, transB != 0, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, work, we, s);
  if (work) {
    const hipError_t e = hipFreeAsync(work, s);
    if (e != hipSuccess && rc == URV_OK) rc = hip_status(e, "urv_dgemm");
  }
  return rc;
}

int urv_dgemm_noalloc(int32_t transA, int32_t transB, int64_t M, int64_t N, int64_t K, double alpha,
                      const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                      int64_t ldc, void* stream) {
  clear_last_error();
  URV_TRY(dgemm_args("urv_dgemm_noalloc", M, N, K, transA, transB, alpha, A, lda, B, ldb, C, ldc));
  if (M == 0 || N == 0) return URV_OK;
  const size_t we = dgemm_work_elems(M, N, K);
  if (we * sizeof(double) > kStaticScratchBytes) {
    set_last_error("urv_dgemm_noalloc: this shape's split-K partial sums need " +
                   std::to_string(we * sizeof(double)) + " bytes, more than the " +
                   std::to_string(kStaticScratchBytes) + "-byte static scratch");
    return URV_EINVAL;
  }
  double* work = nullptr;
  if (we) {
    DeviceStatics d;
    URV_TRY(device_statics(&d));
    work = d.scratch;
  }
  return dgemm(transA != 0, transB != 0, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, work, we,
               static_cast<hipStream_t>(stream));
}

int urv_qr_pos(double* X, int64_t m, int64_t n, int64_t ldx, double* Q, int64_t ldq, double* R,
               int64_t ldr, void* stream) {
  return qr_entry<double>(X, m, n, ldx, Q, ldq, R, ldr, stream);
}

int urv_qr_pos_f32(float* X, int64_t m, int64_t n, int64_t ldx, float* Q, int64_t ldq, float* R,
                   int64_t ldr, void* stream) {
  return qr_entry<float>(X, m, n, ldx, Q, ldq, R, ldr, stream);
}

int urv_metrics(const double* A, int64_t m, int64_t n, const double* U, const double* R,
                const double* V, double* out, double* ek, void* stream) {
  clear_last_error();
  if (n <= 0 || m <= 0 || !A || !U || !R || !V || !out) {
    set_last_error("urv_metrics: need m, n > 0 and non-null pointers");
    return URV_EINVAL;
  }
  return metrics(A, m, n, U, R, V, out, ek, static_cast<hipStream_t>(stream));
}

int64_t urv_max_rows(void) { return kMaxRows; }

const char* urv_strerror(int code) {
  switch (code) {
    case URV_OK: return "success";
    case URV_EINVAL: return "invalid argument";
    case URV_ENOMEM: return "device memory allocation failed";
    case URV_EDEVICE: return "device (HIP) error";
    case URV_ENOTSUP: return "unsupported argument combination";
    case URV_ENONFINITE: return "non-finite input";
    default: return "unknown status";
  }
}

const char* urv_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
