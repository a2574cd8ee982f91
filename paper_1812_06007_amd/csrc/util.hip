// Strided copies and the FP64 checks of a factorisation: relative
// reconstruction error, orthogonality of U and V, and the Frobenius norms of
// the trailing blocks R22 of eq. (blocks) for every k -- the rank-k errors
// plotted in Section 5.  Reductions are two-pass with a fixed assignment of
// elements to threads, so the checks are bitwise reproducible.
#include "common.hpp"

#include <vector>

namespace urv {
namespace {

template <class T>
__global__ void copy_kernel(const T* __restrict__ src, int64_t lds, T* __restrict__ dst,
                            int64_t ldd, int64_t rows, int64_t cols) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t i = idx % rows, j = idx / rows;
  dst[i + j * ldd] = src[i + j * lds];
}

// dst (cols x rows) = src^T, through 32 x 32 LDS tiles (both sides coalesced).
__global__ __launch_bounds__(256) void transpose_kernel(const double* __restrict__ src, int64_t lds,
                                                        int64_t rows, int64_t cols,
                                                        double* __restrict__ dst, int64_t ldd) {
  __shared__ double tile[32][33];
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * 32, j0 = static_cast<int64_t>(blockIdx.y) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + tx, j = j0 + r;
    if (i < rows && j < cols) tile[r][tx] = src[i + j * lds];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t j = j0 + tx, i = i0 + r;  // dst(j, i) = src(i, j)
    if (i < rows && j < cols) dst[j + i * ldd] = tile[tx][r];
  }
}

template <class T>
__global__ void identity_kernel(T* __restrict__ Z, int64_t rows, int64_t cols, int64_t ld) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t i = idx % rows, j = idx / rows;
  Z[i + j * ld] = (i == j) ? T(1) : T(0);
}

// Z(:, j) *= sign(X(j, j)) for j < n, sign(0) = +1.
template <class T>
__global__ void scale_cols_sign_kernel(T* __restrict__ Z, int64_t rows, int64_t n, int64_t ldz,
                                       const T* __restrict__ X, int64_t ldx) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= rows * n) return;
  const int64_t i = idx % rows, j = idx / rows;
  if (X[j + j * ldx] < T(0)) Z[i + j * ldz] = -Z[i + j * ldz];
}

constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;

// partial[b] = sum of (X(i,j) - [i==j] * diag)^2 over elements idx = b*T + t + k*B*T.
__global__ __launch_bounds__(kRedThreads) void sumsq_partial_kernel(
    const double* __restrict__ X, int64_t ld, int64_t rows, int64_t cols, double diag,
    double* __restrict__ partial) {
  __shared__ double red[kRedThreads];
  const int64_t total = rows * cols;
  double s = 0.0;
  for (int64_t idx = blockIdx.x * static_cast<int64_t>(kRedThreads) + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(kRedBlocks) * kRedThreads) {
    const int64_t i = idx % rows, j = idx / rows;
    double v = X[i + j * ld];
    if (i == j) v -= diag;
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kRedThreads) void sum_final_kernel(const double* __restrict__ partial,
                                                                 int count, double* __restrict__ out) {
  __shared__ double red[kRedThreads];
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += kRedThreads) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// rowsq[i] = sum_{j >= i} R(i,j)^2
__global__ void upper_row_sumsq_kernel(const double* __restrict__ R, int64_t ld, int64_t n,
                                       double* __restrict__ rowsq) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t j = i; j < n; ++j) s += R[i + j * ld] * R[i + j * ld];
  rowsq[i] = s;
}

// ek[k] = sqrt(sum_{i >= k} rowsq[i]), ek[n] = 0 (one thread: sequential suffix sum).
__global__ void suffix_sqrt_kernel(const double* __restrict__ rowsq, int64_t n, double* __restrict__ ek) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double acc = 0.0;
  ek[n] = 0.0;
  for (int64_t k = n - 1; k >= 0; --k) {
    acc += rowsq[k];
    ek[k] = sqrt(acc);
  }
}

// out[0] = sqrt(s0/s1), out[1] = sqrt(s2), out[2] = sqrt(s3), out[3] = sqrt(s1)
__global__ void finalize_metrics_kernel(const double* __restrict__ sums, double* __restrict__ out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  out[3] = sqrt(sums[1]);
  out[0] = sqrt(sums[0]) / out[3];
  out[1] = sqrt(sums[2]);
  out[2] = sqrt(sums[3]);
}

int sumsq(const double* X, int64_t ld, int64_t rows, int64_t cols, double diag, double* partial,
          double* out, hipStream_t s) {
  sumsq_partial_kernel<<<kRedBlocks, kRedThreads, 0, s>>>(X, ld, rows, cols, diag, partial);
  URV_LAUNCHED("sumsq_partial_kernel");
  sum_final_kernel<<<1, kRedThreads, 0, s>>>(partial, kRedBlocks, out);
  URV_LAUNCHED("sum_final_kernel");
  return URV_OK;
}

}  // namespace

namespace {
struct TimedLaunch {
  hipEvent_t a = nullptr, b = nullptr;
  int cls = -1;
  double flops = 0;
};
struct Timing {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<TimedLaunch> pending;
  double ms[kTimedClasses] = {};
  int64_t launches[kTimedClasses] = {};
  double flops[kTimedClasses] = {};
};
Timing g_timing;

hipEvent_t take_event() {
  if (!g_timing.pool.empty()) {
    hipEvent_t e = g_timing.pool.back();
    g_timing.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Adds the completed launches to the totals (the caller has synchronised).
void timing_resolve() {
  std::vector<TimedLaunch> left;
  for (TimedLaunch& t : g_timing.pending) {
    float ms = 0.f;
    if (t.cls >= 0 && t.a && t.b && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      g_timing.ms[t.cls] += ms;
      g_timing.launches[t.cls] += 1;
      g_timing.flops[t.cls] += t.flops;
    } else if (t.cls >= 0) {
      (void)hipGetLastError();  // not complete yet: keep it
      left.push_back(t);
      continue;
    }
    if (t.a) g_timing.pool.push_back(t.a);
    if (t.b) g_timing.pool.push_back(t.b);
  }
  g_timing.pending.swap(left);
}
}  // namespace

int timing_begin(hipStream_t s) {
  std::lock_guard<std::mutex> lock(g_timing.mu);
  if (!g_timing.on) return -1;
  TimedLaunch t;
  t.a = take_event();
  if (!t.a || hipEventRecord(t.a, s) != hipSuccess) return -1;
  g_timing.pending.push_back(t);
  return static_cast<int>(g_timing.pending.size()) - 1;
}

void timing_end(int token, int cls, double flops, hipStream_t s) {
  if (token < 0) return;
  std::lock_guard<std::mutex> lock(g_timing.mu);
  if (token >= static_cast<int>(g_timing.pending.size())) return;
  TimedLaunch& t = g_timing.pending[token];
  t.b = take_event();
  if (!t.b || hipEventRecord(t.b, s) != hipSuccess) return;
  t.cls = cls;
  t.flops = flops;
}

int timing_enable(bool on) {
  std::lock_guard<std::mutex> lock(g_timing.mu);
  if (on) {
    for (int c = 0; c < kTimedClasses; ++c) {
      g_timing.ms[c] = 0;
      g_timing.launches[c] = 0;
      g_timing.flops[c] = 0;
    }
    for (TimedLaunch& t : g_timing.pending) {
      if (t.a) g_timing.pool.push_back(t.a);
      if (t.b) g_timing.pool.push_back(t.b);
    }
    g_timing.pending.clear();
  }
  g_timing.on = on;
  return URV_OK;
}

int timing_read(int cls, double* ms, int64_t* launches, double* flops) {
  if (cls < 0 || cls >= kTimedClasses || !ms || !launches || !flops) {
    set_last_error("urv_timing_read: unknown class or null pointer");
    return URV_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_timing.mu);
  timing_resolve();
  *ms = g_timing.ms[cls];
  *launches = g_timing.launches[cls];
  *flops = g_timing.flops[cls];
  return URV_OK;
}

int side_stream(SideStream* out) {
  constexpr int kMaxDevices = 64;
  static std::mutex init_mu;
  static SideStream table[kMaxDevices];
  static std::mutex use_mu[kMaxDevices];
  int dev = 0;
  URV_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_last_error("side_stream: device index out of range");
    return URV_EDEVICE;
  }
  std::lock_guard<std::mutex> g(init_mu);
  SideStream& e = table[dev];
  if (e.stream == nullptr) {
    hipStream_t st[3];
    for (auto& x : st) URV_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    hipEvent_t ev[9];
    for (auto& x : ev) URV_HIP(hipEventCreateWithFlags(&x, hipEventDisableTiming));
    e.ev_defer = ev[7];
    e.ev_defer_done = ev[8];
    e.ev_next = ev[0];
    e.ev_fact = ev[1];
    e.ev_fact2 = ev[6];
    e.ev_tgt = ev[2];
    e.ev_near = ev[3];
    e.ev_bulk = ev[4];
    e.ev_pair = ev[5];
    e.stream3 = st[1];
    e.stream4 = st[2];
    e.mu = &use_mu[dev];
    e.stream = st[0];
  }
  *out = e;
  return URV_OK;
}

int transpose_matrix(const double* src, int64_t lds, int64_t rows, int64_t cols, double* dst, int64_t ldd,
                     hipStream_t s) {
  if (rows == 0 || cols == 0) return URV_OK;
  const dim3 grid(static_cast<unsigned>(ceil_div(rows, 32)), static_cast<unsigned>(ceil_div(cols, 32)));
  transpose_kernel<<<grid, 256, 0, s>>>(src, lds, rows, cols, dst, ldd);
  URV_LAUNCHED("transpose_kernel");
  return URV_OK;
}

template <class T>
int set_identity(T* Z, int64_t rows, int64_t cols, int64_t ld, hipStream_t s) {
  if (rows == 0 || cols == 0) return URV_OK;
  identity_kernel<T><<<static_cast<unsigned>(ceil_div(rows * cols, 256)), 256, 0, s>>>(Z, rows, cols, ld);
  URV_LAUNCHED("identity_kernel");
  return URV_OK;
}
template int set_identity<double>(double*, int64_t, int64_t, int64_t, hipStream_t);
template int set_identity<float>(float*, int64_t, int64_t, int64_t, hipStream_t);

template <class T>
int scale_cols_sign(T* Z, int64_t rows, int64_t n, int64_t ldz, const T* X, int64_t ldx, hipStream_t s) {
  if (rows == 0 || n == 0) return URV_OK;
  scale_cols_sign_kernel<T><<<static_cast<unsigned>(ceil_div(rows * n, 256)), 256, 0, s>>>(Z, rows, n, ldz, X,
                                                                                           ldx);
  URV_LAUNCHED("scale_cols_sign_kernel");
  return URV_OK;
}
template int scale_cols_sign<double>(double*, int64_t, int64_t, int64_t, const double*, int64_t, hipStream_t);
template int scale_cols_sign<float>(float*, int64_t, int64_t, int64_t, const float*, int64_t, hipStream_t);

int copy_matrix(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                int64_t cols, hipStream_t s) {
  if (rows == 0 || cols == 0) return URV_OK;
  copy_kernel<double><<<static_cast<unsigned>(ceil_div(rows * cols, 256)), 256, 0, s>>>(src, lds, dst,
                                                                                         ldd, rows, cols);
  URV_LAUNCHED("copy_kernel");
  return URV_OK;
}

// dst(:, j) = src(:, cols - 1 - j): the columns in reverse order.
__global__ void reverse_cols_kernel(const double* __restrict__ src, int64_t lds, int64_t rows, int64_t cols,
                                    double* __restrict__ dst, int64_t ldd) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t i = idx % rows, j = idx / rows;
  dst[i + j * ldd] = src[i + (cols - 1 - j) * lds];
}

// dst(i, j) = src(p - 1 - j, p - 1 - i) for p x p: J src^T J with J the reversal.
__global__ void transpose_reverse_kernel(const double* __restrict__ src, int64_t lds, int64_t p,
                                         double* __restrict__ dst, int64_t ldd) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= p * p) return;
  const int64_t i = idx % p, j = idx / p;
  dst[i + j * ldd] = src[(p - 1 - j) + (p - 1 - i) * lds];
}

int reverse_cols(const double* src, int64_t lds, int64_t rows, int64_t cols, double* dst, int64_t ldd,
                 hipStream_t s) {
  if (rows == 0 || cols == 0) return URV_OK;
  reverse_cols_kernel<<<static_cast<unsigned>(ceil_div(rows * cols, 256)), 256, 0, s>>>(src, lds, rows, cols, dst,
                                                                                         ldd);
  URV_LAUNCHED("reverse_cols_kernel");
  return URV_OK;
}

int transpose_reverse(const double* src, int64_t lds, int64_t p, double* dst, int64_t ldd, hipStream_t s) {
  if (p == 0) return URV_OK;
  transpose_reverse_kernel<<<static_cast<unsigned>(ceil_div(p * p, 256)), 256, 0, s>>>(src, lds, p, dst, ldd);
  URV_LAUNCHED("transpose_reverse_kernel");
  return URV_OK;
}

int copy_matrix_f32(const float* src, int64_t lds, float* dst, int64_t ldd, int64_t rows, int64_t cols,
                    hipStream_t s) {
  if (rows == 0 || cols == 0) return URV_OK;
  copy_kernel<float><<<static_cast<unsigned>(ceil_div(rows * cols, 256)), 256, 0, s>>>(src, lds, dst,
                                                                                        ldd, rows, cols);
  URV_LAUNCHED("copy_kernel");
  return URV_OK;
}

int metrics(const double* A, int64_t m, int64_t n, const double* U, const double* R,
            const double* V, double* out_host, double* ek_host, hipStream_t s) {
  // U m x p, R p x p, V n x p with p = min(m, n).
  // Workspace: UR (m x p), E (m x n), Gram (p x p), partials, scalars, rowsq, ek.
  const int64_t p = std::min(m, n);
  const size_t mp = static_cast<size_t>(m) * p, mn = static_cast<size_t>(m) * n, pp = static_cast<size_t>(p) * p;
  const size_t gw = std::max({dgemm_work_elems(m, p, p), dgemm_work_elems(m, n, p), dgemm_work_elems(p, p, m),
                              dgemm_work_elems(p, p, n)});
  const size_t total = mp + mn + pp + kRedBlocks + 8 + 2 * (p + 1) + gw;
  double* buf = nullptr;
  URV_HIP(hipMallocAsync(reinterpret_cast<void**>(&buf), total * sizeof(double), s));
  double* UR = buf;
  double* E = UR + mp;
  double* Gm = E + mn;
  double* part = Gm + pp;
  double* scal = part + kRedBlocks;
  double* rowsq = scal + 8;
  double* ek = rowsq + (p + 1);
  double* gwork = ek + (p + 1);
  int rc = URV_OK;
  do {
    if ((rc = dgemm(false, false, m, p, p, 1.0, U, m, R, p, 0.0, UR, m, gwork, gw, s))) break;
    if ((rc = copy_matrix(A, m, E, m, m, n, s))) break;
    if ((rc = dgemm(false, true, m, n, p, -1.0, UR, m, V, n, 1.0, E, m, gwork, gw, s))) break;
    if ((rc = sumsq(E, m, m, n, 0.0, part, scal + 0, s))) break;
    if ((rc = sumsq(A, m, m, n, 0.0, part, scal + 1, s))) break;
    if ((rc = dgemm(true, false, p, p, m, 1.0, U, m, U, m, 0.0, Gm, p, gwork, gw, s))) break;
    if ((rc = sumsq(Gm, p, p, p, 1.0, part, scal + 2, s))) break;
    if ((rc = dgemm(true, false, p, p, n, 1.0, V, n, V, n, 0.0, Gm, p, gwork, gw, s))) break;
    if ((rc = sumsq(Gm, p, p, p, 1.0, part, scal + 3, s))) break;
    upper_row_sumsq_kernel<<<static_cast<unsigned>(ceil_div(p, 256)), 256, 0, s>>>(R, p, p, rowsq);
    suffix_sqrt_kernel<<<1, 1, 0, s>>>(rowsq, p, ek);
    finalize_metrics_kernel<<<1, 1, 0, s>>>(scal, scal + 4);
    if (hipGetLastError() != hipSuccess) { rc = URV_EDEVICE; break; }
    if (hipMemcpyAsync(out_host, scal + 4, 4 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) { rc = URV_EDEVICE; break; }
    if (ek_host && hipMemcpyAsync(ek_host, ek, (p + 1) * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) { rc = URV_EDEVICE; break; }
    if (hipStreamSynchronize(s) != hipSuccess) { rc = URV_EDEVICE; break; }
  } while (false);
  if (hipFreeAsync(buf, s) != hipSuccess && rc == URV_OK) rc = URV_EDEVICE;
  if (rc == URV_EDEVICE) set_last_error("metrics: HIP error");
  return rc;
}

}  // namespace urv
