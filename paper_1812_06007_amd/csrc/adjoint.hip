// Reverse-mode derivative of PowerURV with the Gaussian G held fixed.
//
// The paper (Section 3, eqs. power and powerqr) defines the forward chain
//   V_0 = G;  for t = 1..q:  X_t = A V_{t-1},  (W_t, Rw_t) = Qpos(X_t),
//                            Y_t = A^T W_t,    (V_t, Rv_t) = Qpos(Y_t)
//   (U, R) = Qpos(A V_q),  V = V_q
// (HALF: Y_t = A^T X_t, no W; q = 0: V = Qpos(G), a constant).  It does not
// differentiate it.  The adjoint of one QR X = Q R (m >= n, diag(R) != 0) is
// the published one (Walter & Lehmann 2018; Seeger et al. 2017):
//   M = R Rb^T - Qb^T Q,   S = the symmetric matrix from M's lower triangle,
//   Xb = (Qb + Q S) R^{-T}.
// For square X (m = n) the last column of Qb + Q S is (I - Q Q^T) Qb(:,n) +
// R(n,n) Q Rb(:,n), whose first term vanishes: Xb(:,n) = Q Rb(:,n) is set
// directly and the solve starts from it.  The last pivot of a numerically
// singular square iterate is rounding noise (it can be exactly zero), and the
// quotient of two noise terms would otherwise enter every other column.
// The reverse sweep visits the products in the opposite order: P = A B gives
// Ab += Pb B^T, Bb = A^T Pb; P = A^T B gives Ab += B Pb^T, Bb = A Pb.
//
// Kernels: the products are the MFMA GEMM of gemm.hip; R^{-T} is a recursive
// blocked solve whose off-diagonal blocks are GEMMs and whose 64-column
// diagonal blocks are solved by trsm_rt_block_kernel (one wave per row, the
// block of R in LDS); the QRs are qr_pos.  The tape keeps what the reverse
// sweep reads (every Q and R of the power steps, or only the V's, or nothing,
// in which case the sweep recomputes the V's from G).
#include "common.hpp"

#include <cstring>
#include <vector>

namespace urv {
namespace {

constexpr int kTrsmNB = 64;       // columns of a diagonal block of the solve
constexpr int kTrsmThreads = 512;  // threads per workgroup of the block solve: 8 waves, a row each
constexpr int kLossBlocks = 512;
constexpr int kLossThreads = 256;

template <class T>
__global__ void copy2d_kernel(const T* __restrict__ src, int64_t lds, T* __restrict__ dst, int64_t ldd,
                              int64_t rows, int64_t cols) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t i = idx % rows, j = idx / rows;
  dst[i + j * ldd] = src[i + j * lds];
}

template <class T>
__global__ void fill2d_kernel(T* __restrict__ dst, int64_t ldd, int64_t rows, int64_t cols, T v) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= rows * cols) return;
  dst[idx % rows + (idx / rows) * ldd] = v;
}

// M(i, j) = M(j, i) for i < j: the symmetric matrix taken from the lower
// triangle.  Lanes read only the lower triangle and write only the upper one.
template <class T>
__global__ void copyltu_kernel(T* __restrict__ M, int64_t n, int64_t ld) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx % n, j = idx / n;
  if (i < j) M[i + j * ld] = M[j + i * ld];
}

// X = B R^{-T} in place for one diagonal block: nb <= 64 columns of B (m rows)
// and the nb x nb upper triangle of R.  Column j of X R^T is the sum over
// l >= j of X(:,l) R(j,l), so a row takes its last unknown first and removes
// it from the others: x_j = b_j / R(j,j), b_l -= x_j R(l,j) for l < j.  One
// wave per row, lane l holding b_l: each step broadcasts b_j from lane j and
// every lane l < j updates at once, so a row costs nb dependent steps instead
// of nb^2 / 2 (the arithmetic of every element, and its order, are those of a
// row solved by one lane).  With last_given, column nb - 1 of B already holds its x.
template <class T>
__device__ inline T lane_value(T v, int j);
template <>
__device__ inline float lane_value<float>(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}
template <>
__device__ inline double lane_value<double>(double v, int j) {
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), j);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), j);
  return __hiloint2double(hi, lo);
}

template <class T>
__global__ __launch_bounds__(kTrsmThreads) void trsm_rt_block_kernel(T* __restrict__ B, int64_t ldb, int64_t m,
                                                                     int nb, const T* __restrict__ R,
                                                                     int64_t ldr, int last_given) {
  __shared__ T Rs[kTrsmNB][kTrsmNB + 1];  // Rs[j][l] = R(l, j): row j holds column j of R
  for (int e = threadIdx.x; e < kTrsmNB * kTrsmNB; e += kTrsmThreads) {
    const int l = e % kTrsmNB, j = e / kTrsmNB;
    Rs[j][l] = (l < nb && j < nb && l <= j) ? R[l + j * ldr] : T(0);
  }
  __syncthreads();
  constexpr int kWaves = kTrsmThreads / 64;
  const int l = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kWaves + wave; i < m;
       i += static_cast<int64_t>(gridDim.x) * kWaves) {
    T b = (l < nb) ? B[i + l * ldb] : T(0);
    for (int j = nb - 1; j >= 0; --j) {
      const T bj = lane_value<T>(b, j);
      const T x = (last_given && j == nb - 1) ? bj : bj / Rs[j][j];
      if (l == j) b = x;
      else if (l < j) b = fma(-x, Rs[j][l], b);
    }
    if (l < nb) B[i + l * ldb] = b;
  }
}

// partial[b] = sum of E^2 over a fixed set of elements (in double); then one
// workgroup adds the partials in order: a deterministic ||E||_F^2.
template <class T>
__global__ __launch_bounds__(kLossThreads) void sumsq_partial_kernel(const T* __restrict__ E, int64_t ld,
                                                                     int64_t rows, int64_t cols,
                                                                     double* __restrict__ partial) {
  __shared__ double red[kLossThreads];
  const int64_t total = rows * cols;
  double s = 0.0;
  for (int64_t idx = blockIdx.x * static_cast<int64_t>(kLossThreads) + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(kLossBlocks) * kLossThreads) {
    const double v = static_cast<double>(E[idx % rows + (idx / rows) * ld]);
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kLossThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kLossThreads) void sum_partials_kernel(const double* __restrict__ partial, int count,
                                                                    double* __restrict__ out) {
  __shared__ double red[kLossThreads];
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += kLossThreads) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kLossThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

template <class T>
__global__ void scale_kernel2d(T* __restrict__ X, int64_t ld, int64_t rows, int64_t cols, T a) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= rows * cols) return;
  X[idx % rows + (idx / rows) * ld] *= a;
}

unsigned grid_for(int64_t elems, int threads = 256) {
  return static_cast<unsigned>(ceil_div(elems, threads));
}

template <class T>
int copy2d(const T* src, int64_t lds, T* dst, int64_t ldd, int64_t rows, int64_t cols, hipStream_t s) {
  if (rows * cols == 0) return URV_OK;
  copy2d_kernel<T><<<grid_for(rows * cols), 256, 0, s>>>(src, lds, dst, ldd, rows, cols);
  URV_LAUNCHED("copy2d_kernel");
  return URV_OK;
}

template <class T>
int fill2d(T* dst, int64_t ldd, int64_t rows, int64_t cols, T v, hipStream_t s) {
  if (rows * cols == 0) return URV_OK;
  fill2d_kernel<T><<<grid_for(rows * cols), 256, 0, s>>>(dst, ldd, rows, cols, v);
  URV_LAUNCHED("fill2d_kernel");
  return URV_OK;
}

// ---------------------------------------------------------------- workspace
template <class T>
struct GradWork {
  T* gemm_work = nullptr;
  size_t gemm_work_elems = 0;
  QrWorkT<T> qr;
  T* Xw = nullptr;    // m x n: QR input (overwritten by the QR)
  T* Yw = nullptr;    // n x n: QR input
  T* Xb = nullptr;    // m x n
  T* Pb = nullptr;    // m x n
  T* Vb = nullptr;    // n x n
  T* Yb = nullptr;    // n x n
  T* M = nullptr;     // n x n
  // one power step recomputed by the reverse sweep (tapes without the Q's and R's)
  T* P = nullptr;     // m x n: W_t (FULL) or X_t (HALF)
  T* Rw = nullptr;    // n x n
  T* Vt = nullptr;    // n x n
  T* Rv = nullptr;    // n x n
  T* Vp = nullptr;    // n x n: V_{t-1} recomputed from G
  double* loss_partial = nullptr;  // kLossBlocks
};

template <class T>
void carve_grad(Arena& a, int64_t m, int64_t n, GradWork<T>& w) {
  w.gemm_work_elems = std::max({gemm_work_elems(m, n, n), gemm_work_elems(n, n, m), gemm_work_elems(m, n, m)});
  w.gemm_work = a.take<T>(w.gemm_work_elems);
  qr_work_carve(a, m, n, w.qr);
  const size_t mn = static_cast<size_t>(m) * n, nn = static_cast<size_t>(n) * n;
  w.Xw = a.take<T>(mn);
  w.Yw = a.take<T>(nn);
  w.Xb = a.take<T>(mn);
  w.Pb = a.take<T>(mn);
  w.Vb = a.take<T>(nn);
  w.Yb = a.take<T>(nn);
  w.M = a.take<T>(nn);
  w.P = a.take<T>(mn);
  w.Rw = a.take<T>(nn);
  w.Vt = a.take<T>(nn);
  w.Rv = a.take<T>(nn);
  w.Vp = a.take<T>(nn);
  w.loss_partial = a.take<double>(kLossBlocks);
}

template <class T>
size_t grad_bytes(int64_t m, int64_t n) {
  Arena a;
  GradWork<T> w;
  carve_grad(a, m, n, w);
  return a.used;
}

// What the tape holds for power step t (1-based): P_t (W_t or X_t), Rw_t
// (FULL), Rv_t, and V_t for t < q (V_0 = G and V_q = V are the caller's).
template <class T>
struct StepView {
  T* P = nullptr;
  T* Rw = nullptr;
  T* Rv = nullptr;
  T* V = nullptr;
};

template <class T>
struct TapeLayout {
  int mode = URV_TAPE_ALL;
  std::vector<StepView<T>> steps;  // index t - 1
};

template <class T>
void carve_tape(Arena& a, int64_t m, int64_t n, int32_t q, bool full, int mode, TapeLayout<T>& tl) {
  tl.mode = mode;
  tl.steps.assign(static_cast<size_t>(q), StepView<T>{});
  const size_t mn = static_cast<size_t>(m) * n, nn = static_cast<size_t>(n) * n;
  for (int32_t t = 1; t <= q; ++t) {
    StepView<T>& v = tl.steps[t - 1];
    if (mode == URV_TAPE_ALL) {
      v.P = a.take<T>(mn);
      if (full) v.Rw = a.take<T>(nn);
      v.Rv = a.take<T>(nn);
    }
    if (mode != URV_TAPE_NONE && t < q) v.V = a.take<T>(nn);
  }
}

template <class T>
size_t tape_bytes(int64_t m, int64_t n, int32_t q, bool full, int mode) {
  Arena a;
  TapeLayout<T> tl;
  carve_tape(a, m, n, q, full, mode, tl);
  return a.used;
}

// ---------------------------------------------------------------- pieces
template <class T>
int gemm_w(bool ta, bool tb, int64_t M, int64_t N, int64_t K, T alpha, const T* A, int64_t lda, const T* B,
           int64_t ldb, T beta, T* C, int64_t ldc, const GradWork<T>& w, hipStream_t s) {
  return gemm<T>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, w.gemm_work, w.gemm_work_elems, s);
}

// B (m x n, ldb) <- B R^{-T}, R upper triangular n x n.  The trailing block
// is solved first; X2 R12^T is then removed from the leading columns by one
// GEMM, and the leading block is solved.  With last_given, B's last column
// already holds its x (no division by R(n,n)).
template <class T>
int trsm_rt(T* B, int64_t ldb, int64_t m, int64_t n, const T* R, int64_t ldr, const GradWork<T>& w,
            hipStream_t s, bool last_given = false) {
  if (m == 0 || n == 0) return URV_OK;
  if (n <= kTrsmNB) {
    const unsigned blocks = static_cast<unsigned>(std::min<int64_t>(ceil_div(m, kTrsmThreads / 64), 1024));
    trsm_rt_block_kernel<T><<<blocks, kTrsmThreads, 0, s>>>(B, ldb, m, static_cast<int>(n), R, ldr,
                                                              last_given ? 1 : 0);
    URV_LAUNCHED("trsm_rt_block_kernel");
    return URV_OK;
  }
  const int64_t n1 = std::max<int64_t>(kTrsmNB, (n / 2) / kTrsmNB * kTrsmNB);
  T* B2 = B + n1 * ldb;
  URV_TRY(trsm_rt<T>(B2, ldb, m, n - n1, R + n1 + n1 * ldr, ldr, w, s, last_given));  // X2 = B2 R22^{-T}
  URV_TRY(gemm_w<T>(false, true, m, n1, n - n1, T(-1), B2, ldb, R + n1 * ldr, ldr, T(1), B, ldb, w, s));  // B1 -= X2 R12^T
  return trsm_rt<T>(B, ldb, m, n1, R, ldr, w, s);                                  // X1 = B1 R11^{-T}
}

// Xb (m x n) = adjoint of X = Q R given Qb (may be null) and Rb (may be null).
template <class T>
int qr_adjoint(const T* Q, const T* R, int64_t m, int64_t n, const T* Qb, const T* Rb, T* Xb,
               const GradWork<T>& w, hipStream_t s) {
  if (!Qb && !Rb) return fill2d<T>(Xb, m, m, n, T(0), s);
  if (Rb) URV_TRY(gemm_w<T>(false, true, n, n, n, T(1), R, n, Rb, n, T(0), w.M, n, w, s));          // R Rb^T
  if (Qb) URV_TRY(gemm_w<T>(true, false, n, n, m, T(-1), Qb, m, Q, m, Rb ? T(1) : T(0), w.M, n, w, s));  // - Qb^T Q
  copyltu_kernel<T><<<grid_for(n * n), 256, 0, s>>>(w.M, n, n);
  URV_LAUNCHED("copyltu_kernel");
  if (Qb) URV_TRY(copy2d<T>(Qb, m, Xb, m, m, n, s));
  URV_TRY(gemm_w<T>(false, false, m, n, n, T(1), Q, m, w.M, n, Qb ? T(1) : T(0), Xb, m, w, s));     // + Q S
  const bool square = m == n;
  if (square) {  // Xb(:,n) = Q Rb(:,n): (I - Q Q^T) Qb(:,n) is zero for square Q
    T* xl = Xb + (n - 1) * m;
    if (Rb)
      URV_TRY(gemm_w<T>(false, false, m, 1, n, T(1), Q, m, Rb + (n - 1) * n, n, T(0), xl, m, w, s));
    else
      URV_TRY(fill2d<T>(xl, m, m, 1, T(0), s));
  }
  return trsm_rt<T>(Xb, m, m, n, R, n, w, s, square);                                             // R^{-T}
}

// One power step from V_in: P (W_t or X_t), Rw (FULL), then V_out = Qpos(A^T P), Rv.
// Rw and Rv may be null when only the V's are wanted.
template <class T>
int power_step(const T* A, int64_t m, int64_t n, bool full, const T* Vin, T* P, T* Rw, T* Vout, T* Rv,
               const GradWork<T>& w, hipStream_t s) {
  if (full) {
    URV_TRY(gemm_w<T>(false, false, m, n, n, T(1), A, m, Vin, n, T(0), w.Xw, m, w, s));          // X = A V
    URV_TRY(qr_pos<T>(w.Xw, m, n, m, P, m, Rw, n, w.qr, s));                                      // W = Qpos(X)
  } else {
    URV_TRY(gemm_w<T>(false, false, m, n, n, T(1), A, m, Vin, n, T(0), P, m, w, s));             // X = A V
  }
  URV_TRY(gemm_w<T>(true, false, n, n, m, T(1), A, m, P, m, T(0), w.Yw, n, w, s));               // Y = A^T P
  return qr_pos<T>(w.Yw, n, n, n, Vout, n, Rv, n, w.qr, s);                                       // V = Qpos(Y)
}

template <class T>
int forward_impl(const T* A, int64_t m, int64_t n, int32_t q, bool full, const T* G, T* U, T* R, T* V,
                 const TapeLayout<T>& tl, const GradWork<T>& w, hipStream_t s) {
  if (q == 0) {
    URV_TRY(copy2d<T>(G, n, w.Yw, n, n, n, s));
    URV_TRY(qr_pos<T>(w.Yw, n, n, n, V, n, nullptr, 0, w.qr, s));                                // V = Qpos(G)
  }
  const T* Vin = G;
  for (int32_t t = 1; t <= q; ++t) {
    const StepView<T>& sv = tl.steps[t - 1];
    T* P = sv.P ? sv.P : w.P;
    T* Vout = (t == q) ? V : (sv.V ? sv.V : (Vin == w.Vt ? w.Vp : w.Vt));
    URV_TRY(power_step<T>(A, m, n, full, Vin, P, sv.Rw, Vout, sv.Rv, w, s));
    Vin = Vout;
  }
  URV_TRY(gemm_w<T>(false, false, m, n, n, T(1), A, m, V, n, T(0), w.Xw, m, w, s));             // A V = U R
  return qr_pos<T>(w.Xw, m, n, m, U, m, R, n, w.qr, s);
}

template <class T>
int backward_impl(const T* A, int64_t m, int64_t n, int32_t q, bool full, const T* G, const T* U, const T* R,
                  const T* V, const TapeLayout<T>& tl, const T* dU, const T* dR, const T* dV, T* dA,
                  bool accumulate, const GradWork<T>& w, hipStream_t s) {
  const T acc0 = accumulate ? T(1) : T(0);
  URV_TRY(qr_adjoint<T>(U, R, m, n, dU, dR, w.Xb, w, s));                                          // final QR
  URV_TRY(gemm_w<T>(false, true, m, n, n, T(1), w.Xb, m, V, n, acc0, dA, m, w, s));              // Ab += Xb V^T
  if (q == 0) return URV_OK;                                                                      // V = Qpos(G)
  if (dV) URV_TRY(copy2d<T>(dV, n, w.Vb, n, n, n, s));
  URV_TRY(gemm_w<T>(true, false, n, n, m, T(1), A, m, w.Xb, m, dV ? T(1) : T(0), w.Vb, n, w, s)); // Vb = A^T Xb
  for (int32_t t = q; t >= 1; --t) {
    const StepView<T>& sv = tl.steps[t - 1];
    const T* Vin;
    const T *P, *Rw, *Vout, *Rv;
    if (tl.mode == URV_TAPE_ALL) {
      Vin = (t == 1) ? G : tl.steps[t - 2].V;
      P = sv.P;
      Rw = sv.Rw;
      Rv = sv.Rv;
      Vout = (t == q) ? V : sv.V;
    } else {
      if (t == 1) {
        Vin = G;
      } else if (tl.mode == URV_TAPE_V) {
        Vin = tl.steps[t - 2].V;
      } else {
        // V_{t-1} recomputed from G: t - 1 power steps, V's only
        const T* cur = G;
        for (int32_t u = 1; u < t; ++u) {
          T* out = (cur == w.Vp) ? w.Vt : w.Vp;
          URV_TRY(power_step<T>(A, m, n, full, cur, w.P, nullptr, out, nullptr, w, s));
          cur = out;
        }
        if (cur != w.Vp) URV_TRY(copy2d<T>(cur, n, w.Vp, n, n, n, s));
        Vin = w.Vp;
      }
      URV_TRY(power_step<T>(A, m, n, full, Vin, w.P, full ? w.Rw : nullptr, w.Vt, w.Rv, w, s));
      P = w.P;
      Rw = w.Rw;
      Rv = w.Rv;
      Vout = w.Vt;
    }
    URV_TRY(qr_adjoint<T>(Vout, Rv, n, n, w.Vb, nullptr, w.Yb, w, s));                           // V_t = Qpos(Y_t)
    URV_TRY(gemm_w<T>(false, true, m, n, n, T(1), P, m, w.Yb, n, T(1), dA, m, w, s));            // Ab += P Yb^T
    URV_TRY(gemm_w<T>(false, false, m, n, n, T(1), A, m, w.Yb, n, T(0), w.Pb, m, w, s));         // Pb = A Yb
    const T* Xb = w.Pb;                                                                          // HALF: P = X_t
    if (full) {
      URV_TRY(qr_adjoint<T>(P, Rw, m, n, w.Pb, nullptr, w.Xb, w, s));                            // W_t = Qpos(X_t)
      Xb = w.Xb;
    }
    URV_TRY(gemm_w<T>(false, true, m, n, n, T(1), Xb, m, Vin, n, T(1), dA, m, w, s));            // Ab += Xb V_{t-1}^T
    if (t > 1) URV_TRY(gemm_w<T>(true, false, n, n, m, T(1), A, m, Xb, m, T(0), w.Vb, n, w, s)); // Vb = A^T Xb
  }
  return URV_OK;
}

// L = ||A - U(:,1:k) R(1:k,:) V^T||_F^2 and its adjoints.  E is formed in dA
// (then scaled to 2E, the loss's own term in A); with Akb = -2E:
// dU(:,1:k) = Akb V R_k^T, dR(1:k,:) = U_k^T Akb V, dV = Akb^T U_k R_k.
template <class T>
int loss_impl(const T* A, int64_t m, int64_t n, const T* U, const T* R, const T* V, int64_t k, double* loss,
              T* dU, T* dR, T* dV, T* dA, const GradWork<T>& w, hipStream_t s) {
  URV_TRY(copy2d<T>(A, m, dA, m, m, n, s));
  if (k > 0) {
    URV_TRY(gemm_w<T>(false, true, k, n, n, T(1), R, n, V, n, T(0), w.M, k, w, s));              // R_k V^T
    URV_TRY(gemm_w<T>(false, false, m, n, k, T(-1), U, m, w.M, k, T(1), dA, m, w, s));           // E = A - A_k
  }
  if (loss) {
    sumsq_partial_kernel<T><<<kLossBlocks, kLossThreads, 0, s>>>(dA, m, m, n, w.loss_partial);
    URV_LAUNCHED("sumsq_partial_kernel");
    sum_partials_kernel<<<1, kLossThreads, 0, s>>>(w.loss_partial, kLossBlocks, loss);
    URV_LAUNCHED("sum_partials_kernel");
  }
  if (dU || dR) URV_TRY(gemm_w<T>(false, false, m, n, n, T(-2), dA, m, V, n, T(0), w.Xb, m, w, s));  // Akb V
  if (dU) {
    if (k > 0) URV_TRY(gemm_w<T>(false, true, m, k, n, T(1), w.Xb, m, R, n, T(0), dU, m, w, s));
    URV_TRY(fill2d<T>(dU + k * m, m, m, n - k, T(0), s));
  }
  if (dR) {
    if (k > 0) URV_TRY(gemm_w<T>(true, false, k, n, m, T(1), U, m, w.Xb, m, T(0), dR, n, w, s));
    URV_TRY(fill2d<T>(dR + k, n, n - k, n, T(0), s));
  }
  if (dV) {
    if (k > 0) {
      URV_TRY(gemm_w<T>(false, false, m, n, k, T(1), U, m, R, n, T(0), w.Pb, m, w, s));           // U_k R_k
      URV_TRY(gemm_w<T>(true, false, n, n, m, T(-2), dA, m, w.Pb, m, T(0), dV, n, w, s));        // Akb^T U_k R_k
    } else {
      URV_TRY(fill2d<T>(dV, n, n, n, T(0), s));
    }
  }
  scale_kernel2d<T><<<grid_for(m * n), 256, 0, s>>>(dA, m, m, n, T(2));
  URV_LAUNCHED("scale_kernel2d");
  return URV_OK;
}

// ---------------------------------------------------------------- entry plumbing

int check_opts(const urv_grad_opts& o, const char* who) {
  if (o.precision != URV_FP64 && o.precision != URV_FP32) {
    set_last_error(std::string(who) + ": precision must be URV_FP64 or URV_FP32");
    return URV_EINVAL;
  }
  if (o.variant != URV_REORTH_FULL && o.variant != URV_REORTH_HALF) {
    set_last_error(std::string(who) + ": variant must be FULL or HALF");
    return URV_EINVAL;
  }
  if (o.tape_mode < URV_TAPE_ALL || o.tape_mode > URV_TAPE_NONE) {
    set_last_error(std::string(who) + ": unknown tape mode");
    return URV_EINVAL;
  }
  if (o.workspace == nullptr && o.workspace_bytes != 0) {
    set_last_error(std::string(who) + ": workspace_bytes given without a workspace");
    return URV_EINVAL;
  }
  return URV_OK;
}

int check_sizes(int64_t m, int64_t n, int32_t q, const char* who) {
  if (n < 0 || m < n || q < 0) {
    set_last_error(std::string(who) + ": need 0 <= n <= m and q >= 0");
    return URV_EINVAL;
  }
  if (m > kMaxRows) {
    set_last_error(std::string(who) + ": more rows than the panel kernel supports");
    return URV_ENOTSUP;
  }
  return URV_OK;
}

size_t work_bytes(int64_t m, int64_t n, bool f32) { return f32 ? grad_bytes<float>(m, n) : grad_bytes<double>(m, n); }

// Runs body(GradWork<T>&) on the caller's or a stream-ordered library workspace.
template <class T, class F>
int with_work(int64_t m, int64_t n, const urv_grad_opts& o, const char* who, F body) {
  hipStream_t s = static_cast<hipStream_t>(o.stream);
  const size_t need = grad_bytes<T>(m, n);
  Arena a;
  bool owned = false;
  if (o.workspace) {
    if (o.workspace_bytes < need) {
      set_last_error(std::string(who) + ": workspace too small (see urv_grad_workspace_size)");
      return URV_EINVAL;
    }
    a.base = static_cast<char*>(o.workspace);
    a.size = o.workspace_bytes;
  } else {
    void* p = nullptr;
    const hipError_t e = hipMallocAsync(&p, need, s);
    if (e != hipSuccess) {
      (void)hipGetLastError();  // clear the sticky error; the failure is reported below
      set_last_error(std::string(who) + ": workspace allocation failed: " + hipGetErrorString(e));
      return URV_ENOMEM;
    }
    a.base = static_cast<char*>(p);
    a.size = need;
    owned = true;
  }
  GradWork<T> w;
  carve_grad(a, m, n, w);
  int rc = a.overflow ? URV_EINVAL : qr_clear_error_flag(w.qr, n, s);
  if (rc == URV_OK) rc = body(w, s);
  if (owned) {
    const hipError_t e = hipFreeAsync(a.base, s);
    if (e != hipSuccess && rc == URV_OK) rc = hip_status(e, who);
  }
  return rc;
}

template <class T>
TapeLayout<T> tape_view(void* tape, int64_t m, int64_t n, int32_t q, const urv_grad_opts& o) {
  Arena a;
  a.base = static_cast<char*>(tape);
  a.size = static_cast<size_t>(-1);
  TapeLayout<T> tl;
  carve_tape(a, m, n, q, o.variant == URV_REORTH_FULL, o.tape_mode, tl);
  return tl;
}

template <class T>
int forward_entry(const void* A, int64_t m, int64_t n, int32_t q, const void* G, void* U, void* R, void* V,
                  void* tape, const urv_grad_opts& o) {
  const TapeLayout<T> tl = tape_view<T>(tape, m, n, q, o);
  return with_work<T>(m, n, o, "urv_factor_tape", [&](const GradWork<T>& w, hipStream_t s) {
    return forward_impl<T>(static_cast<const T*>(A), m, n, q, o.variant == URV_REORTH_FULL,
                           static_cast<const T*>(G), static_cast<T*>(U), static_cast<T*>(R), static_cast<T*>(V),
                           tl, w, s);
  });
}

template <class T>
int backward_entry(const void* A, int64_t m, int64_t n, int32_t q, const void* G, const void* U, const void* R,
                   const void* V, const void* tape, const void* dU, const void* dR, const void* dV, void* dA,
                   const urv_grad_opts& o) {
  const TapeLayout<T> tl = tape_view<T>(const_cast<void*>(tape), m, n, q, o);
  return with_work<T>(m, n, o, "urv_factor_backward", [&](const GradWork<T>& w, hipStream_t s) {
    return backward_impl<T>(static_cast<const T*>(A), m, n, q, o.variant == URV_REORTH_FULL,
                            static_cast<const T*>(G), static_cast<const T*>(U), static_cast<const T*>(R),
                            static_cast<const T*>(V), tl, static_cast<const T*>(dU), static_cast<const T*>(dR),
                            static_cast<const T*>(dV), static_cast<T*>(dA), o.accumulate != 0, w, s);
  });
}

}  // namespace
}  // namespace urv

using namespace urv;

extern "C" {

void urv_grad_opts_init(urv_grad_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = URV_FP64;
  o->variant = URV_REORTH_FULL;
  o->tape_mode = URV_TAPE_ALL;
}

size_t urv_tape_bytes(int64_t m, int64_t n, int32_t q, const urv_grad_opts* opts) {
  urv_grad_opts o;
  urv_grad_opts_init(&o);
  if (opts) o = *opts;
  if (n <= 0 || m < n || q <= 0 || check_opts(o, "urv_tape_bytes") != URV_OK) return 0;
  const bool full = o.variant == URV_REORTH_FULL;
  return o.precision == URV_FP32 ? tape_bytes<float>(m, n, q, full, o.tape_mode)
                                 : tape_bytes<double>(m, n, q, full, o.tape_mode);
}

size_t urv_grad_workspace_size(int64_t m, int64_t n, int32_t q, const urv_grad_opts* opts) {
  (void)q;
  urv_grad_opts o;
  urv_grad_opts_init(&o);
  if (opts) o = *opts;
  if (n <= 0 || m < n || check_opts(o, "urv_grad_workspace_size") != URV_OK) return 0;
  return work_bytes(m, n, o.precision == URV_FP32);
}

int urv_factor_tape(const void* A, int64_t m, int64_t n, int32_t q, const void* G, void* U, void* R, void* V,
                    void* tape, const urv_grad_opts* opts) {
  clear_last_error();
  urv_grad_opts o;
  urv_grad_opts_init(&o);
  if (opts) o = *opts;
  URV_TRY(check_opts(o, "urv_factor_tape"));
  URV_TRY(check_sizes(m, n, q, "urv_factor_tape"));
  if (n == 0) return URV_OK;
  if (!A || !G || !U || !R || !V || (!tape && urv_tape_bytes(m, n, q, &o) > 0)) {
    set_last_error("urv_factor_tape: null pointer");
    return URV_EINVAL;
  }
  return o.precision == URV_FP32 ? forward_entry<float>(A, m, n, q, G, U, R, V, tape, o)
                                 : forward_entry<double>(A, m, n, q, G, U, R, V, tape, o);
}

int urv_factor_backward(const void* A, int64_t m, int64_t n, int32_t q, const void* G, const void* U,
                        const void* R, const void* V, const void* tape, const void* dU, const void* dR,
                        const void* dV, void* dA, const urv_grad_opts* opts) {
  clear_last_error();
  urv_grad_opts o;
  urv_grad_opts_init(&o);
  if (opts) o = *opts;
  URV_TRY(check_opts(o, "urv_factor_backward"));
  URV_TRY(check_sizes(m, n, q, "urv_factor_backward"));
  if (n == 0) return URV_OK;
  if (!A || !G || !U || !R || !V || !dA || (!tape && urv_tape_bytes(m, n, q, &o) > 0)) {
    set_last_error("urv_factor_backward: null pointer");
    return URV_EINVAL;
  }
  return o.precision == URV_FP32 ? backward_entry<float>(A, m, n, q, G, U, R, V, tape, dU, dR, dV, dA, o)
                                 : backward_entry<double>(A, m, n, q, G, U, R, V, tape, dU, dR, dV, dA, o);
}

int urv_qr_adjoint(const void* Q, const void* R, int64_t m, int64_t n, const void* dQ, const void* dR, void* dX,
                   int32_t precision, void* stream) {
  clear_last_error();
  urv_grad_opts o;
  urv_grad_opts_init(&o);
  o.precision = precision;
  o.stream = stream;
  URV_TRY(check_opts(o, "urv_qr_adjoint"));
  URV_TRY(check_sizes(m, n, 0, "urv_qr_adjoint"));
  if (n == 0) return URV_OK;
  if (!Q || !R || !dX) {
    set_last_error("urv_qr_adjoint: null pointer");
    return URV_EINVAL;
  }
  if (precision == URV_FP32)
    return with_work<float>(m, n, o, "urv_qr_adjoint", [&](const GradWork<float>& w, hipStream_t s) {
      return qr_adjoint<float>(static_cast<const float*>(Q), static_cast<const float*>(R), m, n,
                               static_cast<const float*>(dQ), static_cast<const float*>(dR),
                               static_cast<float*>(dX), w, s);
    });
  return with_work<double>(m, n, o, "urv_qr_adjoint", [&](const GradWork<double>& w, hipStream_t s) {
    return qr_adjoint<double>(static_cast<const double*>(Q), static_cast<const double*>(R), m, n,
                              static_cast<const double*>(dQ), static_cast<const double*>(dR),
                              static_cast<double*>(dX), w, s);
  });
}

int urv_truncation_loss(const void* A, int64_t m, int64_t n, const void* U, const void* R, const void* V,
                        int64_t k, double* loss, void* dU, void* dR, void* dV, void* dA,
                        const urv_grad_opts* opts) {
  clear_last_error();
  urv_grad_opts o;
  urv_grad_opts_init(&o);
  if (opts) o = *opts;
  URV_TRY(check_opts(o, "urv_truncation_loss"));
  URV_TRY(check_sizes(m, n, 0, "urv_truncation_loss"));
  if (k < 0 || k > n) {
    set_last_error("urv_truncation_loss: need 0 <= k <= n");
    return URV_EINVAL;
  }
  if (n == 0) return URV_OK;
  if (!A || !U || !R || !V || !dA) {
    set_last_error("urv_truncation_loss: null pointer");
    return URV_EINVAL;
  }
  if (o.precision == URV_FP32)
    return with_work<float>(m, n, o, "urv_truncation_loss", [&](const GradWork<float>& w, hipStream_t s) {
      return loss_impl<float>(static_cast<const float*>(A), m, n, static_cast<const float*>(U),
                              static_cast<const float*>(R), static_cast<const float*>(V), k, loss,
                              static_cast<float*>(dU), static_cast<float*>(dR), static_cast<float*>(dV),
                              static_cast<float*>(dA), w, s);
    });
  return with_work<double>(m, n, o, "urv_truncation_loss", [&](const GradWork<double>& w, hipStream_t s) {
    return loss_impl<double>(static_cast<const double*>(A), m, n, static_cast<const double*>(U),
                             static_cast<const double*>(R), static_cast<const double*>(V), k, loss,
                             static_cast<double*>(dU), static_cast<double*>(dR), static_cast<double*>(dV),
                             static_cast<double*>(dA), w, s);
  });
}

}  // extern "C"
