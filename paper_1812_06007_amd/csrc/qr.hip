// Unpivoted blocked Householder QR with explicit Q and a non-negative
// diagonal of R -- the "Qpos" of the PowerURV iteration (Section 3, eqs.
// power and powerqr) and of DDH-URV (Section 2.2).  Following Section 2.2,
// reflectors are accumulated per block of kPanelNB columns and applied to the
// trailing matrix with matrix-matrix products (compact WY form
// H_1 ... H_b = I - Y T Y^T, Schreiber & Van Loan 1989).
//
// Per block:
//   panel_kernel     Householder vectors of an (m-j0) x b panel, column by
//                    column.  The panel is spread over P workgroups by rows;
//                    each holds its rows in registers (one column per lane).
//                    One column needs one device-wide reduction: the partial
//                    inner products of the pivot column with every column of
//                    the panel, from which the norm, the reflector and its
//                    action follow.  Workgroups meet at a counter barrier;
//                    partial sums are added in a fixed order, so every
//                    workgroup derives bitwise-identical reflectors.
//   S = Y^T Y        FP64 MFMA GEMM
//   build_t_kernel   T (upper triangular) from tau and S, in LDS
//   trailing update  C <- (I - Y T^T Y^T) C by three GEMMs.
// Q is formed afterwards from the stored blocks, last block first, starting
// from [D; 0] with D = sign(diag R), which makes diag(R) >= 0 at no cost.
#include "common.hpp"

namespace urv {
namespace {

constexpr int NB = kPanelNB;        // columns per panel (one lane per column)
constexpr int PANEL_WAVES = 4;      // row groups per workgroup
constexpr int RPT = 64;             // rows per lane
constexpr int RPW = PANEL_WAVES * RPT;  // rows per workgroup
constexpr int kMaxPanelWgs = 240;   // all panel workgroups must be co-resident
constexpr long kSpinLimit = 1L << 23;   // bounded wait: ~seconds, then give up

__device__ inline bool grid_barrier(unsigned* counter, unsigned target, unsigned* err) {
  // Release our writes, count in, poll (relaxed, so the loop does not keep
  // invalidating caches), then acquire everybody's writes once.
  __threadfence();
  __syncthreads();
  __shared__ int failed;
  if (threadIdx.x == 0) {
    failed = 0;
    __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    long spins = 0;
    while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          ++spins > kSpinLimit) {
        __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        failed = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return failed == 0;
}

// Panel rows [0, mp) x columns [0, jb) at X (ld ldx); the panel's first row is
// the diagonal row of its first column.  Writes the factored panel back in
// place (R above / beta on the diagonal / v below), the explicit unit-lower
// reflector block to Y (ld ldy, same row origin), and tau[0..jb).
__global__ __launch_bounds__(256) void panel_kernel(double* __restrict__ X, int64_t ldx,
                                                     int64_t mp, int jb, double* __restrict__ Y,
                                                     int64_t ldy, double* __restrict__ tau,
                                                     double* __restrict__ part,
                                                     double* __restrict__ rowj,
                                                     unsigned* __restrict__ counter,
                                                     unsigned* __restrict__ err) {
  __shared__ double stage[64][NB + 1];
  __shared__ double colj[RPW];
  __shared__ double red[PANEL_WAVES][NB];

  const int P = gridDim.x;
  const int wg = blockIdx.x;
  const int c = threadIdx.x & 63;       // column owned by this lane
  const int g = threadIdx.x >> 6;       // row group (wave)
  const int64_t row0 = static_cast<int64_t>(wg) * RPW;
  const int64_t myrow0 = row0 + g * RPT;  // first panel row of this lane

  // ---- load: chunk k (64 rows) of the workgroup belongs to wave k
  double x[RPT];
  for (int k = 0; k < PANEL_WAVES; ++k) {
    for (int e = threadIdx.x; e < 64 * NB; e += 256) {
      const int r = e & 63, col = e >> 6;
      const int64_t gi = row0 + k * 64 + r;
      stage[r][col] = (gi < mp && col < jb) ? X[gi + col * ldx] : 0.0;
    }
    __syncthreads();
    if (g == k) {
#pragma unroll
      for (int r = 0; r < RPT; ++r) x[r] = stage[r][c];
    }
    __syncthreads();
  }

  bool ok = true;
  for (int j = 0; j < jb && ok; ++j) {
    const int buf = j & 1;
    double* pj = part + static_cast<int64_t>(buf) * P * NB;
    double* rj = rowj + buf * NB;
    // 1. pivot column of this workgroup's rows into LDS; pivot row to global
    if (c == j) {
#pragma unroll
      for (int r = 0; r < RPT; ++r) colj[g * RPT + r] = x[r];
    }
    if (j >= myrow0 && j < myrow0 + RPT && c >= j && c < jb) {
      const int rr = static_cast<int>(j - myrow0);
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if (r == rr) rj[c] = x[r];
    }
    __syncthreads();
    // 2. partial inner products over rows below the pivot
    double p = 0.0;
    if (c >= j && c < jb) {
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int64_t gi = myrow0 + r;
        if (gi > j && gi < mp) p += colj[g * RPT + r] * x[r];
      }
    }
    red[g][c] = p;
    __syncthreads();
    if (g == 0 && c >= j && c < jb) pj[static_cast<int64_t>(wg) * NB + c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
    // 3. all workgroups
    ok = grid_barrier(counter, static_cast<unsigned>(P) * (j + 1), err);
    if (!ok) break;
    // 4. reflector of column j and its action on columns c >= j
    if (c >= j && c < jb) {
      double sigma2 = 0.0, d = 0.0;
      for (int w = 0; w < P; ++w) {
        sigma2 += pj[static_cast<int64_t>(w) * NB + j];
        d += pj[static_cast<int64_t>(w) * NB + c];
      }
      const double alpha = rj[j];
      if (sigma2 != 0.0) {
        const double norm = sqrt(alpha * alpha + sigma2);
        const double beta = (alpha >= 0.0) ? -norm : norm;
        const double denom = alpha - beta;
        const double t = (beta - alpha) / beta;
        if (c == j) {
#pragma unroll
          for (int r = 0; r < RPT; ++r) {
            const int64_t gi = myrow0 + r;
            if (gi > j) x[r] = x[r] / denom;
            else if (gi == j) x[r] = beta;
          }
          if (wg == 0 && g == 0) tau[j] = t;
        } else {
          const double xcj = rj[c];
          const double tw = t * (xcj + d / denom);  // tau * (v^T x_c)
#pragma unroll
          for (int r = 0; r < RPT; ++r) {
            const int64_t gi = myrow0 + r;
            if (gi > j) x[r] -= tw * (colj[g * RPT + r] / denom);
            else if (gi == j) x[r] -= tw;
          }
        }
      } else if (c == j && wg == 0 && g == 0) {
        tau[j] = 0.0;
      }
    }
  }

  if (!ok) {
    // Device-side wait gave up: poison the outputs so the failure is visible.
    const double nan = __builtin_nan("");
    if (wg == 0 && threadIdx.x < jb) tau[threadIdx.x] = nan;
#pragma unroll
    for (int r = 0; r < RPT; ++r) x[r] = nan;
  }

  // ---- store: panel in place, and explicit Y (0 above, 1 on the diagonal)
  for (int k = 0; k < PANEL_WAVES; ++k) {
    if (g == k) {
#pragma unroll
      for (int r = 0; r < RPT; ++r) stage[r][c] = x[r];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * NB; e += 256) {
      const int r = e & 63, col = e >> 6;
      const int64_t gi = row0 + k * 64 + r;
      if (gi < mp && col < jb) {
        const double v = stage[r][col];
        X[gi + col * ldx] = v;
        Y[gi + col * ldy] = (gi > col) ? v : (gi == col ? 1.0 : 0.0);
      }
    }
    __syncthreads();
  }
}

// T (jb x jb, upper) with H_0 ... H_{jb-1} = I - Y T Y^T from tau and the
// Gram matrix S = Y^T Y:  T(j,j) = tau_j,  T(0:j, j) = -tau_j T(0:j,0:j) S(0:j, j).
__global__ __launch_bounds__(256) void build_t_kernel(const double* __restrict__ S, int lds,
                                                       const double* __restrict__ tau, int jb,
                                                       double* __restrict__ T, int ldt) {
  __shared__ double Ts[NB][NB + 1];
  __shared__ double Ss[NB][NB + 1];
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
    const int i = e % NB, j = e / NB;
    Ss[i][j] = (i < jb && j < jb) ? S[i + j * lds] : 0.0;
    Ts[i][j] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < jb; ++j) {
    const double t = tau[j];
    const int i = threadIdx.x;
    double v = 0.0;
    if (i < j) {
      for (int k = i; k < j; ++k) v += Ts[i][k] * Ss[k][j];
      v = -t * v;
    }
    __syncthreads();
    if (i < j) Ts[i][j] = v;
    if (i == j) Ts[j][j] = t;
    __syncthreads();
  }
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
    const int i = e % NB, j = e / NB;
    if (i < jb && j < jb) T[i + j * ldt] = Ts[i][j];
  }
}

// R(i,c) = d_i X(i,c) for i <= c, 0 below; d_i = sign(X(i,i)), sign(0) = +1.
__global__ void extract_r_kernel(const double* __restrict__ X, int64_t ldx, int64_t n,
                                 double* __restrict__ R, int64_t ldr) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx % n, c = idx / n;
  double v = 0.0;
  if (i <= c) {
    const double d = (X[i + i * ldx] < 0.0) ? -1.0 : 1.0;
    v = d * X[i + c * ldx];
  }
  R[i + c * ldr] = v;
}

// Q = [D; 0], D = diag(sign(X(c,c))).
__global__ void init_q_kernel(const double* __restrict__ X, int64_t ldx, int64_t m, int64_t n,
                              double* __restrict__ Q, int64_t ldq) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= m * n) return;
  const int64_t i = idx % m, c = idx / m;
  double v = 0.0;
  if (i == c) v = (X[c + c * ldx] < 0.0) ? -1.0 : 1.0;
  Q[i + c * ldq] = v;
}

__global__ void fill_u32_kernel(unsigned* p, int64_t count, unsigned v) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx < count) p[idx] = v;
}

int64_t panel_wgs(int64_t mp) { return ceil_div(mp, RPW); }

struct QrSizes {
  size_t y, t, tau, s, w, part, rowj, sync, gemm_work;
};

QrSizes qr_sizes(int64_t m, int64_t n) {
  QrSizes z;
  const int64_t nblocks = ceil_div(n, NB);
  z.y = static_cast<size_t>(m) * n;
  z.t = static_cast<size_t>(NB) * n;
  z.tau = n;
  z.s = NB * NB;
  z.w = static_cast<size_t>(NB) * n;
  z.part = 2 * static_cast<size_t>(panel_wgs(m)) * NB;
  z.rowj = 2 * NB;
  z.sync = nblocks + 2;
  size_t gw = 0;
  for (int64_t j0 = 0; j0 < n; j0 += NB) {
    const int64_t jb = std::min<int64_t>(NB, n - j0), mp = m - j0;
    gw = std::max(gw, dgemm_work_elems(jb, jb, mp));
    gw = std::max(gw, dgemm_work_elems(jb, n - j0 - jb, mp));
    gw = std::max(gw, dgemm_work_elems(jb, n - j0, mp));
  }
  z.gemm_work = gw;
  return z;
}

}  // namespace

size_t qr_work_bytes(int64_t m, int64_t n) {
  Arena a;
  QrWork w;
  qr_work_carve(a, m, n, w);
  return a.used;
}

void qr_work_carve(Arena& a, int64_t m, int64_t n, QrWork& w) {
  const QrSizes z = qr_sizes(m, n);
  w.Y = a.take<double>(z.y);
  w.T = a.take<double>(z.t);
  w.tau = a.take<double>(z.tau);
  w.S = a.take<double>(z.s);
  w.W1 = a.take<double>(z.w);
  w.W2 = a.take<double>(z.w);
  w.part = a.take<double>(z.part);
  w.rowj = a.take<double>(z.rowj);
  w.sync = a.take<unsigned>(z.sync);
  w.gemm_work = a.take<double>(z.gemm_work);
  w.gemm_work_elems = z.gemm_work;
}

int qr_pos(double* X, int64_t m, int64_t n, int64_t ldx, double* Q, int64_t ldq, double* R,
           int64_t ldr, const QrWork& w, hipStream_t s) {
  if (n == 0) return URV_OK;
  const int64_t nblocks = ceil_div(n, NB);
  if (panel_wgs(m) > kMaxPanelWgs) {
    set_last_error("qr_pos: too many rows for the panel kernel");
    return URV_ENOTSUP;
  }
  unsigned* err = w.sync + nblocks;
  fill_u32_kernel<<<static_cast<unsigned>(ceil_div(nblocks + 2, 256)), 256, 0, s>>>(w.sync, nblocks + 2, 0u);
  URV_LAUNCHED("fill_u32_kernel");

  for (int64_t j0 = 0, blk = 0; j0 < n; j0 += NB, ++blk) {
    const int jb = static_cast<int>(std::min<int64_t>(NB, n - j0));
    const int64_t mp = m - j0;
    double* Xp = X + j0 + j0 * ldx;
    double* Yb = w.Y + j0 + j0 * m;
    double* Tb = w.T + j0 * NB;
    const unsigned P = static_cast<unsigned>(panel_wgs(mp));
    panel_kernel<<<P, 256, 0, s>>>(Xp, ldx, mp, jb, Yb, m, w.tau + j0, w.part, w.rowj,
                                   w.sync + blk, err);
    URV_LAUNCHED("panel_kernel");
    URV_TRY(dgemm(true, false, jb, jb, mp, 1.0, Yb, m, Yb, m, 0.0, w.S, NB, w.gemm_work,
                  w.gemm_work_elems, s));
    build_t_kernel<<<1, 256, 0, s>>>(w.S, NB, w.tau + j0, jb, Tb, NB);
    URV_LAUNCHED("build_t_kernel");
    const int64_t nc = n - j0 - jb;
    if (nc > 0) {
      double* Cb = X + j0 + (j0 + jb) * ldx;
      URV_TRY(dgemm(true, false, jb, nc, mp, 1.0, Yb, m, Cb, ldx, 0.0, w.W1, NB, w.gemm_work,
                    w.gemm_work_elems, s));
      URV_TRY(dgemm(true, false, jb, nc, jb, 1.0, Tb, NB, w.W1, NB, 0.0, w.W2, NB, nullptr, 0, s));
      URV_TRY(dgemm(false, false, mp, nc, jb, -1.0, Yb, m, w.W2, NB, 1.0, Cb, ldx, nullptr, 0, s));
    }
  }

  if (R) {
    extract_r_kernel<<<static_cast<unsigned>(ceil_div(n * n, 256)), 256, 0, s>>>(X, ldx, n, R, ldr);
    URV_LAUNCHED("extract_r_kernel");
  }
  if (Q) {
    init_q_kernel<<<static_cast<unsigned>(ceil_div(m * n, 256)), 256, 0, s>>>(X, ldx, m, n, Q, ldq);
    URV_LAUNCHED("init_q_kernel");
    for (int64_t blk = nblocks - 1; blk >= 0; --blk) {
      const int64_t j0 = blk * NB;
      const int jb = static_cast<int>(std::min<int64_t>(NB, n - j0));
      const int64_t mp = m - j0, nq = n - j0;
      const double* Yb = w.Y + j0 + j0 * m;
      const double* Tb = w.T + j0 * NB;
      double* Qb = Q + j0 + j0 * ldq;
      URV_TRY(dgemm(true, false, jb, nq, mp, 1.0, Yb, m, Qb, ldq, 0.0, w.W1, NB, w.gemm_work,
                    w.gemm_work_elems, s));
      URV_TRY(dgemm(false, false, jb, nq, jb, 1.0, Tb, NB, w.W1, NB, 0.0, w.W2, NB, nullptr, 0, s));
      URV_TRY(dgemm(false, false, mp, nq, jb, -1.0, Yb, m, w.W2, NB, 1.0, Qb, ldq, nullptr, 0, s));
    }
  }
  return URV_OK;
}

unsigned* qr_error_flag(const QrWork& w, int64_t n) { return w.sync + ceil_div(n, NB); }

}  // namespace urv
