// Batched PowerURV: many independent FP32 matrices (up to 1024 rows) factored
// in one persistent launch.
//
// Each matrix runs the method of Section 3 (eqs. power and powerqr, FULL
// re-orthonormalisation): G from Philox stream 2 under key (seed + i, 0),
// rounded to FP32; q times X = A V, W = Qpos(X), Y = A^T W, V = Qpos(Y); then
// A V = U R.  Qpos is the unpivoted Householder QR of Section 2.2 with the
// reflectors accumulated in compact WY form (I - V T V^T) and diag(R) made
// non-negative (the footnote on Haar matrices).
//
// Design for gfx950: one workgroup (4 waves) owns one matrix at a time and
// takes the next matrix from a device-side counter; matrices are queued
// largest first, so the long ones start early and the short ones fill the
// tail.  Within a workgroup:
//  * GEMMs (A V, A^T W and the block-reflector updates, T applied as a
//    product too) on FP32 MFMA (v_mfma_f32_16x16x4f32), 64 x 64 tiles (32 x 64
//    for the products with 32 rows) staged through double-buffered LDS, 4
//    waves; the short-K updates run one flat loop over tiles that loads the
//    next tile while the current one computes;
//  * the panel of NB columns lives in registers (4 rows per lane, rows up to
//    1024); each column takes two workgroup reductions in a fixed order: the
//    norm below the pivot, then the reflector's products with the remaining
//    columns together with its Gram entries against the earlier reflectors,
//    from which T is built without another pass;
//  * Q is accumulated backward from [I; 0], then the sign fix.
// The last workgroup to leave resets the counters, so one launch needs no
// host-side clearing and can be replayed from a captured graph.
#include "common.hpp"
#include "philox.hpp"

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

struct urv_batch_plan;

namespace urv {
namespace {

constexpr int BT = 256;                  // threads per workgroup: 4 waves
constexpr int RPT = 4;                   // panel rows per lane
constexpr int kBatchMaxRows = BT * RPT;  // 1024
constexpr int kNBMax = 32;               // widest panel
constexpr int kLT = 2 * kNBMax;          // leading dimension of T and W: a pair of panels

typedef float f4 __attribute__((ext_vector_type(4)));

struct BatchItem {
  int m = 0, n = 0;
  uint64_t seed = 0;
  const float* A = nullptr;  // m x n, ld m (read only)
  float* U = nullptr;        // m x n
  float* R = nullptr;        // n x n
  float* V = nullptr;        // n x n
  // scratch, packed column-major
  float* X = nullptr;        // m x n: A V, factored in place
  float* Q = nullptr;        // m x n: W = Qpos(X)
  float* Y = nullptr;        // n x n: A^T W, factored in place
  float* Vc = nullptr;       // n x n: the current V
  float* Vr = nullptr;       // m x n: explicit unit-lower reflectors of the current QR
  float* T = nullptr;        // kLT x n: T of each pair of panels
  float* Wb = nullptr;       // kLT x n
  float* W2b = nullptr;      // kLT x n
};

constexpr int GBK = 32;  // k step of the workgroup GEMM
constexpr int RED_LD = BT + BT / 32;  // reduction staging: value v of lane t at v RED_LD + t + t / 32
constexpr int PARTS = BT / 32;

struct Lds {
  union {
    struct {
      float As[2][GBK][64 + 1];  // double-buffered tiles of the GEMM
      float Bs[2][GBK][64 + 1];
    } g;
    struct {
      float As[2][2 * GBK][64 + 1];  // the short GEMM's tiles: K <= 2 GBK in one step
      float Bs[2][2 * GBK][64 + 1];
    } g2;
    float red[kNBMax * RED_LD];
  } u;
  float part[kNBMax][PARTS + 1];
  float res[kNBMax];
  float gram[kNBMax][kNBMax + 1];      // gram[b][c] = v_b^T v_c, b < c
  float tau[kNBMax];
  float trow[kNBMax][kNBMax + 1];      // rows of T, one per lane
  float alpha;
  int idx;
};

// Sums vals[0..CNT) over the workgroup into s.res (every lane may read it on
// return).  Lane (v, p) = (t / PARTS, t % PARTS) adds lanes 32p .. 32p + 31 of
// value v, then lane v adds the PARTS parts: a fixed order, bitwise
// reproducible.
template <int CNT>
__device__ __forceinline__ void block_sum(const float (&vals)[CNT], Lds& s) {
  static_assert(CNT >= 1 && CNT <= kNBMax && kNBMax * PARTS == BT, "reduction width");
  const int t = threadIdx.x;
#pragma unroll
  for (int v = 0; v < CNT; ++v) s.u.red[v * RED_LD + t + (t >> 5)] = vals[v];
  __syncthreads();
  {
    const int v = t / PARTS, p = t % PARTS;
    if (v < CNT) {
      const float* r = &s.u.red[v * RED_LD + p * 33];
      float a = 0.f;
#pragma unroll 8
      for (int i = 0; i < 32; ++i) a += r[i];
      s.part[v][p] = a;
    }
  }
  __syncthreads();
  if (t < CNT) {
    float a = 0.f;
#pragma unroll
    for (int p = 0; p < PARTS; ++p) a += s.part[t][p];
    s.res[t] = a;
  }
  __syncthreads();
}

// A team of `size` workgroups factoring one matrix together; `member` is this
// workgroup's rank.  Work of a phase is split over the members (GEMM tiles,
// element ranges); the panel is factored by member 0; team_sync separates the
// phases.  A team of one is a plain workgroup.
struct Team {
  int member = 0, size = 1;
  unsigned* bar = nullptr;  // arrivals at the task's barriers (agent-scope counter)
  unsigned* err = nullptr;  // raised when a bounded wait expires
  unsigned phase = 0;       // barriers passed so far
};

constexpr long kTeamSpinLimit = 1l << 24;  // polls before a barrier wait gives up

// Barrier of the whole team.  Lane 0 publishes its workgroup's writes with an
// agent-scope fence, counts itself in, waits (bounded) until every member has
// arrived, and fences again before the workgroup reads the others' results.
__device__ __forceinline__ void team_sync(Team& tm) {
  __syncthreads();
  if (tm.size == 1) return;
  ++tm.phase;
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(tm.bar, 1u);
    const unsigned target = tm.phase * static_cast<unsigned>(tm.size);
    long spins = 0;
    while (__hip_atomic_load(tm.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if ((++spins & 255) == 0 &&
          (spins > kTeamSpinLimit || __hip_atomic_load(tm.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
        __hip_atomic_store(tm.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
  }
  __syncthreads();
}

// C (M x N) = alpha op(A) B + beta C for the whole workgroup; op(A) = A (TA
// false, A M x K) or A^T (A K x M).  BM x 64 tiles of C (BM = 64, or 32 for
// the short products with M <= 32), K in steps of GBK through double-buffered
// LDS with the next step's global loads in flight during the current step's
// MFMAs; the 4 waves are 2 x 2, each owning (BM / 2) x 32 of the tile.  The
// members of a team take every size-th tile.  beta == 0 never reads C.  C must
// not overlap A or B.  Ends with a team barrier, so the team may read C right
// after.
template <bool TA, int BM>
__device__ __noinline__ void wg_gemm_t(int M, int N, int K, float alpha, const float* __restrict__ A, int lda,
                                          const float* __restrict__ B, int ldb, float beta, float* __restrict__ C,
                                          int ldc, Lds& s, Team& tm) {
  constexpr int FM = BM / 32;                  // 16-row MFMA blocks per wave
  constexpr int FN = 2;                        // 16-column MFMA blocks per wave
  constexpr int LA = BM * GBK / BT, LB = 64 * GBK / BT;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lrow = lane & 15, lk = lane >> 4;
  const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + 63) / 64;
  float ra[LA], rb[LB];
  auto load = [&](int m0, int n0, int k0) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int qa = t + BT * r;
      int i, k;
      if (!TA) {
        i = qa % BM;
        k = qa / BM;
      } else {
        k = qa % GBK;
        i = qa / GBK;
      }
      const int gi = m0 + i, gk = k0 + k;
      float v = 0.f;
      if (gi < M && gk < K)
        v = TA ? A[gk + static_cast<int64_t>(gi) * lda] : A[gi + static_cast<int64_t>(gk) * lda];
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int qb = t + BT * r;
      const int k = qb % GBK, j = qb / GBK;
      const int gj = n0 + j, gk = k0 + k;
      rb[r] = (gj < N && gk < K) ? B[gk + static_cast<int64_t>(gj) * ldb] : 0.f;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int qa = t + BT * r;
      int i, k;
      if (!TA) {
        i = qa % BM;
        k = qa / BM;
      } else {
        k = qa % GBK;
        i = qa / GBK;
      }
      s.u.g.As[buf][k][i] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int qb = t + BT * r;
      s.u.g.Bs[buf][qb % GBK][qb / GBK] = rb[r];
    }
  };
  for (int tile = tm.member; tile < tiles_m * tiles_n; tile += tm.size) {
    const int m0 = (tile % tiles_m) * BM, n0 = (tile / tiles_m) * 64;
    f4 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    const int nk = (K + GBK - 1) / GBK;
    load(m0, n0, 0);
    store(0);
    __syncthreads();
    for (int ks = 0; ks < nk; ++ks) {
      const int cur = ks & 1;
      if (ks + 1 < nk) load(m0, n0, (ks + 1) * GBK);
#pragma unroll
      for (int kk = 0; kk < GBK / 4; ++kk) {
        float fa[FM], fb[FN];
#pragma unroll
        for (int a = 0; a < FM; ++a) fa[a] = s.u.g.As[cur][kk * 4 + lk][wm * (BM / 2) + a * 16 + lrow];
#pragma unroll
        for (int b = 0; b < FN; ++b) fb[b] = s.u.g.Bs[cur][kk * 4 + lk][wn * 32 + b * 16 + lrow];
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fb[b], fa[a], acc[a][b], 0, 0, 0);
      }
      if (ks + 1 < nk) store(cur ^ 1);
      __syncthreads();
    }
    // lane holds C(m0 + (BM/2) wm + 16 a + lrow, n0 + 32 wn + 16 b + 4 lk + r)
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      const int gm = m0 + wm * (BM / 2) + a * 16 + lrow;
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gn = n0 + wn * 32 + b * 16 + 4 * lk + r;
          if (gm < M && gn < N) {
            float* c = C + gm + static_cast<int64_t>(gn) * ldc;
            *c = (beta == 0.f) ? alpha * acc[a][b][r] : alpha * acc[a][b][r] + beta * *c;
          }
        }
    }
  }
  team_sync(tm);
}

template <bool TA, int BM, int KS>
__device__ __noinline__ void wg_gemm_short(int M, int N, int K, float alpha, const float* __restrict__ A, int lda,
                                          const float* __restrict__ B, int ldb, float beta, float* __restrict__ C,
                                          int ldc, Lds& s, Team& tm) {
  constexpr int FM = BM / 32;                  // 16-row MFMA blocks per wave
  constexpr int FN = 2;                        // 16-column MFMA blocks per wave
  constexpr int LA = BM * KS / BT, LB = 64 * KS / BT;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lrow = lane & 15, lk = lane >> 4;
  const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + 63) / 64;
  float ra[LA], rb[LB];
  auto load = [&](int m0, int n0, int k0) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int qa = t + BT * r;
      int i, k;
      if (!TA) {
        i = qa % BM;
        k = qa / BM;
      } else {
        k = qa % KS;
        i = qa / KS;
      }
      const int gi = m0 + i, gk = k0 + k;
      float v = 0.f;
      if (gi < M && gk < K)
        v = TA ? A[gk + static_cast<int64_t>(gi) * lda] : A[gi + static_cast<int64_t>(gk) * lda];
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int qb = t + BT * r;
      const int k = qb % KS, j = qb / KS;
      const int gj = n0 + j, gk = k0 + k;
      rb[r] = (gj < N && gk < K) ? B[gk + static_cast<int64_t>(gj) * ldb] : 0.f;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int qa = t + BT * r;
      int i, k;
      if (!TA) {
        i = qa % BM;
        k = qa / BM;
      } else {
        k = qa % KS;
        i = qa / KS;
      }
      s.u.g2.As[buf][k][i] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int qb = t + BT * r;
      s.u.g2.Bs[buf][qb % KS][qb / KS] = rb[r];
    }
  };
  // K <= KS: one k step per tile.  Tiles are taken in pairs, so the C values
  // of the next tile (for beta != 0) are loaded into the other register set
  // while the current tile computes and stores; A and B of the next tile are
  // in flight meanwhile too.
  const int ntiles = tiles_m * tiles_n;
  const int my_tiles = (tm.member < ntiles) ? (ntiles - tm.member + tm.size - 1) / tm.size : 0;
  const bool with_c = beta != 0.f;
  auto origin = [&](int lt, int& m0, int& n0) {
    const int tile = tm.member + lt * tm.size;
    m0 = (tile % tiles_m) * BM;
    n0 = (tile / tiles_m) * 64;
  };
  auto load_c = [&](int m0, int n0, float (&dst)[FM][FN][4]) {
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      const int gm = m0 + wm * (BM / 2) + a * 16 + lrow;
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gn = n0 + wn * 32 + b * 16 + 4 * lk + r;
          dst[a][b][r] = (gm < M && gn < N) ? C[gm + static_cast<int64_t>(gn) * ldc] : 0.f;
        }
    }
  };
  float c0[FM][FN][4], c1[FM][FN][4];
  auto step = [&](int lt, int cur, float (&cv)[FM][FN][4], float (&cn)[FM][FN][4]) {
    const bool has_next = lt + 1 < my_tiles;
    if (has_next) {
      int m1, n1;
      origin(lt + 1, m1, n1);
      load(m1, n1, 0);
      if (with_c) load_c(m1, n1, cn);
    }
    f4 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < KS / 4; ++kk) {
      float fa[FM], fb[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) fa[a] = s.u.g2.As[cur][kk * 4 + lk][wm * (BM / 2) + a * 16 + lrow];
#pragma unroll
      for (int b = 0; b < FN; ++b) fb[b] = s.u.g2.Bs[cur][kk * 4 + lk][wn * 32 + b * 16 + lrow];
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fb[b], fa[a], acc[a][b], 0, 0, 0);
    }
    // lane holds C(m0 + (BM/2) wm + 16 a + lrow, n0 + 32 wn + 16 b + 4 lk + r)
    int m0, n0;
    origin(lt, m0, n0);
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      const int gm = m0 + wm * (BM / 2) + a * 16 + lrow;
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gn = n0 + wn * 32 + b * 16 + 4 * lk + r;
          if (gm < M && gn < N)
            C[gm + static_cast<int64_t>(gn) * ldc] =
                with_c ? alpha * acc[a][b][r] + beta * cv[a][b][r] : alpha * acc[a][b][r];
        }
    }
    if (has_next) store(cur ^ 1);
    __syncthreads();
  };
  if (my_tiles > 0) {
    int m0, n0;
    origin(0, m0, n0);
    load(m0, n0, 0);
    store(0);
    if (with_c) load_c(m0, n0, c0);
    __syncthreads();
  }
  for (int lt = 0; lt < my_tiles; lt += 2) {
    step(lt, 0, c0, c1);
    if (lt + 1 < my_tiles) step(lt + 1, 1, c1, c0);
  }
  team_sync(tm);
}

template <bool TA>
__device__ __forceinline__ void wg_gemm(int M, int N, int K, float alpha, const float* __restrict__ A, int lda,
                                        const float* __restrict__ B, int ldb, float beta, float* __restrict__ C,
                                        int ldc, Lds& s, Team& tm) {
  if (K <= GBK) {  // rank-GBK updates: latency hidden across tiles
    if (M <= 32)
      wg_gemm_short<TA, 32, GBK>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s, tm);
    else
      wg_gemm_short<TA, 64, GBK>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s, tm);
  } else if (K <= 2 * GBK) {  // the rank-2 NB updates of a pair of panels
    if (M <= 32)
      wg_gemm_short<TA, 32, 2 * GBK>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s, tm);
    else
      wg_gemm_short<TA, 64, 2 * GBK>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s, tm);
  } else if (M <= 32) {
    wg_gemm_t<TA, 32>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s, tm);
  } else {
    wg_gemm_t<TA, 64>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s, tm);
  }
}

// One column c of the panel factorisation (c a compile-time constant, so the
// panel stays in registers).  The pivot row c is lane c's first row (c < NB
// <= BT).  Reflector of x (pivot alpha, sigma^2 below it): beta = -sgn(alpha)
// ||x||, tau = (beta - alpha) / beta, v = x / (alpha - beta) (LAPACK's
// convention, sgn(0) = +1); tau = 0 when nothing lies below the pivot.
template <int NB, int C>
__device__ __forceinline__ void panel_column(float (&x)[RPT][NB], Lds& s) {
  const int t = threadIdx.x;
  float sg[1] = {0.f};
#pragma unroll
  for (int sl = 0; sl < RPT; ++sl)
    if (t + sl * BT > C) sg[0] += x[sl][C] * x[sl][C];
  if (t == C) s.alpha = x[0][C];
  block_sum<1>(sg, s);
  const float sigma2 = s.res[0], alpha = s.alpha;
  float tau_c = 0.f, beta = alpha, scale = 0.f;
  if (sigma2 != 0.f) {
    const float nrm = sqrtf(alpha * alpha + sigma2);
    beta = (alpha >= 0.f) ? -nrm : nrm;
    tau_c = (beta - alpha) / beta;
    scale = 1.f / (alpha - beta);
  }
#pragma unroll
  for (int sl = 0; sl < RPT; ++sl) {
    const int r = t + sl * BT;
    if (r > C) x[sl][C] *= scale;
    else if (r == C) x[sl][C] = beta;
  }
  // products of v_c with the later columns (index i >= C: column i + 1) and
  // with the earlier reflectors (index i < C: v_i^T v_c)
  constexpr int CNT = NB - 1;
  float vals[CNT];
#pragma unroll
  for (int i = 0; i < CNT; ++i) vals[i] = 0.f;
#pragma unroll
  for (int sl = 0; sl < RPT; ++sl) {
    const int r = t + sl * BT;
    const float vc = (r > C) ? x[sl][C] : ((r == C) ? 1.f : 0.f);
#pragma unroll
    for (int i = 0; i < CNT; ++i) {
      if (i < C) {
        const float va = (r > i) ? x[sl][i] : ((r == i) ? 1.f : 0.f);
        vals[i] += va * vc;
      } else {
        vals[i] += vc * x[sl][i + 1];
      }
    }
  }
  block_sum<CNT>(vals, s);
#pragma unroll
  for (int d = C + 1; d < NB; ++d) {
    const float w = tau_c * s.res[d - 1];
#pragma unroll
    for (int sl = 0; sl < RPT; ++sl) {
      const int r = t + sl * BT;
      const float vc = (r > C) ? x[sl][C] : ((r == C) ? 1.f : 0.f);
      x[sl][d] -= w * vc;
    }
  }
  if (t < C) s.gram[t][C] = s.res[t];
  if (t == 0) s.tau[C] = tau_c;
}

// The columns C..NB-1 that exist (C < jb), one instantiation per column.
template <int NB, int C>
struct PanelColumns {
  static __device__ __forceinline__ void run(float (&x)[RPT][NB], int jb, Lds& s) {
    if (C < jb) {
      panel_column<NB, C>(x, s);
      PanelColumns<NB, C + 1>::run(x, jb, s);
    }
  }
};
template <int NB>
struct PanelColumns<NB, NB> {
  static __device__ __forceinline__ void run(float (&)[RPT][NB], int, Lds&) {}
};

// Householder factorisation of the panel P (mp x jb, jb <= NB, top-left on the
// diagonal) in registers: on return P holds R on and above the diagonal and
// the reflectors below it, Vp the explicit unit-lower reflectors and Tp
// (ld kLT) the upper triangular T with H_1 ... H_jb = I - V T V^T.
template <int NB>
__device__ __forceinline__ void panel_factor(float* __restrict__ P, int ldp, int mp, int jb,
                                             float* __restrict__ Vp, int ldv, float* __restrict__ Tp, Lds& s) {
  const int t = threadIdx.x;
  float x[RPT][NB];
#pragma unroll
  for (int sl = 0; sl < RPT; ++sl) {
    const int r = t + sl * BT;
#pragma unroll
    for (int c = 0; c < NB; ++c) x[sl][c] = (r < mp && c < jb) ? P[r + static_cast<int64_t>(c) * ldp] : 0.f;
  }
  PanelColumns<NB, 0>::run(x, jb, s);
#pragma unroll
  for (int sl = 0; sl < RPT; ++sl) {
    const int r = t + sl * BT;
    if (r < mp) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < jb) {
          P[r + static_cast<int64_t>(c) * ldp] = x[sl][c];
          Vp[r + static_cast<int64_t>(c) * ldv] = (r > c) ? x[sl][c] : ((r == c) ? 1.f : 0.f);
        }
    }
  }
  __syncthreads();
  // row a = t of T from the Gram entries, built in the lane's own LDS row:
  // T(a,a) = tau_a and, for c > a, T(a,c) = -tau_c sum_{a <= b < c} T(a,b) v_b^T v_c
  if (t < jb) {
    for (int c = 0; c < jb; ++c) {
      float v = 0.f;
      if (c == t) {
        v = s.tau[c];
      } else if (c > t) {
        float acc = 0.f;
        for (int b = t; b < c; ++b) acc += s.trow[t][b] * s.gram[b][c];
        v = -s.tau[c] * acc;
      }
      s.trow[t][c] = v;
      Tp[t + c * kLT] = v;
    }
  }
  __syncthreads();
}

// Qpos of X (rows x cols, ld ldx, rows <= 1024, overwritten): Q (rows x cols,
// ld ldq) explicit with diag(R) >= 0, R (cols x cols, ld ldr, zero below the
// diagonal) when R is not null.
template <int NB>
__device__ __forceinline__ void qr_wg(float* X, int rows, int cols, int ldx, float* Q, int ldq, float* R, int ldr,
                                      const BatchItem& it, Lds& s, Team& tm) {
  const int e0 = tm.member * BT + static_cast<int>(threadIdx.x), es = tm.size * BT;
  const int ldv = rows;
  // Panels A and B of NB columns each form a pair whose joined T
  // [[T_A, -T_A (V_A^T V_B) T_B], [0, T_B]] (ld kLT) lets the rest of the
  // matrix, and later Q, take one rank-2NB update per pair instead of two
  // rank-NB ones.  V_B is kept zero in the rows of A, so V_A and V_B form one
  // unit-lower block from the pair's first row.
  for (int j0 = 0; j0 < cols; j0 += 2 * NB) {
    const int ja = min(NB, cols - j0), jbb = max(0, min(NB, cols - j0 - NB)), jb = ja + jbb;
    const int mp = rows - j0;
    float* P = X + j0 + static_cast<int64_t>(j0) * ldx;
    float* Vp = it.Vr + j0 + static_cast<int64_t>(j0) * ldv;
    float* Tp = it.T + static_cast<int64_t>(j0) * kLT;
    if (tm.member == 0) panel_factor<NB>(P, ldx, mp, ja, Vp, ldv, Tp, s);
    team_sync(tm);
    if (jbb > 0) {
      const int r1 = j0 + ja;
      // B's columns: C_B -= V_A (T_A^T (V_A^T C_B))
      float* CB = X + j0 + static_cast<int64_t>(r1) * ldx;
      wg_gemm<true>(ja, jbb, mp, 1.f, Vp, ldv, CB, ldx, 0.f, it.Wb, kLT, s, tm);
      wg_gemm<true>(ja, jbb, ja, 1.f, Tp, kLT, it.Wb, kLT, 0.f, it.W2b, kLT, s, tm);
      wg_gemm<false>(mp, jbb, ja, -1.f, Vp, ldv, it.W2b, kLT, 1.f, CB, ldx, s, tm);
      float* VB = it.Vr + j0 + static_cast<int64_t>(r1) * ldv;  // from the pair's first row
      float* TB = Tp + ja + static_cast<int64_t>(ja) * kLT;
      if (tm.member == 0) {
        panel_factor<NB>(X + r1 + static_cast<int64_t>(r1) * ldx, ldx, rows - r1, jbb, VB + ja, ldv, TB, s);
        for (int e = threadIdx.x; e < ja * jbb; e += BT) {
          VB[e % ja + static_cast<int64_t>(e / ja) * ldv] = 0.f;  // V_B in the rows of A
          Tp[ja + e % jbb + static_cast<int64_t>(e / jbb) * kLT] = 0.f;  // T's lower-left block
        }
      }
      team_sync(tm);
      // T_AB = -T_A (V_A^T V_B) T_B, V_B zero in the rows of A
      wg_gemm<true>(ja, jbb, mp, 1.f, Vp, ldv, VB, ldv, 0.f, it.Wb, kLT, s, tm);
      wg_gemm<false>(ja, jbb, jbb, 1.f, it.Wb, kLT, TB, kLT, 0.f, it.W2b, kLT, s, tm);
      wg_gemm<false>(ja, jbb, ja, -1.f, Tp, kLT, it.W2b, kLT, 0.f, Tp + static_cast<int64_t>(ja) * kLT, kLT, s, tm);
    }
    const int nrest = cols - j0 - jb;
    if (nrest > 0) {
      // C -= V (T^T (V^T C))
      float* C = X + j0 + static_cast<int64_t>(j0 + jb) * ldx;
      wg_gemm<true>(jb, nrest, mp, 1.f, Vp, ldv, C, ldx, 0.f, it.Wb, kLT, s, tm);
      wg_gemm<true>(jb, nrest, jb, 1.f, Tp, kLT, it.Wb, kLT, 0.f, it.W2b, kLT, s, tm);  // T^T W
      wg_gemm<false>(mp, nrest, jb, -1.f, Vp, ldv, it.W2b, kLT, 1.f, C, ldx, s, tm);
    }
  }
  // Q = H_1 ... H_k [I; 0], accumulated from the last pair back
  for (int e = e0; e < rows * cols; e += es) {
    const int i = e % rows, j = e / rows;
    Q[i + static_cast<int64_t>(j) * ldq] = (i == j) ? 1.f : 0.f;
  }
  team_sync(tm);
  for (int j0 = ((cols - 1) / (2 * NB)) * (2 * NB); j0 >= 0; j0 -= 2 * NB) {
    const int jb = min(2 * NB, cols - j0), mp = rows - j0, nq = cols - j0;
    const float* Vp = it.Vr + j0 + static_cast<int64_t>(j0) * ldv;
    const float* Tp = it.T + static_cast<int64_t>(j0) * kLT;
    float* Qs = Q + j0 + static_cast<int64_t>(j0) * ldq;
    wg_gemm<true>(jb, nq, mp, 1.f, Vp, ldv, Qs, ldq, 0.f, it.Wb, kLT, s, tm);
    wg_gemm<false>(jb, nq, jb, 1.f, Tp, kLT, it.Wb, kLT, 0.f, it.W2b, kLT, s, tm);   // T W
    wg_gemm<false>(mp, nq, jb, -1.f, Vp, ldv, it.W2b, kLT, 1.f, Qs, ldq, s, tm);
  }
  // sign fix: Q(:,j) *= sgn(R(j,j)), R(j,:) = sgn(R(j,j)) R(j,:), sgn(0) = +1
  for (int e = e0; e < rows * cols; e += es) {
    const int i = e % rows, j = e / rows;
    if (X[j + static_cast<int64_t>(j) * ldx] < 0.f) Q[i + static_cast<int64_t>(j) * ldq] *= -1.f;
  }
  if (R) {
    for (int e = e0; e < cols * cols; e += es) {
      const int i = e % cols, j = e / cols;
      float v = 0.f;
      if (i <= j) {
        v = X[i + static_cast<int64_t>(j) * ldx];
        if (X[i + static_cast<int64_t>(i) * ldx] < 0.f) v = -v;
      }
      R[i + static_cast<int64_t>(j) * ldr] = v;
    }
  }
  team_sync(tm);
}

template <int NB>
__device__ __forceinline__ void factor_one(const BatchItem& it, int q, Lds& s, Team& tm) {
  const int m = it.m, n = it.n;
  const int64_t e0 = tm.member * BT + static_cast<int64_t>(threadIdx.x), es = tm.size * BT;
  // G: FP32 rounding of the FP64 Gaussian of stream 2 under key (seed, 0)
  const int64_t total = static_cast<int64_t>(n) * n;
  for (int64_t blk = e0; 4 * blk < total; blk += es) {
    double z[4];
    gaussian_block(static_cast<uint64_t>(blk), 2u, it.seed, z);
#pragma unroll
    for (int l = 0; l < 4; ++l)
      if (4 * blk + l < total) it.Vc[4 * blk + l] = static_cast<float>(z[l]);
  }
  team_sync(tm);
  // 2q + 1 QRs (2 for q = 0), each after its product, in one loop so that the
  // QR's code appears once: X-jobs factor A V (the last one into U, R),
  // Y-jobs factor A^T W (or G itself when q = 0) into the next V.
  const float* Vin = it.Vc;
  const int nqr = (q == 0) ? 2 : 2 * q + 1;
  for (int job = 0; job < nqr; ++job) {
    const bool last = job == nqr - 1;
    const bool on_x = last || (q > 0 && job % 2 == 0);
    float *Xp, *Qp, *Rp = nullptr;
    int rows;
    if (on_x) {
      wg_gemm<false>(m, n, n, 1.f, it.A, m, Vin, n, 0.f, it.X, m, s, tm);  // X = A V
      Xp = it.X;
      rows = m;
      Qp = last ? it.U : it.Q;                                          // W = Qpos(X), or U
      if (last) Rp = it.R;
    } else {
      if (q == 0) {                                                     // DDH-URV (Section 2.2): Qpos(G)
        for (int64_t e = e0; e < total; e += es) it.Y[e] = it.Vc[e];
        team_sync(tm);
      } else {
        wg_gemm<true>(n, n, m, 1.f, it.A, m, it.Q, m, 0.f, it.Y, n, s, tm);  // Y = A^T W
      }
      Xp = it.Y;
      rows = n;
      Qp = (job == nqr - 2) ? it.V : it.Vc;                             // V = Qpos(Y)
    }
    qr_wg<NB>(Xp, rows, n, rows, Qp, rows, Rp, n, it, s, tm);
    if (!on_x) Vin = Qp;
  }
}

// The queue is a list of tickets in largest-first order: matrix order[k] has
// team_size[k] consecutive tickets, one per member.  A workgroup draws the next
// ticket, joins that matrix's team, and draws again when it is done.  Tickets
// are drawn in order by co-resident workgroups, so every team's members are
// all running or finishing an earlier (complete) team: a team barrier never
// waits on a workgroup that cannot arrive.
// counters[0]: next ticket; counters[1]: workgroups that have left;
// counters[2]: error flag (a bounded team wait expired).  bars[k]: arrivals
// at the barriers of queue entry k.  The last workgroup to leave clears the
// counters and the barriers for the next launch.
struct Ticket {
  int entry;   // queue position k
  int member;  // rank in the team
};

template <int NB>
__global__ __launch_bounds__(BT) void batched_urv_kernel(const BatchItem* __restrict__ items,
                                                         const int* __restrict__ order, const int* __restrict__ team_size,
                                                         const Ticket* __restrict__ tickets, int ntickets, int count,
                                                         int q, unsigned* __restrict__ counters,
                                                         unsigned* __restrict__ bars) {
  __shared__ Lds s;
  for (;;) {
    if (threadIdx.x == 0) s.idx = static_cast<int>(atomicAdd(&counters[0], 1u));
    __syncthreads();
    const int tk = s.idx;
    __syncthreads();
    if (tk >= ntickets) break;
    const Ticket ticket = tickets[tk];
    Team tm;
    tm.member = ticket.member;
    tm.size = team_size[ticket.entry];
    tm.bar = bars + ticket.entry;
    tm.err = counters + 2;
    const BatchItem it = items[order[ticket.entry]];
    factor_one<NB>(it, q, s, tm);
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&counters[1], 1u) == gridDim.x - 1) {
      for (int k = 0; k < count; ++k) atomicExch(&bars[k], 0u);
      atomicExch(&counters[0], 0u);
      atomicExch(&counters[1], 0u);
    }
  }
}

size_t item_scratch_floats(int64_t m, int64_t n) {
  auto a = [](int64_t e) { return static_cast<int64_t>(align_up(static_cast<size_t>(e), 64)); };
  return static_cast<size_t>(3 * a(m * n) + 2 * a(n * n) + 3 * a(kLT * n));
}

struct DeviceQueue {
  const BatchItem* items;
  const int* order;
  const int* team_size;
  const Ticket* tickets;
  int ntickets;
  int count;
  unsigned* counters;
  unsigned* bars;
};

int launch_batched(int nb, int grid, const DeviceQueue& dq, int q, hipStream_t s) {
  if (nb == 16)
    batched_urv_kernel<16><<<grid, BT, 0, s>>>(dq.items, dq.order, dq.team_size, dq.tickets, dq.ntickets, dq.count,
                                                q, dq.counters, dq.bars);
  else
    batched_urv_kernel<32><<<grid, BT, 0, s>>>(dq.items, dq.order, dq.team_size, dq.tickets, dq.ntickets, dq.count,
                                                q, dq.counters, dq.bars);
  URV_LAUNCHED("batched_urv_kernel");
  return URV_OK;
}

// Workgroups of the kernel for this panel width that fit on the device at once.
int resident_capacity(int nb, int device) {
  int per_cu = 0, cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e == hipSuccess)
    e = (nb == 16) ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batched_urv_kernel<16>, BT, 0)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batched_urv_kernel<32>, BT, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // clear the sticky error: no capacity means no team schedules
    return 0;
  }
  return per_cu * cus;
}

}  // namespace
}  // namespace urv

struct urv_batch_plan {
  int64_t count = 0;
  int32_t q = 0;
  uint64_t seed = 0;
  int device = 0;
  std::vector<urv::BatchItem> items;
  std::vector<int> order;      // queue position -> matrix, largest first
  std::vector<double> cost;    // per queue position
  char* scratch = nullptr;
  urv::BatchItem* d_items = nullptr;
  int* d_order = nullptr;
  int* d_team = nullptr;            // team size per queue position
  urv::Ticket* d_tickets = nullptr; // capacity count * kMaxTeam
  int ntickets = 0;
  unsigned* d_counters = nullptr;   // next ticket, workgroups out, error flag
  unsigned* d_bars = nullptr;       // per queue position
  bool buffers = false;
  int nb = 32;
  int grid = 256;
  int team_max = 1;
  int capacity[2] = {0, 0};         // co-resident workgroups for nb = 16, 32
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {
using urv::clear_last_error;
using urv::set_last_error;

constexpr int kMaxTeam = 64;

void drop_graph(urv_batch_plan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);  // teardown: nothing to do on failure
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
}

int check_plan(const urv_batch_plan* p, const char* who) {
  if (!p) {
    set_last_error(std::string(who) + ": null plan");
    return URV_EINVAL;
  }
  if (!p->buffers) {
    set_last_error(std::string(who) + ": urv_batch_set_buffers has not been called");
    return URV_EINVAL;
  }
  return URV_OK;
}

int capacity_of(const urv_batch_plan* p, int nb) { return p->capacity[nb == 16 ? 0 : 1]; }

// Team sizes for a configuration: a matrix whose cost exceeds the average
// load of one workgroup (total cost / grid) gets ceil(cost / load) members,
// at most team_max and grid; then the tickets, in queue order.
int build_queue(urv_batch_plan* p, int nb, int grid, int team_max) {
  double total = 0.0;
  for (double c : p->cost) total += c;
  const double load = total / grid;
  std::vector<int> team(static_cast<size_t>(p->count));
  std::vector<urv::Ticket> tickets;
  const int cap = std::max(1, std::min({team_max, grid, kMaxTeam}));
  for (int64_t k = 0; k < p->count; ++k) {
    int sz = 1;
    if (cap > 1 && load > 0.0) sz = static_cast<int>(std::min<double>(cap, std::max(1.0, std::ceil(p->cost[k] / load))));
    team[static_cast<size_t>(k)] = sz;
    for (int r = 0; r < sz; ++r) tickets.push_back(urv::Ticket{static_cast<int>(k), r});
  }
  if (cap > 1 && grid > capacity_of(p, nb)) {
    set_last_error("urv_batch: teams of workgroups need every workgroup resident at once (grid <= " +
                   std::to_string(capacity_of(p, nb)) + " here)");
    return URV_EINVAL;
  }
  URV_HIP(hipMemcpy(p->d_team, team.data(), sizeof(int) * team.size(), hipMemcpyHostToDevice));
  URV_HIP(hipMemcpy(p->d_tickets, tickets.data(), sizeof(urv::Ticket) * tickets.size(), hipMemcpyHostToDevice));
  p->ntickets = static_cast<int>(tickets.size());
  return URV_OK;
}

urv::DeviceQueue queue_of(const urv_batch_plan* p) {
  return urv::DeviceQueue{p->d_items, p->d_order, p->d_team, p->d_tickets, p->ntickets,
                          static_cast<int>(p->count), p->d_counters, p->d_bars};
}

void free_plan(urv_batch_plan* p) {
  drop_graph(p);
  // teardown: failures here cannot be reported to anyone, and are ignored
  if (p->cap) (void)hipStreamDestroy(p->cap);
  (void)hipFree(p->scratch);
  (void)hipFree(p->d_items);
  (void)hipFree(p->d_order);
  (void)hipFree(p->d_team);
  (void)hipFree(p->d_tickets);
  (void)hipFree(p->d_counters);
  (void)hipFree(p->d_bars);
  delete p;
}

const int kCandNB[] = {16, 32};
const int kCandTeam[] = {1, 2, 4, 8, 16};
}  // namespace

extern "C" {

int urv_batch_create(int64_t count, const int64_t* m, const int64_t* n, int32_t q, uint64_t seed,
                     urv_batch_plan** plan) {
  clear_last_error();
  if (!plan) {
    set_last_error("urv_batch_create: null plan pointer");
    return URV_EINVAL;
  }
  *plan = nullptr;
  if (count < 1 || count > (int64_t{1} << 24) || !m || !n || q < 0) {
    set_last_error("urv_batch_create: need count >= 1, size arrays and q >= 0");
    return URV_EINVAL;
  }
  for (int64_t i = 0; i < count; ++i) {
    if (n[i] < 1 || m[i] < n[i]) {
      set_last_error("urv_batch_create: every matrix needs 1 <= n <= m");
      return URV_EINVAL;
    }
    if (m[i] > urv::kBatchMaxRows) {
      set_last_error("urv_batch_create: the batched kernel takes at most 1024 rows per matrix");
      return URV_ENOTSUP;
    }
  }
  auto* p = new urv_batch_plan();
  p->count = count;
  p->q = q;
  p->seed = seed;
  p->items.resize(static_cast<size_t>(count));
  size_t floats = 0;
  std::vector<size_t> off(static_cast<size_t>(count));
  for (int64_t i = 0; i < count; ++i) {
    off[static_cast<size_t>(i)] = floats;
    floats += urv::item_scratch_floats(m[i], n[i]);
  }
  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->scratch), std::max<size_t>(floats, 1) * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->d_items), sizeof(urv::BatchItem) * count);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->d_order), sizeof(int) * count);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->d_team), sizeof(int) * count);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->d_tickets), sizeof(urv::Ticket) * count * kMaxTeam);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->d_counters), 3 * sizeof(unsigned));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->d_bars), sizeof(unsigned) * count);
  if (e == hipSuccess) e = hipMemset(p->d_counters, 0, 3 * sizeof(unsigned));
  if (e == hipSuccess) e = hipMemset(p->d_bars, 0, sizeof(unsigned) * count);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    p->capacity[k] = urv::resident_capacity(k == 0 ? 16 : 32, p->device);
    if (p->capacity[k] < 1) e = hipErrorInvalidDeviceFunction;
  }
  if (e != hipSuccess) {
    const int rc = urv::hip_status(e, "urv_batch_create");
    free_plan(p);
    return rc;
  }
  for (int64_t i = 0; i < count; ++i) {
    urv::BatchItem& it = p->items[static_cast<size_t>(i)];
    it.m = static_cast<int>(m[i]);
    it.n = static_cast<int>(n[i]);
    it.seed = seed + static_cast<uint64_t>(i);
    float* base = reinterpret_cast<float*>(p->scratch) + off[static_cast<size_t>(i)];
    auto take = [&](int64_t elems) {
      float* r = base;
      base += urv::align_up(static_cast<size_t>(elems), 64);
      return r;
    };
    it.X = take(m[i] * n[i]);
    it.Q = take(m[i] * n[i]);
    it.Vr = take(m[i] * n[i]);
    it.Y = take(n[i] * n[i]);
    it.Vc = take(n[i] * n[i]);
    it.T = take(urv::kLT * n[i]);
    it.Wb = take(urv::kLT * n[i]);
    it.W2b = take(urv::kLT * n[i]);
  }
  // largest first (LPT): cost ~ m n^2, ties by index
  p->order.resize(static_cast<size_t>(count));
  std::iota(p->order.begin(), p->order.end(), 0);
  std::stable_sort(p->order.begin(), p->order.end(), [&](int a, int b) {
    return static_cast<double>(m[a]) * n[a] * n[a] > static_cast<double>(m[b]) * n[b] * n[b];
  });
  p->cost.resize(static_cast<size_t>(count));
  for (int64_t k = 0; k < count; ++k) {
    const int i = p->order[static_cast<size_t>(k)];
    p->cost[static_cast<size_t>(k)] = static_cast<double>(m[i]) * n[i] * n[i];
  }
  p->grid = p->capacity[1];
  int rc = URV_OK;
  e = hipMemcpy(p->d_order, p->order.data(), sizeof(int) * count, hipMemcpyHostToDevice);
  if (e != hipSuccess) rc = urv::hip_status(e, "urv_batch_create");
  if (rc == URV_OK) rc = build_queue(p, p->nb, p->grid, p->team_max);
  if (rc != URV_OK) {
    free_plan(p);
    return rc;
  }
  *plan = p;
  return URV_OK;
}

int urv_batch_set_buffers(urv_batch_plan* p, const float* const* A, float* const* U, float* const* R,
                          float* const* V) {
  clear_last_error();
  if (!p || !A || !U || !R || !V) {
    set_last_error("urv_batch_set_buffers: null argument");
    return URV_EINVAL;
  }
  for (int64_t i = 0; i < p->count; ++i) {
    if (!A[i] || !U[i] || !R[i] || !V[i]) {
      set_last_error("urv_batch_set_buffers: null matrix pointer");
      return URV_EINVAL;
    }
    urv::BatchItem& it = p->items[static_cast<size_t>(i)];
    it.A = A[i];
    it.U = U[i];
    it.R = R[i];
    it.V = V[i];
  }
  URV_HIP(hipMemcpy(p->d_items, p->items.data(), sizeof(urv::BatchItem) * p->count, hipMemcpyHostToDevice));
  p->buffers = true;
  return URV_OK;
}

int urv_batch_set_config(urv_batch_plan* p, int32_t nb, int32_t grid, int32_t team_max) {
  clear_last_error();
  if (!p || (nb != 16 && nb != 32) || grid < 1 || grid > 65536 || team_max < 1 || team_max > kMaxTeam) {
    set_last_error("urv_batch_set_config: need a plan, nb 16 or 32, 1 <= grid <= 65536, 1 <= team_max <= 64");
    return URV_EINVAL;
  }
  URV_TRY(build_queue(p, nb, grid, team_max));
  if (p->nb != nb || p->grid != grid || p->team_max != team_max) drop_graph(p);
  p->nb = nb;
  p->grid = grid;
  p->team_max = team_max;
  return URV_OK;
}

int urv_batch_get_config(const urv_batch_plan* p, int32_t* nb, int32_t* grid, int32_t* team_max) {
  clear_last_error();
  if (!p || !nb || !grid || !team_max) {
    set_last_error("urv_batch_get_config: null argument");
    return URV_EINVAL;
  }
  *nb = p->nb;
  *grid = p->grid;
  *team_max = p->team_max;
  return URV_OK;
}

int urv_batch_run(urv_batch_plan* p, void* stream) {
  clear_last_error();
  URV_TRY(check_plan(p, "urv_batch_run"));
  return urv::launch_batched(p->nb, p->grid, queue_of(p), p->q, static_cast<hipStream_t>(stream));
}

int urv_batch_run_graph(urv_batch_plan* p, void* stream) {
  clear_last_error();
  URV_TRY(check_plan(p, "urv_batch_run_graph"));
  if (!p->exec) {
    if (!p->cap) URV_HIP(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
    URV_HIP(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    const int rc = urv::launch_batched(p->nb, p->grid, queue_of(p), p->q, p->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap, &g);
    if (rc != URV_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    URV_HIP(e);
    p->graph = g;
    URV_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
  }
  URV_HIP(hipGraphLaunch(p->exec, static_cast<hipStream_t>(stream)));
  return URV_OK;
}

int urv_batch_status(urv_batch_plan* p, void* stream) {
  clear_last_error();
  if (!p) {
    set_last_error("urv_batch_status: null plan");
    return URV_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned flag = 0;
  URV_HIP(hipMemcpyAsync(&flag, p->d_counters + 2, sizeof(flag), hipMemcpyDeviceToHost, s));
  URV_HIP(hipStreamSynchronize(s));
  if (flag != 0) {
    set_last_error("urv_batch: a team barrier's bounded wait expired (another kernel held CUs?)");
    return URV_EDEVICE;
  }
  return URV_OK;
}

int urv_batch_autotune(urv_batch_plan* p, void* stream, double* best_ms) {
  clear_last_error();
  URV_TRY(check_plan(p, "urv_batch_autotune"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  URV_HIP(hipEventCreate(&e0));
  URV_HIP(hipEventCreate(&e1));
  float best = -1.f;
  int best_nb = p->nb, best_team = p->team_max;
  int rc = URV_OK;
  for (int nb : kCandNB) {
    for (int team : kCandTeam) {
      // every workgroup resident: the grid is the device's capacity for this kernel
      rc = build_queue(p, nb, capacity_of(p, nb), team);
      const urv::DeviceQueue dq = queue_of(p);
      // one untimed run, then one timed run of the whole batch
      if (rc == URV_OK) rc = urv::launch_batched(nb, capacity_of(p, nb), dq, p->q, s);
      if (rc == URV_OK && hipEventRecord(e0, s) != hipSuccess) rc = URV_EDEVICE;
      if (rc == URV_OK) rc = urv::launch_batched(nb, capacity_of(p, nb), dq, p->q, s);
      if (rc == URV_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
        rc = urv::hip_status(hipGetLastError(), "urv_batch_autotune");
      if (rc != URV_OK) break;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = urv::hip_status(hipGetLastError(), "urv_batch_autotune");
        break;
      }
      if (best < 0.f || ms < best) {
        best = ms;
        best_nb = nb;
        best_team = team;
      }
    }
    if (rc != URV_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != URV_OK) {
    build_queue(p, p->nb, p->grid, p->team_max);
    return rc;
  }
  if (best_ms) *best_ms = best;
  p->nb = -1;  // force the queue and the graph to follow the choice
  return urv_batch_set_config(p, best_nb, capacity_of(p, best_nb), best_team);
}

void urv_batch_destroy(urv_batch_plan* p) {
  if (!p) return;
  free_plan(p);
}

}  // extern "C"
