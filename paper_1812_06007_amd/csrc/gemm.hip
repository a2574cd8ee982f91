// FP64 and FP32 GEMM on CDNA4 matrix cores: C = alpha op(A) op(B) + beta C.
//
// This is the level-3 kernel behind the products A V and A^T W of the power
// iteration (Section 3, eq. power) and behind the compact-WY block-reflector
// updates of the Householder QR (Section 2.2: reflectors accumulated and
// applied to the trailing matrix with a matrix-matrix multiply).
//
// Design for gfx950:
//  * v_mfma_f64_16x16x4_f64 (FP64) / v_mfma_f32_16x16x4_f32 (FP32) tiles; a
//    workgroup of WGM x WGN waves owns a BM x BN tile of C, each wave a
//    (BM/WGM) x (BN/WGN) sub-tile held in registers.
//  * K is walked in steps of BK = 32 through double-buffered LDS tiles (one
//    barrier per step: 132 KB of LDS for a 128 x 128 tile); the next step's
//    global loads are in flight while the current step's MFMAs run.  Each
//    thread loads pairs of elements that are adjacent along the operand's
//    contiguous index, as one 16-byte load when the operands are 16-byte
//    aligned with even leading dimensions (the bounds-checked edge tiles use
//    the same element mapping, one element at a time).  Measured on MI355X,
//    8000^3 NN: 19.3 ms with BK = 16 and single loads, 18.2 ms like this.
//  * The MFMA is fed (op(B) fragment, op(A) fragment) so that each lane ends
//    with 16 consecutive rows of one column of C: column-major stores of C
//    are 128-byte segments.
//  * Workgroups are mapped to tiles XCD by XCD (the dispatcher deals
//    workgroups round-robin to the 8 XCDs) and in groups of 4 tile rows, so
//    tiles that share rows of op(A) / columns of op(B) share an L2.
//  * When the tile grid alone cannot fill 256 CUs and K is long, K is split
//    into chunks whose partial sums go to scratch and are added in a fixed
//    order by a second kernel: results do not depend on scheduling.
#include "common.hpp"

#include <cstdio>
#include <cstdlib>

namespace urv {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
template <class T> struct Vec2T;
template <> struct Vec2T<double> { using type = double2; };
template <> struct Vec2T<float> { using type = float2; };
typedef float f4 __attribute__((ext_vector_type(4)));

// One 16x16x4 MFMA per element type.  The result layouts differ: lane l, entry
// r holds output row l/16 + 4r for FP64 and row 4(l/16) + r for FP32.
template <class T>
struct Mma;
template <>
struct Mma<double> {
  using acc = d4;
  static __device__ inline acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lk, int r) { return lk + 4 * r; }
};
template <>
struct Mma<float> {
  using acc = f4;
  static __device__ inline acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lk, int r) { return 4 * lk + r; }
};

constexpr int BK = 32;
__device__ inline int lrow0(int lane) { return lane & 15; }
constexpr int PAD = 1;  // LDS row padding (elements): spreads transposed LDS writes over banks

// BKT: the k-step (BK, or 16 for short sums, where the halved LDS lets two
// workgroups share a CU and overlap one's prologue and epilogue with the
// other's MFMAs).  kPreC: with beta != 0, C is loaded at the start, so its
// latency hides behind the (short) k loop instead of following it.
template <class T, bool TA, bool TB, int BM, int BN, int WGM, int WGN, int BKT = BK, bool kPreC = false>
__global__ __launch_bounds__(64 * WGM * WGN)
__attribute__((amdgpu_waves_per_eu(BKT < BK ? 4 : 1))) void gemm_kernel(
    int64_t M, int64_t N, int64_t K, T alpha, const T* __restrict__ A, int64_t lda,
    const T* __restrict__ B, int64_t ldb, T beta, T* __restrict__ C, int64_t ldc,
    T* __restrict__ partial, int64_t k_chunk, int tiles_m, int tiles_n) {
  using acc_t = typename Mma<T>::acc;
  constexpr int NT = 64 * WGM * WGN;             // threads
  constexpr int WM = BM / WGM, WN = BN / WGN;    // wave tile
  constexpr int FM = WM / 16, FN = WN / 16;     // MFMA blocks per wave
  constexpr int LA = BM * BKT / NT, LB = BN * BKT / NT;  // loads per thread per step
  __shared__ T As[2][BKT][BM + PAD];
  __shared__ T Bs[2][BKT][BN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;

  // ---- workgroup -> tile, XCD-major then grouped rows
  const int ntiles = tiles_m * tiles_n;
  const int wg = xcd_tile_order(static_cast<int>(blockIdx.x), ntiles);
  constexpr int GROUP = 4;  // tile rows per group; measured on MI355X (8000^3 NN): 4 beats 8 by 6-8%
  const int group = wg / (GROUP * tiles_n);
  const int first_m = group * GROUP;
  const int gsize = min(tiles_m - first_m, GROUP);
  const int tm = first_m + (wg % (GROUP * tiles_n)) % gsize;
  const int tn = (wg % (GROUP * tiles_n)) / gsize;
  const int64_t m0 = static_cast<int64_t>(tm) * BM;
  const int64_t n0 = static_cast<int64_t>(tn) * BN;

  const int64_t kb = static_cast<int64_t>(blockIdx.y) * k_chunk;
  const int64_t ke = min(K, kb + k_chunk);
  const int nk = static_cast<int>(ceil_div(ke - kb, BKT));

  T ra[LA], rb[LB];
  static_assert(LA % 2 == 0 && LB % 2 == 0, "pairs of loads");
  const bool vec_ok = ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15) == 0 &&
                      ((lda | ldb) & 1) == 0;

  // element slot s of a thread: pair p = s / 2 of the thread, half s % 2; the pair's
  // two elements are consecutive in memory (along the operand's contiguous index)
  auto a_idx = [&](int s, int& i, int& k) {
    const int e = 2 * (tid + NT * (s >> 1)) + (s & 1);
    if (!TA) { i = e % BM; k = e / BM; } else { k = e % BKT; i = e / BKT; }
  };
  auto b_idx = [&](int s, int& j, int& k) {
    const int e = 2 * (tid + NT * (s >> 1)) + (s & 1);
    if (TB) { j = e % BN; k = e / BN; } else { k = e % BKT; j = e / BKT; }
  };
  using V2 = typename Vec2T<T>::type;
  const bool aligned = vec_ok;
  const bool full_mn = (m0 + BM <= M) && (n0 + BN <= N);
  auto load_global = [&](int64_t k0) {
    if (aligned && full_mn && k0 + BKT <= ke) {
#pragma unroll
      for (int s = 0; s < LA; s += 2) {
        int i, k;
        a_idx(s, i, k);
        const int64_t gi = m0 + i, gk = k0 + k;
        const V2 v = *reinterpret_cast<const V2*>(TA ? A + gk + gi * lda : A + gi + gk * lda);
        ra[s] = v.x;
        ra[s + 1] = v.y;
      }
#pragma unroll
      for (int s = 0; s < LB; s += 2) {
        int j, k;
        b_idx(s, j, k);
        const int64_t gj = n0 + j, gk = k0 + k;
        const V2 v = *reinterpret_cast<const V2*>(TB ? B + gj + gk * ldb : B + gk + gj * ldb);
        rb[s] = v.x;
        rb[s + 1] = v.y;
      }
      return;
    }
#pragma unroll
    for (int s = 0; s < LA; ++s) {
      int i, k;
      a_idx(s, i, k);
      const int64_t gi = m0 + i, gk = k0 + k;
      T v = 0;
      if (gi < M && gk < ke) v = TA ? A[gk + gi * lda] : A[gi + gk * lda];
      ra[s] = v;
    }
#pragma unroll
    for (int s = 0; s < LB; ++s) {
      int j, k;
      b_idx(s, j, k);
      const int64_t gj = n0 + j, gk = k0 + k;
      T v = 0;
      if (gj < N && gk < ke) v = TB ? B[gj + gk * ldb] : B[gk + gj * ldb];
      rb[s] = v;
    }
  };
  auto store_lds = [&](int buf) {
#pragma unroll
    for (int s = 0; s < LA; ++s) {
      int i, k;
      a_idx(s, i, k);
      As[buf][k][i] = ra[s];
    }
#pragma unroll
    for (int s = 0; s < LB; ++s) {
      int j, k;
      b_idx(s, j, k);
      Bs[buf][k][j] = rb[s];
    }
  };

  acc_t acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

  if (nk > 0) {
    load_global(kb);
    store_lds(0);
  }
  // C of a short sum: loaded now, its latency hidden behind the k loop
  acc_t cpre[FM][FN];
  const bool pre_c = kPreC && partial == nullptr && full_mn && beta != T(0);
  if (pre_c) {
    const T* cb = C + (m0 + wm * WM + lrow0(lane)) + (n0 + wn * WN) * ldc;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) cpre[a][b][r] = cb[a * 16 + (b * 16 + Mma<T>::row(lane >> 4, r)) * ldc];
  }
  __syncthreads();

  const int lrow = lane & 15;  // index within a 16-block
  const int lk = lane >> 4;    // k within a 4-step
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load_global(kb + static_cast<int64_t>(kt + 1) * BKT);
#pragma unroll
    for (int kk = 0; kk < BKT / 4; ++kk) {
      T fa[FM], fb[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) fa[a] = As[cur][kk * 4 + lk][wm * WM + a * 16 + lrow];
#pragma unroll
      for (int b = 0; b < FN; ++b) fb[b] = Bs[cur][kk * 4 + lk][wn * WN + b * 16 + lrow];
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
          acc[a][b] = Mma<T>::run(fb[b], fa[a], acc[a][b]);
    }
    if (kt + 1 < nk) store_lds(cur ^ 1);
    __syncthreads();
  }

  // ---- epilogue: lane holds C(m0 + .. + lrow, n0 + .. + lk + 4r).  All loads of C
  // are issued before any store, so the read-modify-write costs one round trip.
  if (partial) {
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      const int64_t gm = m0 + wm * WM + a * 16 + lrow;
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gn = n0 + wn * WN + b * 16 + Mma<T>::row(lk, r);
          if (gm < M && gn < N) partial[(static_cast<int64_t>(blockIdx.y) * N + gn) * M + gm] = acc[a][b][r];
        }
    }
    return;
  }
  if (full_mn) {
    T* cbase = C + (m0 + wm * WM + lrow) + (n0 + wn * WN) * ldc;
    if (beta != T(0)) {
      // all of a group's loads of C before its stores; the short-sum variant (two
      // workgroups per CU, half the registers) takes one row block of the wave at a time
      constexpr int EG = (BKT < BK) ? 1 : FM;
#pragma unroll
      for (int a0 = 0; a0 < FM; a0 += EG) {
        acc_t cv[EG][FN];
#pragma unroll
        for (int a = 0; a < EG; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              cv[a][b][r] = pre_c ? cpre[a0 + a][b][r]
                                  : cbase[(a0 + a) * 16 + (b * 16 + Mma<T>::row(lk, r)) * ldc];
#pragma unroll
        for (int a = 0; a < EG; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              cbase[(a0 + a) * 16 + (b * 16 + Mma<T>::row(lk, r)) * ldc] =
                  alpha * acc[a0 + a][b][r] + beta * cv[a][b][r];
      }
    } else {
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) cbase[a * 16 + (b * 16 + Mma<T>::row(lk, r)) * ldc] = alpha * acc[a][b][r];
    }
    return;
  }
  if (beta != T(0)) {
    acc_t cv[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      const int64_t gm = m0 + wm * WM + a * 16 + lrow;
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gn = n0 + wn * WN + b * 16 + Mma<T>::row(lk, r);
          cv[a][b][r] = (gm < M && gn < N) ? C[gm + gn * ldc] : 0.0;
        }
    }
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      const int64_t gm = m0 + wm * WM + a * 16 + lrow;
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gn = n0 + wn * WN + b * 16 + Mma<T>::row(lk, r);
          if (gm < M && gn < N) C[gm + gn * ldc] = alpha * acc[a][b][r] + beta * cv[a][b][r];
        }
    }
  } else {
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      const int64_t gm = m0 + wm * WM + a * 16 + lrow;
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gn = n0 + wn * WN + b * 16 + Mma<T>::row(lk, r);
          if (gm < M && gn < N) C[gm + gn * ldc] = alpha * acc[a][b][r];
        }
    }
  }
}

// C = alpha * sum_z P[z] + beta * C, z ascending.
template <class T>
__global__ void splitk_reduce_kernel(int64_t M, int64_t N, int splits, T alpha,
                                     const T* __restrict__ P, T beta,
                                     T* __restrict__ C, int64_t ldc) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t i = idx % M, j = idx / M;
  T s = 0;
  for (int z = 0; z < splits; ++z) s += P[z * M * N + idx];
  T* c = C + i + j * ldc;
  *c = (beta == T(0)) ? alpha * s : alpha * s + beta * *c;
}

template <class T>
__global__ void scale_kernel(int64_t M, int64_t N, T beta, T* __restrict__ C,
                             int64_t ldc) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= M * N) return;
  T* c = C + idx % M + (idx / M) * ldc;
  *c = (beta == T(0)) ? T(0) : beta * *c;
}

struct Plan {
  int bm, bn, wgm, wgn, tiles_m, tiles_n, splits;
  int64_t k_chunk;
  bool short_k = false;  // 128 x 64 tiles, k-step 16, 8 waves (two workgroups per CU), C loaded first
};

Plan make_plan(int64_t M, int64_t N, int64_t K) {
  Plan p;
  p.bm = (M <= 64) ? 64 : 128;
  p.bn = (N <= 64) ? 64 : 128;
  // Short sums cannot be split over k: use smaller tiles to fill more CUs instead.
  if (K < 512) {
    if (p.bm == 128 && ceil_div(M, 128) * ceil_div(N, p.bn) < 256) p.bm = 64;
    if (p.bn == 128 && ceil_div(M, p.bm) * ceil_div(N, 128) < 256) p.bn = 64;
  }
  // waves per workgroup: 16 for full 128 x 128 tiles, 8 otherwise (measured best on MI355X)
  p.wgm = (p.bm == 128) ? 4 : 2;
  p.wgn = (p.bn == 128) ? 4 : 2;
  if (p.bm == 64 && p.bn == 128) p.wgn = 4;
  if (const char* e = std::getenv("URV_GEMM_WAVES")) {  // tuning only: "WGMxWGN"
    int a = 0, b = 0;
    if (std::sscanf(e, "%dx%d", &a, &b) == 2 && (a == 2 || a == 4) && (b == 2 || b == 4)) {
      p.wgm = a;
      p.wgn = b;
    }
  }
  p.tiles_m = static_cast<int>(ceil_div(M, p.bm));
  p.tiles_n = static_cast<int>(ceil_div(N, p.bn));
  const int64_t tiles = static_cast<int64_t>(p.tiles_m) * p.tiles_n;
  p.splits = 1;
  const int64_t target = 512;  // workgroups wanted in flight (256 CUs, 2 per CU)
  if (tiles > 0 && tiles < 256 && K >= 512) {
    int64_t s = ceil_div(target, tiles);
    s = std::min<int64_t>(s, K / 256);
    s = std::min<int64_t>(s, 64);
    p.splits = static_cast<int>(std::max<int64_t>(s, 1));
  }
  p.k_chunk = ceil_div(ceil_div(K, p.splits), BK) * BK;
  if (K > 0) p.splits = static_cast<int>(ceil_div(K, p.k_chunk));
  // Sums of at most 256 over many 128 x 128 tiles (the block-reflector updates): a
  // workgroup's prologue and epilogue are as long as its k loop, so 128 x 64 tiles with
  // a k-step of 16 (8 waves, 50 KB of LDS, at most 128 registers) let two workgroups
  // share each CU, one's MFMAs covering the other's loads and stores of C
  // (URV_GEMM_SHORTK=0: off, for tuning).
  const char* sk = std::getenv("URV_GEMM_SHORTK");
  p.short_k = K > 0 && K <= 256 && p.bm == 128 && p.bn == 128 && p.splits == 1 && !(sk && std::atoi(sk) == 0);
  if (p.short_k) {
    p.bn = 64;
    p.wgm = 4;
    p.wgn = 2;
    p.tiles_n = static_cast<int>(ceil_div(N, 64));
  }
  return p;
}

template <class T, bool TA, bool TB>
void launch_tiles(const Plan& p, int64_t M, int64_t N, int64_t K, T alpha, const T* A,
                  int64_t lda, const T* B, int64_t ldb, T beta, T* C, int64_t ldc,
                  T* partial, hipStream_t s) {
  const dim3 grid(p.tiles_m * p.tiles_n, p.splits);
  if (p.short_k) {
    // C loaded before the k loop (URV_GEMM_PREC=0: after it, for tuning); measured on
    // MI355X in the FP64 factorisation at n = 8000: FULL 252.3-252.7 ms against 253.6-254.0
    static const bool prec = [] {
      const char* e = std::getenv("URV_GEMM_PREC");
      return !(e && std::atoi(e) == 0);
    }();
    if (prec)
      gemm_kernel<T, TA, TB, 128, 64, 4, 2, 16, true><<<grid, 64 * 8, 0, s>>>(
          M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, partial, p.k_chunk, p.tiles_m, p.tiles_n);
    else
      gemm_kernel<T, TA, TB, 128, 64, 4, 2, 16, false><<<grid, 64 * 8, 0, s>>>(
          M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, partial, p.k_chunk, p.tiles_m, p.tiles_n);
    return;
  }
#define URV_GEMM_CASE(TBM, TBN, GM, GN)                                                          \
  if (p.bm == TBM && p.bn == TBN && p.wgm == GM && p.wgn == GN) {                               \
    gemm_kernel<T, TA, TB, TBM, TBN, GM, GN><<<grid, 64 * GM * GN, 0, s>>>(                       \
        M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, partial, p.k_chunk, p.tiles_m, p.tiles_n); \
    return;                                                                                     \
  }
  URV_GEMM_CASE(128, 128, 2, 2)
  URV_GEMM_CASE(128, 128, 2, 4)
  URV_GEMM_CASE(128, 128, 4, 2)
  URV_GEMM_CASE(128, 128, 4, 4)
  URV_GEMM_CASE(64, 128, 2, 2)
  URV_GEMM_CASE(64, 128, 2, 4)
  URV_GEMM_CASE(128, 64, 2, 2)
  URV_GEMM_CASE(128, 64, 4, 2)
  URV_GEMM_CASE(64, 64, 2, 2)
#undef URV_GEMM_CASE
  // any other combination (only reachable through the tuning variable): 2 x 2 waves
  Plan q = p;
  q.wgm = q.wgn = 2;
  launch_tiles<T, TA, TB>(q, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, partial, s);
}

}  // namespace

size_t gemm_work_elems(int64_t M, int64_t N, int64_t K) {
  const Plan p = make_plan(M, N, K);
  return p.splits > 1 ? static_cast<size_t>(p.splits) * M * N : 0;
}

size_t gemm_partials_elems(int64_t M, int64_t N, int64_t K) {
  const Plan p = make_plan(M, N, K);
  return static_cast<size_t>(std::max(p.splits, 1)) * M * N;
}

template <class T>
int gemm_partials(bool ta, bool tb, int64_t M, int64_t N, int64_t K, const T* A, int64_t lda, const T* B,
                  int64_t ldb, T* partial, size_t work_elems, int* splits, hipStream_t s) {
  *splits = 0;
  if (M == 0 || N == 0) return URV_OK;
  const size_t mn = static_cast<size_t>(M) * N;
  if (partial == nullptr || work_elems < mn) {
    set_last_error("gemm_partials: scratch smaller than one M x N slice");
    return URV_EINVAL;
  }
  if (K == 0) {
    scale_kernel<<<static_cast<unsigned>(ceil_div(M * N, 256)), 256, 0, s>>>(M, N, T(0), partial, M);
    URV_LAUNCHED("scale_kernel");
    *splits = 1;
    return URV_OK;
  }
  Plan p = make_plan(M, N, K);
  const int64_t cap = static_cast<int64_t>(work_elems / mn);
  if (p.splits > cap) {
    p.k_chunk = ceil_div(ceil_div(K, cap), BK) * BK;
    p.splits = static_cast<int>(ceil_div(K, p.k_chunk));
  }
  const int tok = sizeof(T) == 8 ? timing_begin(s) : -1;
  if (!ta && !tb) launch_tiles<T, false, false>(p, M, N, K, T(1), A, lda, B, ldb, T(0), nullptr, M, partial, s);
  else if (ta && !tb) launch_tiles<T, true, false>(p, M, N, K, T(1), A, lda, B, ldb, T(0), nullptr, M, partial, s);
  else if (!ta && tb) launch_tiles<T, false, true>(p, M, N, K, T(1), A, lda, B, ldb, T(0), nullptr, M, partial, s);
  else launch_tiles<T, true, true>(p, M, N, K, T(1), A, lda, B, ldb, T(0), nullptr, M, partial, s);
  timing_end(tok, ta ? (tb ? kTimedGemmTT : kTimedGemmTN) : (tb ? kTimedGemmNT : kTimedGemmNN),
             2.0 * static_cast<double>(M) * N * K, s);
  URV_LAUNCHED("gemm_kernel");
  *splits = p.splits;
  return URV_OK;
}

template int gemm_partials<double>(bool, bool, int64_t, int64_t, int64_t, const double*, int64_t, const double*,
                                   int64_t, double*, size_t, int*, hipStream_t);
template int gemm_partials<float>(bool, bool, int64_t, int64_t, int64_t, const float*, int64_t, const float*,
                                  int64_t, float*, size_t, int*, hipStream_t);

template <class T>
int gemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, T alpha, const T* A, int64_t lda,
         const T* B, int64_t ldb, T beta, T* C, int64_t ldc, T* work, size_t work_elems,
         hipStream_t s) {
  if (M == 0 || N == 0) return URV_OK;
  if (K == 0 || alpha == T(0)) {
    const int64_t total = M * N;
    scale_kernel<<<static_cast<unsigned>(ceil_div(total, 256)), 256, 0, s>>>(M, N, beta, C, ldc);
    URV_LAUNCHED("scale_kernel");
    return URV_OK;
  }
  Plan p = make_plan(M, N, K);
  if (p.splits > 1 && (work == nullptr || work_elems < static_cast<size_t>(p.splits) * M * N)) {
    p.splits = 1;
    p.k_chunk = ceil_div(K, BK) * BK;
  }
  T* partial = p.splits > 1 ? work : nullptr;
  const int tok = sizeof(T) == 8 ? timing_begin(s) : -1;
  if (!ta && !tb) launch_tiles<T, false, false>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, partial, s);
  else if (ta && !tb) launch_tiles<T, true, false>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, partial, s);
  else if (!ta && tb) launch_tiles<T, false, true>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, partial, s);
  else launch_tiles<T, true, true>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, partial, s);
  URV_LAUNCHED("gemm_kernel");
  timing_end(tok, ta ? (tb ? kTimedGemmTT : kTimedGemmTN) : (tb ? kTimedGemmNT : kTimedGemmNN),
             2.0 * static_cast<double>(M) * N * K, s);
  if (partial) {
    const int64_t total = M * N;
    splitk_reduce_kernel<<<static_cast<unsigned>(ceil_div(total, 256)), 256, 0, s>>>(
        M, N, p.splits, alpha, partial, beta, C, ldc);
    URV_LAUNCHED("splitk_reduce_kernel");
  }
  return URV_OK;
}

template int gemm<double>(bool, bool, int64_t, int64_t, int64_t, double, const double*, int64_t,
                          const double*, int64_t, double, double*, int64_t, double*, size_t,
                          hipStream_t);
template int gemm<float>(bool, bool, int64_t, int64_t, int64_t, float, const float*, int64_t,
                         const float*, int64_t, float, float*, int64_t, float*, size_t,
                         hipStream_t);

}  // namespace urv
