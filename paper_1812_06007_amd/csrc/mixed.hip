// Kernels of the mixed-precision form: the products of the power iteration
// (A V and A^T W of Section 3, eq. power) on BF16 / FP16 matrix cores with
// FP32 accumulation, and the precision conversions around them.
//
// gemm_lowp computes C = alpha A^T B + beta C for 16-bit A (K x M) and B
// (K x N), both column-major with K contiguous, so one lane's MFMA operand (8
// consecutive k) is one 16-byte load.  A V is computed as (A^T)^T V from a
// transposed 16-bit copy of A made once, A^T W directly from the 16-bit A.
// The 16-bit buffers have leading dimensions padded to a multiple of 32 and
// zero padding, so every K step of 32 is a full, unguarded load.
#include "common.hpp"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

namespace urv {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

template <bool BF16>
struct Lowp;
template <>
struct Lowp<true> {
  using elem = __bf16;
  using vec8 = bf8;
  static __device__ inline f4 mma(vec8 a, vec8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Lowp<false> {
  using elem = _Float16;
  using vec8 = h8;
  static __device__ inline f4 mma(vec8 a, vec8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

constexpr int LBK = 64;
constexpr int LPAD = 8;  // 16-byte row padding in LDS: 144-byte rows, conflict-free 16-byte reads

// v_mfma_f32_16x16x32_{bf16,f16}: lane l holds A(i = l%16, k = 8(l/16) + e), e = 0..7,
// B(k = 8(l/16) + e, j = l%16); result entry r of lane l is D(4(l/16) + r, l%16).
// The MFMA is fed (B fragment, A fragment), so lane l ends with C(m = l%16, n = 4(l/16)+r):
// sixteen consecutive rows of C per column.
// An LBM x LBN tile of C per workgroup of WGM x WGN waves, each wave a (LBM / WGM) x
// (LBN / WGN) sub-tile: the larger the wave tile, the fewer LDS bytes per MFMA.
template <bool BF16, int LBM, int LBN, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_lowp_kernel(int64_t M, int64_t N, int64_t K, float alpha,
                                                                  const void* __restrict__ Av, int64_t lda,
                                                                  const void* __restrict__ Bv, int64_t ldb,
                                                                  float beta, float* __restrict__ C,
                                                                  int64_t ldc, int tiles_m, int tiles_n) {
  using E = typename Lowp<BF16>::elem;
  using V8 = typename Lowp<BF16>::vec8;
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WTM = LBM / WGM, WTN = LBN / WGN;  // wave tile
  constexpr int FA = WTM / 16, FB = WTN / 16;      // MFMA blocks per wave
  constexpr int LA = LBM * LBK / 8 / NT, LB = LBN * LBK / 8 / NT;  // 16-byte chunks per thread and K step
  static_assert(LA * NT * 8 == LBM * LBK && LB * NT * 8 == LBN * LBK, "whole chunks per thread");
  const E* A = static_cast<const E*>(Av);
  const E* B = static_cast<const E*>(Bv);
  __shared__ __attribute__((aligned(16))) E As[2][LBM][LBK + LPAD];
  __shared__ __attribute__((aligned(16))) E Bs[2][LBN][LBK + LPAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int ntiles = tiles_m * tiles_n;
  // XCD-contiguous ranges of the tile sequence, walked in groups of 8 tile rows
  const int wg = xcd_tile_order(static_cast<int>(blockIdx.x), ntiles);
  constexpr int GROUP = 8;
  const int first_m = (wg / (GROUP * tiles_n)) * GROUP;
  const int gsize = min(tiles_m - first_m, GROUP);
  const int tm = first_m + (wg % (GROUP * tiles_n)) % gsize;
  const int tn = (wg % (GROUP * tiles_n)) / gsize;
  const int64_t m0 = static_cast<int64_t>(tm) * LBM, n0 = static_cast<int64_t>(tn) * LBN;
  const int nk = static_cast<int>(ceil_div(K, LBK));
  // K padded to a multiple of 32 with zeros: a 16-byte chunk lies wholly below kp or wholly
  // at or above it, and the last K step of 64 may hold chunks past the padding (read as 0)
  const int64_t kp = ceil_div(K, 32) * 32;

  // each thread moves LA 16-byte chunks of A and LB of B per K step: 8 threads per
  // 128-byte row segment
  uint4 ra[LA], rb[LB];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int q = tid + NT * r;
      const int row = q >> 3, ch = q & 7;
      const int64_t gi = m0 + row, gk = k0 + 8 * ch;
      ra[r] = (gi < M && gk < kp) ? *reinterpret_cast<const uint4*>(A + gi * lda + gk) : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int q = tid + NT * r;
      const int row = q >> 3, ch = q & 7;
      const int64_t gj = n0 + row, gk = k0 + 8 * ch;
      rb[r] = (gj < N && gk < kp) ? *reinterpret_cast<const uint4*>(B + gj * ldb + gk) : make_uint4(0, 0, 0, 0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int q = tid + NT * r;
      *reinterpret_cast<uint4*>(&As[buf][q >> 3][8 * (q & 7)]) = ra[r];
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int q = tid + NT * r;
      *reinterpret_cast<uint4*>(&Bs[buf][q >> 3][8 * (q & 7)]) = rb[r];
    }
  };

  f4 acc[FA][FB];
#pragma unroll
  for (int a = 0; a < FA; ++a)
#pragma unroll
    for (int b = 0; b < FB; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

  if (nk > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  const int lrow = lane & 15, lk = lane >> 4;
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load(static_cast<int64_t>(kt + 1) * LBK);
#pragma unroll
    for (int kk = 0; kk < LBK / 32; ++kk) {
      V8 fa[FA], fb[FB];
#pragma unroll
      for (int a = 0; a < FA; ++a)
        fa[a] = *reinterpret_cast<const V8*>(&As[cur][wm * WTM + a * 16 + lrow][32 * kk + 8 * lk]);
#pragma unroll
      for (int b = 0; b < FB; ++b)
        fb[b] = *reinterpret_cast<const V8*>(&Bs[cur][wn * WTN + b * 16 + lrow][32 * kk + 8 * lk]);
#pragma unroll
      for (int a = 0; a < FA; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b) acc[a][b] = Lowp<BF16>::mma(fb[b], fa[a], acc[a][b]);
    }
    if (kt + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int a = 0; a < FA; ++a) {
    const int64_t gm = m0 + wm * WTM + a * 16 + lrow;
#pragma unroll
    for (int b = 0; b < FB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gn = n0 + wn * WTN + b * 16 + 4 * lk + r;
        if (gm < M && gn < N) {
          float* c = C + gm + gn * ldc;
          *c = (beta == 0.f) ? alpha * acc[a][b][r] : alpha * acc[a][b][r] + beta * *c;
        }
      }
  }
}

// dst (rows_pad x cols, ld ldd) = 16-bit RNE rounding of src (rows x cols), zero in rows >= rows.
// The power of two by which a cast scales its source: with amax (the bits of
// max |x| over the source, from absmax_kernel) set, 2^(14 - e) for max |x| in
// [2^(e-1), 2^e), so the largest magnitude lands in [2^13, 2^14) and FP16's
// range (65504) leaves room; 1 when amax is null, zero or not finite.
// Scaling by a power of two is exact, and Qpos(c X) = Qpos(X) for c > 0, so no
// scale is ever undone.
__device__ inline float cast_scale(const unsigned* amax) {
  if (amax == nullptr) return 1.f;
  const float mx = __uint_as_float(*amax);
  if (!(mx > 0.f) || !(mx <= 3.4e38f)) return 1.f;
  int e = 0;
  (void)frexpf(mx, &e);
  return ldexpf(1.f, 14 - e);
}

// dst (ldd x cols, 16-bit, RNE) = scale * src (rows x cols), zero in rows [rows, ldd).
template <bool BF16, class S>
__global__ void to_lowp_kernel(const S* __restrict__ src, int64_t lds, int64_t rows, int64_t cols,
                               void* __restrict__ dstv, int64_t ldd, const unsigned* __restrict__ amax) {
  using E = typename Lowp<BF16>::elem;
  E* dst = static_cast<E*>(dstv);
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= ldd * cols) return;
  const float sc = cast_scale(amax);
  const int64_t i = idx % ldd, j = idx / ldd;
  const float v = (i < rows) ? static_cast<float>(src[i + j * lds]) * sc : 0.f;
  dst[i + j * ldd] = static_cast<E>(v);
}

// dst = 16-bit rounding of scale * src^T: src rows x cols (ld lds), dst cols x rows (ld ldd, padded
// with zeros in rows >= cols), through 32 x 32 LDS tiles so both sides are coalesced.
template <bool BF16, class S>
__global__ __launch_bounds__(256) void to_lowp_transposed_kernel(const S* __restrict__ src,
                                                                  int64_t lds, int64_t rows,
                                                                  int64_t cols, void* __restrict__ dstv,
                                                                  int64_t ldd, const unsigned* __restrict__ amax) {
  using E = typename Lowp<BF16>::elem;
  E* dst = static_cast<E*>(dstv);
  __shared__ float tile[32][33];
  const float sc = cast_scale(amax);
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * 32;  // src row block
  const int64_t j0 = static_cast<int64_t>(blockIdx.y) * 32;  // src column block
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;    // 32 x 8
  for (int y = ty; y < 32; y += 8) {
    const int64_t i = i0 + tx, j = j0 + y;
    tile[y][tx] = (i < rows && j < cols) ? static_cast<float>(src[i + j * lds]) * sc : 0.f;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t di = j0 + tx, dj = i0 + y;  // dst(di, dj) = src(dj, di)
    if (di < ldd && dj < rows) dst[di + dj * ldd] = static_cast<E>(tile[tx][y]);
  }
}

// *amax = the bits of max |x| over src (rows x cols), as an FP32 value (NaN wins):
// non-negative floats order like their bits, so an integer maximum serves.
// *amax must be 0 before the launch (zero_u32_kernel).
template <class S>
__global__ __launch_bounds__(256) void absmax_kernel(const S* __restrict__ src, int64_t lds, int64_t rows,
                                                     int64_t cols, unsigned* __restrict__ amax) {
  __shared__ unsigned red[256];
  unsigned mx = 0;
  const int64_t total = rows * cols;
  for (int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t i = idx % rows, j = idx / rows;
    const unsigned b = __float_as_uint(fabsf(static_cast<float>(src[i + j * lds])));
    mx = b > mx ? b : mx;
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (static_cast<int>(threadIdx.x) < h && red[threadIdx.x + h] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(amax, red[0]);
}

__global__ void zero_u32_kernel(unsigned* p) { *p = 0u; }

template <class S, class D>
__global__ void convert_kernel(const S* __restrict__ src, int64_t lds, int64_t rows, int64_t cols,
                               D* __restrict__ dst, int64_t ldd) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t i = idx % rows, j = idx / rows;
  dst[i + j * ldd] = static_cast<D>(src[i + j * lds]);
}

}  // namespace

int64_t lowp_ld(int64_t rows) { return ceil_div(std::max<int64_t>(rows, 1), 32) * 32; }

int gemm_lowp(bool bf16, int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
              const void* B, int64_t ldb, float beta, float* C, int64_t ldc, hipStream_t s) {
  if (M == 0 || N == 0) return URV_OK;
  if (lda % 32 != 0 || ldb % 32 != 0 || lda < lowp_ld(K) || ldb < lowp_ld(K)) {
    set_last_error("gemm_lowp: 16-bit operands need padded leading dimensions");
    return URV_EINVAL;
  }
  // 256 x 256 tiles (8 waves of 128 x 64: a third fewer LDS bytes per MFMA than 64 x 64
  // wave tiles) when they still fill the 256 CUs, else 128 x 128 (URV_LOWP_TILE=128 or
  // 256 forces one, for tuning)
  int tb = ceil_div(M, 256) * ceil_div(N, 256) >= 256 ? 256 : 128;
  if (const char* te = std::getenv("URV_LOWP_TILE")) {
    if (std::atoi(te) == 128) tb = 128;
    if (std::atoi(te) == 256) tb = 256;
  }
  const int tiles_m = static_cast<int>(ceil_div(M, tb)), tiles_n = static_cast<int>(ceil_div(N, tb));
  const dim3 grid(tiles_m * tiles_n);
  if (tb == 256) {
    if (bf16)
      gemm_lowp_kernel<true, 256, 256, 2, 4><<<grid, 512, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                                                                  tiles_m, tiles_n);
    else
      gemm_lowp_kernel<false, 256, 256, 2, 4><<<grid, 512, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                                                                   tiles_m, tiles_n);
  } else if (bf16) {
    gemm_lowp_kernel<true, 128, 128, 2, 2><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                                                                tiles_m, tiles_n);
  } else {
    gemm_lowp_kernel<false, 128, 128, 2, 2><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                                                                 tiles_m, tiles_n);
  }
  URV_LAUNCHED("gemm_lowp_kernel");
  return URV_OK;
}

template <class S>
int to_lowp(bool bf16, const S* src, int64_t lds, int64_t rows, int64_t cols, void* dst, int64_t ldd,
            hipStream_t s, const unsigned* amax) {
  if (rows == 0 || cols == 0) return URV_OK;
  const unsigned blocks = static_cast<unsigned>(ceil_div(ldd * cols, 256));
  if (bf16)
    to_lowp_kernel<true, S><<<blocks, 256, 0, s>>>(src, lds, rows, cols, dst, ldd, amax);
  else
    to_lowp_kernel<false, S><<<blocks, 256, 0, s>>>(src, lds, rows, cols, dst, ldd, amax);
  URV_LAUNCHED("to_lowp_kernel");
  return URV_OK;
}
template int to_lowp<double>(bool, const double*, int64_t, int64_t, int64_t, void*, int64_t, hipStream_t,
                             const unsigned*);
template int to_lowp<float>(bool, const float*, int64_t, int64_t, int64_t, void*, int64_t, hipStream_t,
                            const unsigned*);

template <class S>
int to_lowp_transposed(bool bf16, const S* src, int64_t lds, int64_t rows, int64_t cols, void* dst, int64_t ldd,
                       hipStream_t s, const unsigned* amax) {
  if (rows == 0 || cols == 0) return URV_OK;
  // cover dst rows [0, ldd) (zero padding included) and dst columns [0, rows)
  const dim3 grid(static_cast<unsigned>(ceil_div(rows, 32)), static_cast<unsigned>(ceil_div(ldd, 32)));
  if (bf16)
    to_lowp_transposed_kernel<true, S><<<grid, 256, 0, s>>>(src, lds, rows, cols, dst, ldd, amax);
  else
    to_lowp_transposed_kernel<false, S><<<grid, 256, 0, s>>>(src, lds, rows, cols, dst, ldd, amax);
  URV_LAUNCHED("to_lowp_transposed_kernel");
  return URV_OK;
}
template int to_lowp_transposed<double>(bool, const double*, int64_t, int64_t, int64_t, void*, int64_t,
                                        hipStream_t, const unsigned*);
template int to_lowp_transposed<float>(bool, const float*, int64_t, int64_t, int64_t, void*, int64_t, hipStream_t,
                                       const unsigned*);

template <class S>
int absmax(const S* src, int64_t lds, int64_t rows, int64_t cols, unsigned* amax, hipStream_t s) {
  zero_u32_kernel<<<1, 1, 0, s>>>(amax);
  URV_LAUNCHED("zero_u32_kernel");
  if (rows == 0 || cols == 0) return URV_OK;
  const unsigned blocks = static_cast<unsigned>(std::min<int64_t>(ceil_div(rows * cols, 256), 1024));
  absmax_kernel<S><<<blocks, 256, 0, s>>>(src, lds, rows, cols, amax);
  URV_LAUNCHED("absmax_kernel");
  return URV_OK;
}
template int absmax<double>(const double*, int64_t, int64_t, int64_t, unsigned*, hipStream_t);
template int absmax<float>(const float*, int64_t, int64_t, int64_t, unsigned*, hipStream_t);

template <class S, class D>
int convert(const S* src, int64_t lds, int64_t rows, int64_t cols, D* dst, int64_t ldd, hipStream_t s) {
  if (rows == 0 || cols == 0) return URV_OK;
  convert_kernel<S, D><<<static_cast<unsigned>(ceil_div(rows * cols, 256)), 256, 0, s>>>(src, lds, rows, cols,
                                                                                        dst, ldd);
  URV_LAUNCHED("convert_kernel");
  return URV_OK;
}
template int convert<float, double>(const float*, int64_t, int64_t, int64_t, double*, int64_t, hipStream_t);
template int convert<double, float>(const double*, int64_t, int64_t, int64_t, float*, int64_t, hipStream_t);

}  // namespace urv
