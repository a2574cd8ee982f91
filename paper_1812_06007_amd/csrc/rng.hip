// Gaussian starting matrix G of eq. (power), Section 3: a counter-based
// Philox4x64-10 stream (Salmon, Moraes, Dror & Shaw, SC'11) mapped to normal
// deviates by Box-Muller.  One thread produces one 4-word Philox block, i.e.
// four consecutive elements in column-major linear order.
#include "common.hpp"

namespace urv {
namespace {

struct U64x4 {
  uint64_t v[4];
};

__device__ inline U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                       uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
    const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return {{c0, c1, c2, c3}};
}

__device__ inline double unit_open(uint64_t w) {
  return (static_cast<double>(w >> 11) + 0.5) * 0x1p-53;
}

template <bool F32>
__global__ void gaussian_kernel(void* __restrict__ out, int64_t rows, int64_t total, int64_t ld,
                                uint64_t seed, uint32_t stream_id) {
  const int64_t block = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (4 * block >= total) return;
  const U64x4 w = philox4x64_10(static_cast<uint64_t>(block), stream_id, 0, 0, seed, 0);
  const double two_pi = 6.28318530717958647692528676655900577;
  double z[4];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const double radius = sqrt(-2.0 * log(unit_open(w.v[2 * p])));
    const double angle = two_pi * unit_open(w.v[2 * p + 1]);
    double sn, cs;
    sincos(angle, &sn, &cs);
    z[2 * p] = radius * cs;
    z[2 * p + 1] = radius * sn;
  }
#pragma unroll
  for (int lane = 0; lane < 4; ++lane) {
    const int64_t l = 4 * block + lane;
    if (l < total) {
      const int64_t i = l % rows, j = l / rows;
      if (F32)
        static_cast<float*>(out)[i + j * ld] = static_cast<float>(z[lane]);
      else
        static_cast<double*>(out)[i + j * ld] = z[lane];
    }
  }
}

}  // namespace

int launch_gaussian(void* G, int64_t rows, int64_t cols, int64_t ld, uint64_t seed,
                    uint32_t stream_id, bool out_f32, hipStream_t s) {
  const int64_t total = rows * cols;
  if (total == 0) return URV_OK;
  const int64_t blocks = ceil_div(total, 4);
  const int threads = 256;
  const dim3 grid(static_cast<unsigned>(ceil_div(blocks, threads)));
  if (out_f32)
    gaussian_kernel<true><<<grid, threads, 0, s>>>(G, rows, total, ld, seed, stream_id);
  else
    gaussian_kernel<false><<<grid, threads, 0, s>>>(G, rows, total, ld, seed, stream_id);
  URV_LAUNCHED("gaussian_kernel");
  return URV_OK;
}

}  // namespace urv
