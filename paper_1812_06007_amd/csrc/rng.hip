// Gaussian starting matrix G of eq. (power), Section 3: a counter-based
// Philox4x64-10 stream (Salmon, Moraes, Dror & Shaw, SC'11) mapped to normal
// deviates by Box-Muller.  One thread produces one 4-word Philox block, i.e.
// four consecutive elements in column-major linear order.
#include "common.hpp"
#include "philox.hpp"

namespace urv {
namespace {

template <bool F32>
__global__ void gaussian_kernel(void* __restrict__ out, int64_t rows, int64_t total, int64_t ld,
                                uint64_t seed, uint32_t stream_id) {
  const int64_t block = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (4 * block >= total) return;
  double z[4];
  gaussian_block(static_cast<uint64_t>(block), stream_id, seed, z);
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
