// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11) and the Box-Muller map
// behind the Gaussian G of eq. (power), Section 3, as device functions (shared
// by the Gaussian fill kernel and the batched factorisation).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace urv {

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

// The four normal deviates of Philox block `block` of stream `stream_id` under
// key (seed, 0): elements 4 block .. 4 block + 3 in column-major linear order.
__device__ inline void gaussian_block(uint64_t block, uint32_t stream_id, uint64_t seed, double z[4]) {
  const U64x4 w = philox4x64_10(block, stream_id, 0, 0, seed, 0);
  const double two_pi = 6.28318530717958647692528676655900577;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const double radius = sqrt(-2.0 * log(unit_open(w.v[2 * p])));
    const double angle = two_pi * unit_open(w.v[2 * p + 1]);
    double sn, cs;
    sincos(angle, &sn, &cs);
    z[2 * p] = radius * cs;
    z[2 * p + 1] = radius * sn;
  }
}

}  // namespace urv
