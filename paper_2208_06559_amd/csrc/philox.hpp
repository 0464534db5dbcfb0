// Counter-based Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11) and the uniform / Gaussian maps used
// for the Brownian noise of Eq. 6.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bd {

struct U64x4 {
  uint64_t v[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ULL, kM1 = 0xCA5A826395121157ULL;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ULL, kW1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(kM0, c0), lo0 = kM0 * c0;
    const uint64_t hi1 = __umul64hi(kM1, c2), lo1 = kM1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += kW0;
    k1 += kW1;
  }
  U64x4 o;
  o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

// 53 random bits to (0,1): ((w >> 11) + 1/2) * 2^-53.
__device__ __forceinline__ double u01_open(uint64_t w) {
  return ((double)(w >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

// Four noise values of Philox block `blk` for (seed, chain, step):
// Gaussian by Box-Muller on lane pairs (0,1), (2,3), or 2u - 1 (uniform).
__device__ __forceinline__ void noise4(uint64_t seed, uint64_t chain, uint64_t step, uint64_t blk,
                                       int uniform, double z[4]) {
  const U64x4 w = philox4x64_10(blk, step, 0ull, 0ull, seed, chain);
  double u[4];
#pragma unroll
  for (int l = 0; l < 4; ++l) u[l] = u01_open(w.v[l]);
  if (uniform) {
#pragma unroll
    for (int l = 0; l < 4; ++l) z[l] = 2.0 * u[l] - 1.0;
  } else {
    constexpr double kTwoPi = 6.283185307179586476925286766559;
#pragma unroll
    for (int pr = 0; pr < 2; ++pr) {
      const double rad = sqrt(-2.0 * log(u[2 * pr]));
      double sn, cs;
      sincos(kTwoPi * u[2 * pr + 1], &sn, &cs);
      z[2 * pr] = rad * cs;
      z[2 * pr + 1] = rad * sn;
    }
  }
}

}  // namespace bd
