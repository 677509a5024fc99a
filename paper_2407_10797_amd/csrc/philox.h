// philox.h -- Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11), written from its
// published definition: ten rounds of two 64x64->128-bit multiplies with the
// multipliers below, Weyl-sequence key bumps between rounds.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fstat {

constexpr uint64_t kPhM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhW1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox4x64_10(const uint64_t ctr_in[4], uint64_t k0, uint64_t k1,
                                              uint64_t out[4]) {
  uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kPhW0;
      k1 += kPhW1;
    }
    uint64_t lo0 = kPhM0 * c0, hi0 = __umul64hi(kPhM0, c0);
    uint64_t lo1 = kPhM1 * c2, hi1 = __umul64hi(kPhM1, c2);
    uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// 12 uniforms in [0, 1) for (run, t, particle)
__device__ __forceinline__ void draw12(uint64_t seed, uint64_t run, uint64_t t, uint64_t i,
                                       double u[12]) {
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    uint64_t ctr[4] = {t, i, (uint64_t)b, 0ull}, o[4];
    philox4x64_10(ctr, seed, run, o);
#pragma unroll
    for (int m = 0; m < 4; ++m) u[4 * b + m] = (double)(o[m] >> 11) * 0x1.0p-53;
  }
}

}  // namespace fstat
