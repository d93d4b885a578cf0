// cp_philox.hpp -- Philox4x32-10 (Salmon et al., "Parallel random numbers:
// as easy as 1, 2, 3", SC'11): a counter-based generator, so every sample's
// random words are a pure function of (counter, key) and results do not
// depend on the launch configuration.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cp {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

// Ten rounds on the counter c in place, key (k0, k1).  Each round's two
// 32 x 32 -> 64-bit products are formed whole (one v_mad_u64_u32 each rather
// than a high and a low multiply: a third faster on gfx950).
__device__ __forceinline__ void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c[0], p1 = (uint64_t)kPhiloxM1 * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = (uint32_t)p1;
    c[2] = n2;
    c[3] = (uint32_t)p0;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
}

// Uniform in (0, 1] from the top 24 bits of a word: ((r >> 8) + 1/2) 2^-24,
// exact in FP64; in FP32 the values above 1/2 need a 25th bit and round to
// the nearest even multiple of 2^-24 (by at most 2^-25; the top one to 1).
template <typename T>
__device__ __forceinline__ T u24_of(uint32_t r) {
  return (T(r >> 8) + T(0.5)) * T(5.9604644775390625e-8);
}

}  // namespace cp
