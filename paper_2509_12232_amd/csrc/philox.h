// philox.h -- Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11), device side.
//
// Draw stream: for (individual, generation, ligand, purpose), draw n is half
// (n & 1: 0 low, 1 high) of 64-bit word ((n >> 1) & 3) of the block with counter
// (individual, generation, ligand, purpose << 32 | n >> 3) under key (seed, 0).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dock {

enum : uint64_t { kPurposeInit = 1, kPurposeSelect = 2, kPurposeCross = 3, kPurposeProposal = 4 };

__device__ __forceinline__ void philox4x64_10(uint64_t &x0, uint64_t &x1, uint64_t &x2, uint64_t &x3,
                                              uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, x0), lo0 = M0 * x0;
    const uint64_t hi1 = __umul64hi(M1, x2), lo1 = M1 * x2;
    const uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
    k0 += W0;
    k1 += W1;
  }
}

struct DrawStream {
  uint64_t seed, c0, c1, c2, purpose;
  uint64_t n;
  uint64_t blk;            // index of the cached block (~0 = none)
  uint64_t w0, w1, w2, w3;  // the cached block (named, so it stays in registers)

  __device__ DrawStream(uint64_t seed_, uint64_t indiv, uint64_t gen, uint64_t lig, uint64_t purpose_)
      : seed(seed_), c0(indiv), c1(gen), c2(lig), purpose(purpose_), n(0), blk(~0ull) {}

  __device__ __forceinline__ uint32_t u32() {
    const uint64_t b = n >> 3;
    if (b != blk) {
      w0 = c0; w1 = c1; w2 = c2; w3 = (purpose << 32) | b;
      philox4x64_10(w0, w1, w2, w3, seed, 0);
      blk = b;
    }
    const uint32_t k = (uint32_t)(n >> 1) & 3u;
    const uint64_t word = k == 0 ? w0 : k == 1 ? w1 : k == 2 ? w2 : w3;
    const uint32_t v = (n & 1) ? (uint32_t)(word >> 32) : (uint32_t)word;
    ++n;
    return v;
  }
  // uniform on the 2^-24 lattice in [0, 1), exact in float and double
  __device__ __forceinline__ double unit() { return (double)(u32() >> 8) * (1.0 / 16777216.0); }
  // uniform integer in [0, m)
  __device__ __forceinline__ int index(int m) { return (int)(((uint64_t)u32() * (uint64_t)m) >> 32); }
};

}  // namespace dock
