// Device-side counter-based random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11) and float64 Box-Muller.
//
// One round multiplies counter words 0 and 2 by two odd 64-bit constants and rebuilds the
// counter from the high/low product halves, the other two words and the key; the key is
// advanced by two Weyl increments between rounds.  Counter layout used by the library:
//   (block, step_or_analysis_index, (tag << 32) | ensemble_id, particle), key = (seed, 0).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace iewpf {

struct U64x4 {
  uint64_t x0, x1, x2, x3;
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  const uint64_t kMulA = 0xD2E7470EE14C6C93ull;
  const uint64_t kMulB = 0xCA5A826395121157ull;
  const uint64_t kWeylA = 0x9E3779B97F4A7C15ull;
  const uint64_t kWeylB = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t hiA = __umul64hi(kMulA, c0);
    const uint64_t loA = kMulA * c0;
    const uint64_t hiB = __umul64hi(kMulB, c2);
    const uint64_t loB = kMulB * c2;
    const uint64_t n0 = hiB ^ c1 ^ k0;
    const uint64_t n2 = hiA ^ c3 ^ k1;
    c0 = n0;
    c1 = loB;
    c2 = n2;
    c3 = loA;
    k0 += kWeylA;
    k1 += kWeylB;
  }
  return U64x4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint64_t stream_word(uint32_t tag, uint32_t ens) {
  return (static_cast<uint64_t>(tag) << 32) | static_cast<uint64_t>(ens);
}

// Two 64-bit words -> two N(0,1) draws (float64): u1 in (0, 1], u2 in [0, 1).
__device__ __forceinline__ void box_muller(uint64_t a, uint64_t b, double& z0, double& z1) {
  const double u1 = (static_cast<double>(a >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = static_cast<double>(b >> 11) * 0x1.0p-53;
  const double r = sqrt(-2.0 * log(u1));
  double s, c;
  sincos(6.283185307179586 * u2, &s, &c);
  z0 = r * c;
  z1 = r * s;
}

// Four consecutive normals of block `blk` of a stream.
__device__ __forceinline__ void normals4(uint64_t blk, uint64_t step, uint32_t tag, uint32_t ens,
                                         uint64_t particle, uint64_t seed, double z[4]) {
  const U64x4 w = philox4x64_10(blk, step, stream_word(tag, ens), particle, seed, 0);
  box_muller(w.x0, w.x1, z[0], z[1]);
  box_muller(w.x2, w.x3, z[2], z[3]);
}

}  // namespace iewpf
