// Counter-based random numbers of one Monte Carlo update.
//
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64->128-bit multiplies with a Weyl-sequence key schedule.  Counter words
// are (sweep, site, stream, attempt), key (seed, 0), so a draw depends only on
// which update it belongs to, never on how updates are batched on the GPU.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tca {

enum : uint64_t {
  kStreamProposal = 0,
  kStreamMetropolis = 1,
  kStreamSize = 2,
  kStreamInit = 3,
};
constexpr uint64_t kInitSweep = ~0ull;
constexpr int kMaxSphereAttempts = 64;

struct U64x4 {
  uint64_t w0, w1, w2, w3;
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t k0, uint64_t k1, uint64_t c0,
                                               uint64_t c1, uint64_t c2, uint64_t c3) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  return {c0, c1, c2, c3};
}

// Uniform double in [0,1) and [-1,1) from the top 53 bits (exact conversions).
__device__ __forceinline__ double u53(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }
__device__ __forceinline__ double v52(uint64_t r) { return (double)(r >> 11) * 0x1.0p-52 - 1.0; }

// Marsaglia (1972) point on the unit sphere from (v1, v2) in the unit disc.
// Every operation is a separately rounded IEEE-754 +, * or sqrt so the result
// is reproducible bit for bit by any conforming implementation.
__device__ __attribute__((noinline)) bool marsaglia(double v1, double v2, double* out) {
#pragma clang fp contract(off)
  double s = v1 * v1;
  s = s + v2 * v2;
  if (s >= 1.0 || s == 0.0) return false;
  const double q = __builtin_sqrt(1.0 - s);
  out[0] = (2.0 * v1) * q;
  out[1] = (2.0 * v2) * q;
  out[2] = 1.0 - 2.0 * s;
  return true;
}

// Uniform point on S^2 for counter (sweep, site, stream, attempt = 0, 1, ...);
// each Philox block offers the pairs (w0, w1) then (w2, w3).
__device__ inline void sphere_point(uint64_t seed, uint64_t sweep, uint64_t site,
                                    uint64_t stream, double* out) {
  for (int a = 0; a < kMaxSphereAttempts; ++a) {
    const U64x4 r = philox4x64_10(seed, 0, sweep, site, stream, (uint64_t)a);
    if (marsaglia(v52(r.w0), v52(r.w1), out)) return;
    if (marsaglia(v52(r.w2), v52(r.w3), out)) return;
  }
  out[0] = 0.0;  // unreachable in practice (probability ~1e-85)
  out[1] = 0.0;
  out[2] = 1.0;
}

// Index in [0, n) of the cluster size class of one update.
__device__ __forceinline__ int size_class(uint64_t seed, uint64_t sweep, uint64_t site, int n) {
  const U64x4 r = philox4x64_10(seed, 0, sweep, site, kStreamSize, 0);
  return (int)(((r.w0 >> 32) * (uint64_t)n) >> 32);
}

}  // namespace tca
