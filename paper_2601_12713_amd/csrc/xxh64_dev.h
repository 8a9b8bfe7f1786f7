// XXH64 building blocks for gfx950, from the public xxHash specification:
// five 64-bit primes, four accumulators over 32-byte stripes, the 8/4/1-byte
// remainder steps and the final avalanche. The library runs the four
// accumulators of one input on four adjacent lanes of a wavefront.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace odp {

constexpr uint64_t kP1 = 0x9E3779B185EBCA87ull;
constexpr uint64_t kP2 = 0xC2B2AE3D27D4EB4Full;
constexpr uint64_t kP3 = 0x165667B19E3779F9ull;
constexpr uint64_t kP4 = 0x85EBCA77C2B2AE63ull;
constexpr uint64_t kP5 = 0x27D4EB2F165667C5ull;

__device__ __forceinline__ uint64_t rotl64(uint64_t x, int r) { return (x << r) | (x >> (64 - r)); }

// One stripe word folded into one accumulator.
__device__ __forceinline__ uint64_t xx_round(uint64_t acc, uint64_t w) {
  acc += w * kP2;
  acc = rotl64(acc, 31);
  return acc * kP1;
}

__device__ __forceinline__ uint64_t xx_merge(uint64_t h, uint64_t v) {
  h ^= xx_round(0, v);
  return h * kP1 + kP4;
}

// Initial value of accumulator `a` (0..3) for `seed`.
__device__ __forceinline__ uint64_t xx_acc_init(uint64_t seed, int a) {
  return a == 0 ? seed + kP1 + kP2 : a == 1 ? seed + kP2 : a == 2 ? seed : seed - kP1;
}

// Folds the four accumulators into the running hash (inputs of >= 32 bytes).
__device__ __forceinline__ uint64_t xx_converge(uint64_t v1, uint64_t v2, uint64_t v3, uint64_t v4) {
  uint64_t h = rotl64(v1, 1) + rotl64(v2, 7) + rotl64(v3, 12) + rotl64(v4, 18);
  h = xx_merge(h, v1);
  h = xx_merge(h, v2);
  h = xx_merge(h, v3);
  return xx_merge(h, v4);
}

__device__ __forceinline__ uint64_t xx_step8(uint64_t h, uint64_t w) {
  h ^= xx_round(0, w);
  return rotl64(h, 27) * kP1 + kP4;
}
__device__ __forceinline__ uint64_t xx_step4(uint64_t h, uint32_t w) {
  h ^= uint64_t(w) * kP1;
  return rotl64(h, 23) * kP2 + kP3;
}
__device__ __forceinline__ uint64_t xx_step1(uint64_t h, uint8_t b) {
  h ^= uint64_t(b) * kP5;
  return rotl64(h, 11) * kP1;
}

__device__ __forceinline__ uint64_t xx_avalanche(uint64_t h) {
  h ^= h >> 33;
  h *= kP2;
  h ^= h >> 29;
  h *= kP3;
  h ^= h >> 32;
  return h;
}

// Little-endian 8 bytes at any address. Both aligned words read contain bytes
// of [p, p+8), so nothing outside the 8-byte granules of the range is touched.
__device__ __forceinline__ uint64_t load64_any(const uint8_t* p) {
  uintptr_t a = reinterpret_cast<uintptr_t>(p);
  const uint64_t* q = reinterpret_cast<const uint64_t*>(a & ~uintptr_t(7));
  uint32_t sh = uint32_t(a & 7) * 8;
  uint64_t lo = q[0];
  if (sh == 0) return lo;
  uint64_t hi = q[1];
  return (lo >> sh) | (hi << (64 - sh));
}

// The remainder steps over rem (< 32) bytes at p (any alignment, byte reads).
__device__ __forceinline__ uint64_t xx_tail_bytes(uint64_t h, const uint8_t* p, uint32_t rem) {
  while (rem >= 8) {
    uint64_t w = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) w |= uint64_t(p[i]) << (8 * i);
    h = xx_step8(h, w);
    p += 8;
    rem -= 8;
  }
  if (rem >= 4) {
    uint32_t w = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) w |= uint32_t(p[i]) << (8 * i);
    h = xx_step4(h, w);
    p += 4;
    rem -= 4;
  }
  while (rem > 0) {
    h = xx_step1(h, *p);
    ++p;
    --rem;
  }
  return h;
}

// Lane k of each group of four lanes, broadcast to the group (DPP quad_perm,
// a VALU move: no LDS round trip on the accumulator chain). Every lane of the
// group must be active.
template <int K>
__device__ __forceinline__ uint64_t xx_quad_bcast(uint64_t x) {
  constexpr int ctrl = K * 0x55;  // quad_perm:[K,K,K,K]
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, ctrl, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), ctrl, 0xF, 0xF, false);
  return ((uint64_t)hi << 32) | lo;
}

// Gathers the accumulator of lanes 4g..4g+3 into all four lanes.
__device__ __forceinline__ void xx_gather4(uint64_t acc, uint64_t& v1, uint64_t& v2, uint64_t& v3, uint64_t& v4) {
  v1 = xx_quad_bcast<0>(acc);
  v2 = xx_quad_bcast<1>(acc);
  v3 = xx_quad_bcast<2>(acc);
  v4 = xx_quad_bcast<3>(acc);
}

// XXH64 of `nw` little-endian u64 words (a tree node's children), computed by
// the four lanes 4g..4g+3 together; every one of them returns the digest.
// `w` may point to LDS or global memory.
__device__ __forceinline__ uint64_t xx_words4(const uint64_t* w, uint32_t nw, uint64_t seed) {
  const int a = threadIdx.x & 3;
  uint32_t nstripes = nw / 4;
  uint64_t acc = xx_acc_init(seed, a);
  for (uint32_t s = 0; s < nstripes; ++s) acc = xx_round(acc, w[s * 4 + a]);
  uint64_t v1, v2, v3, v4;
  xx_gather4(acc, v1, v2, v3, v4);
  uint64_t h = nstripes ? xx_converge(v1, v2, v3, v4) : seed + kP5;
  h += uint64_t(nw) * 8;
  for (uint32_t i = nstripes * 4; i < nw; ++i) h = xx_step8(h, w[i]);
  return xx_avalanche(h);
}

// XXH64 of exactly 64 words (a full tree node) by lanes 4g..4g+3; every lane
// returns the digest. One four-lane chain is bound by latency, not issue, so
// every stripe word and its product with P2 are formed before the chain
// starts, and only the add, the rotation and the multiply by P1 wait on the
// previous round. Same result as xx_words4(w, 64, seed).
__device__ __forceinline__ uint64_t xx_words4_full64(const uint64_t* w, uint64_t seed) {
  const int a = threadIdx.x & 3;
  uint64_t t[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) t[s] = w[s * 4 + a];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    t[s] *= kP2;
    asm volatile("" : "+v"(t[s]));  // keeps the product out of the accumulator's multiply-add
  }
  uint64_t acc = xx_acc_init(seed, a);
#pragma unroll
  for (int s = 0; s < 16; ++s) acc = rotl64(acc + t[s], 31) * kP1;
  uint64_t v1, v2, v3, v4;
  xx_gather4(acc, v1, v2, v3, v4);
  return xx_avalanche(xx_converge(v1, v2, v3, v4) + 64 * 8);
}

}  // namespace odp
