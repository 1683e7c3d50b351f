// plas_random.h -- counter-based random draws of the PLAS library, usable in
// host and device code.
//
// The paper asks for random positions at the start, a random block shift and
// a random permutation of each block's elements for the grouping (Sec. 3.1).
// Every draw here is a pure function of (seed, purpose, index), so a kernel
// can produce any element of any permutation without state or storage:
//  - Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter
//    (purpose, index, 0, 0), key (seed, 0);
//  - a keyed bijection of [0, n): a balanced 4-round Feistel network on
//    2h bits, h = max(1, ceil(ceil(log2 n) / 2)), round function
//    fmix64(R ^ K) mod 2^h (MurmurHash3's finaliser), round keys = the four
//    Philox words, and cycle walking (Black and Rogaway, 2002) into [0, n).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace plas {

enum DrawPurpose : uint64_t { kDrawStart = 0, kDrawGrouping = 1, kDrawShift = 2 };

struct Words4 {
  uint64_t v[4];
};

// 64 x 64 -> 128-bit product from 32-bit halves.
__host__ __device__ inline void wide_mul(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  const uint64_t a_lo = a & 0xffffffffu, a_hi = a >> 32;
  const uint64_t b_lo = b & 0xffffffffu, b_hi = b >> 32;
  const uint64_t ll = a_lo * b_lo;
  const uint64_t lh = a_lo * b_hi;
  const uint64_t hl = a_hi * b_lo;
  const uint64_t hh = a_hi * b_hi;
  const uint64_t mid = (ll >> 32) + (lh & 0xffffffffu) + (hl & 0xffffffffu);
  *lo = (mid << 32) | (ll & 0xffffffffu);
  *hi = hh + (lh >> 32) + (hl >> 32) + (mid >> 32);
}

__host__ __device__ inline Words4 philox4x64_10(Words4 x, uint64_t key0, uint64_t key1) {
  constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ull;
  constexpr uint64_t kMulB = 0xCA5A826395121157ull;
  constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ull;
  constexpr uint64_t kWeylB = 0xBB67AE8584CAA73Bull;
  for (int round = 0; round < 10; ++round) {
    uint64_t hiA, loA, hiB, loB;
    wide_mul(kMulA, x.v[0], &hiA, &loA);
    wide_mul(kMulB, x.v[2], &hiB, &loB);
    Words4 y;
    y.v[0] = hiB ^ x.v[1] ^ key0;
    y.v[1] = loB;
    y.v[2] = hiA ^ x.v[3] ^ key1;
    y.v[3] = loA;
    x = y;
    key0 += kWeylA;
    key1 += kWeylB;
  }
  return x;
}

__host__ __device__ inline Words4 draw(uint64_t seed, uint64_t purpose, uint64_t index) {
  Words4 ctr;
  ctr.v[0] = purpose;
  ctr.v[1] = index;
  ctr.v[2] = 0;
  ctr.v[3] = 0;
  return philox4x64_10(ctr, seed, 0);
}

__host__ __device__ inline uint64_t murmur_fmix64(uint64_t k) {
  k = (k ^ (k >> 33)) * 0xff51afd7ed558ccdull;
  k = (k ^ (k >> 33)) * 0xc4ceb53fe1a85ec3ull;
  return k ^ (k >> 33);
}

// Half width h of the Feistel domain for [0, n): 2h >= ceil(log2 n).
__host__ __device__ inline int feistel_half_bits(uint64_t n) {
  const int bits = n <= 1 ? 0 : 64 - __builtin_clzll(n - 1);
  const int h = (bits + 1) >> 1;
  return h > 0 ? h : 1;
}

struct Bijection {
  uint64_t n;
  uint64_t mask;
  int h;
  uint64_t key[4];

  __host__ __device__ Bijection(uint64_t n_, const uint64_t k[4]) : n(n_) {
    h = feistel_half_bits(n_);
    mask = (uint64_t(1) << h) - 1;
    key[0] = k[0];
    key[1] = k[1];
    key[2] = k[2];
    key[3] = k[3];
  }

  __host__ __device__ uint64_t round4(uint64_t x) const {
    uint64_t l = x >> h, r = x & mask;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint64_t t = l ^ (murmur_fmix64(r ^ key[i]) & mask);
      l = r;
      r = t;
    }
    return (l << h) | r;
  }

  // Image of i < n. Cycle walking ends because i's cycle under round4
  // contains i itself, which lies in [0, n).
  __host__ __device__ uint64_t operator()(uint64_t i) const {
    uint64_t y = round4(i);
    while (y >= n) y = round4(y);
    return y;
  }
};

// Block shift of draw j on a grid of side w: the top 32 bits of the first
// two words scaled to [0, w).
__host__ __device__ inline void block_shift(uint64_t seed, uint64_t j, int32_t w, int32_t* dy,
                                            int32_t* dx) {
  const Words4 u = draw(seed, kDrawShift, j);
  *dy = static_cast<int32_t>(((u.v[0] >> 32) * static_cast<uint64_t>(w)) >> 32);
  *dx = static_cast<int32_t>(((u.v[1] >> 32) * static_cast<uint64_t>(w)) >> 32);
}

}  // namespace plas
