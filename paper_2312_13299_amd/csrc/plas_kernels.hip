// plas_kernels.hip -- gfx950 kernels of one PLAS sort (Sec. 3.1 of arXiv
// 2312.13299): ingest, range, start arrangement, gather, separable box blur,
// grouping table, blockwise assignment with its energy, and the controller.
//
// Working layout: a grid is [n][DP], cell-major, DP a power of two (4..64)
// with zero padding beyond the d real channels, stored as float32 or as
// bfloat16 (S = float or S = uint16_t holding bfloat16 bits). A cell of
// DP = 64 is 256 bytes in float32 (two 128-byte lines) or 128 bytes in
// bfloat16 (one line), so the assignment kernel's random cell reads waste
// nothing, and a blur line is read as whole cells. All arithmetic is float32:
// bfloat16 values widen exactly, and results are rounded to bfloat16 (nearest,
// ties to even) only when they are stored.
//
// Floating point: compiled without contraction (-ffp-contract=off) and with
// denormals kept, so every float operation below is one IEEE-rounded add,
// subtract or multiply in the order written. That is what makes the results
// equal, bit for bit, to a CPU that evaluates the same expressions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <mutex>

#include "plas_launch.h"
#include "plas_random.h"

namespace plas {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kRangeBlocks = 256;
// Blocks of an assignment launch (its waves stride over the items). 4096 is
// the measured best over grid sides and storages together: 8192 gains 2 %
// on a 1024^2 float32 assignment and loses more on 512^2..724^2 grids and
// on bfloat16.
#ifndef PLAS_ASSIGN_MAX_BLOCKS
#define PLAS_ASSIGN_MAX_BLOCKS 4096
#endif
// Waves per block of the staged blur (each wave walks one group of 64/dp
// lines): two-wave blocks of 48 KB LDS let three blocks share a CU.
constexpr int kBlurWavesPerBlock = 2;
constexpr int kMaxGridBlocks = 4096;

inline int blocks_for(int64_t threads, int64_t cap = kMaxGridBlocks) {
  int64_t b = (threads + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return static_cast<int>(b);
}

// ---------------------------------------------------------------- storage

// bfloat16 is the high half of a float32: widening is exact.
__device__ __forceinline__ float bf16_to_float(uint32_t bits) { return __uint_as_float(bits << 16); }

// Nearest bfloat16, ties to even: gfx950 converts in one instruction
// (v_cvt_pk_bf16_f32). Every finite value and both infinities round as the
// integer form (add 0x7fff plus the kept part's lowest bit, keep the high
// half) does; a NaN stays a NaN with its sign, so the quiet NaNs that
// arithmetic produces keep their high half too.
__device__ __forceinline__ uint32_t float_to_bf16(float f) {
  return __builtin_bit_cast(unsigned short, static_cast<__bf16>(f));
}

template <typename S>
struct Storage;

template <>
struct Storage<float> {
  using Quad = float4;  // four channels
  __device__ static __forceinline__ float widen(float v) { return v; }
  __device__ static __forceinline__ float narrow(float v) { return v; }
  __device__ static __forceinline__ float4 widen4(float4 q) { return q; }
};

template <>
struct Storage<uint16_t> {
  using Quad = uint2;  // four channels
  __device__ static __forceinline__ float widen(uint16_t v) { return bf16_to_float(v); }
  __device__ static __forceinline__ uint16_t narrow(float v) { return static_cast<uint16_t>(float_to_bf16(v)); }
  __device__ static __forceinline__ float4 widen4(uint2 q) {
    return make_float4(bf16_to_float(q.x & 0xffffu), bf16_to_float(q.x >> 16), bf16_to_float(q.y & 0xffffu),
                       bf16_to_float(q.y >> 16));
  }
};

// ----------------------------------------------------------------- ingest

// Channel-major [d][n] -> [n][DP]: a 64-cell tile goes through LDS so that
// both the reads (64 consecutive cells of one channel) and the writes
// (64 consecutive cells of DP channels) are contiguous.
template <int DP, typename SI, typename SO>
__global__ __launch_bounds__(kBlock) void k_ingest_cn(const SI* __restrict__ F, int64_t n, int d,
                                                      SO* __restrict__ X) {
  __shared__ float tile[DP][65];
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * 64;
  for (int e = threadIdx.x; e < DP * 64; e += kBlock) {
    const int c = e >> 6, i = e & 63;
    const int64_t cell = n0 + i;
    tile[c][i] = (c < d && cell < n) ? Storage<SI>::widen(F[static_cast<int64_t>(c) * n + cell]) : 0.0f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < DP * 64; e += kBlock) {
    const int i = e / DP, c = e % DP;
    const int64_t cell = n0 + i;
    if (cell < n) X[cell * DP + c] = Storage<SO>::narrow(tile[c][i]);
  }
}

template <int DP, typename SI, typename SO>
__global__ __launch_bounds__(kBlock) void k_ingest_nc(const SI* __restrict__ F, int64_t n, int d,
                                                      SO* __restrict__ X) {
  const int64_t total = n * DP;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; e < total; e += stride) {
    const int64_t cell = e / DP;
    const int c = static_cast<int>(e % DP);
    X[e] = Storage<SO>::narrow(c < d ? Storage<SI>::widen(F[cell * d + c]) : 0.0f);
  }
}

// ------------------------------------------------------------------ range

// Each thread owns one channel (the grid stride is a multiple of DP), so a
// block reduces to DP partial min/max values in LDS.
template <int DP, typename S>
__global__ __launch_bounds__(kBlock) void k_range_partial(const S* __restrict__ X, int64_t n,
                                                          float* __restrict__ part) {
  __shared__ float s_lo[kBlock], s_hi[kBlock], s_bad[kBlock];
  const int t = threadIdx.x;
  float lo = INFINITY, hi = -INFINITY, bad = 0.0f;
  const int64_t total = n * DP;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + t; e < total; e += stride) {
    const float v = Storage<S>::widen(X[e]);
    if (!__builtin_isfinite(v)) bad = 1.0f;
    lo = fminf(lo, v);
    hi = fmaxf(hi, v);
  }
  s_lo[t] = lo;
  s_hi[t] = hi;
  s_bad[t] = bad;
  __syncthreads();
  for (int s = kBlock / 2; s >= DP; s >>= 1) {
    if (t < s) {
      s_lo[t] = fminf(s_lo[t], s_lo[t + s]);
      s_hi[t] = fmaxf(s_hi[t], s_hi[t + s]);
      s_bad[t] = fmaxf(s_bad[t], s_bad[t + s]);
    }
    __syncthreads();
  }
  if (t < DP) {
    float* out = part + static_cast<int64_t>(blockIdx.x) * 3 * DP;
    out[t] = s_lo[t];
    out[DP + t] = s_hi[t];
    out[2 * DP + t] = s_bad[t];
  }
}

template <int DP>
__global__ void k_range_finish(const float* __restrict__ part, int nparts, int d,
                               float* __restrict__ out) {
  // Launched with one wave of 64 threads; lanes c >= DP only join the barrier.
  __shared__ float s_bad[64];
  const int c = threadIdx.x;
  float bad = 0.0f;
  if (c < DP) {
    float lo = INFINITY, hi = -INFINITY;
    for (int b = 0; b < nparts; ++b) {
      const float* p = part + static_cast<int64_t>(b) * 3 * DP;
      lo = fminf(lo, p[c]);
      hi = fmaxf(hi, p[DP + c]);
      bad = fmaxf(bad, p[2 * DP + c]);
    }
    out[c] = lo;
    out[DP + c] = hi;
  }
  // One flag for all real channels, reduced by lane 0 from the others.
  s_bad[c] = c < d ? bad : 0.0f;
  __syncthreads();
  if (c == 0) {
    float any = 0.0f;
    for (int i = 0; i < DP; ++i) any = fmaxf(any, s_bad[i]);
    out[2 * DP] = any;
  }
}

// ------------------------------------------------- start arrangement, gather

__global__ __launch_bounds__(kBlock) void k_start_perm(int32_t* __restrict__ P, int64_t n, Words4 keys) {
  const Bijection f(static_cast<uint64_t>(n), keys.v);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n; p += stride)
    P[p] = static_cast<int32_t>(f(static_cast<uint64_t>(p)));
}

__global__ __launch_bounds__(kBlock) void k_count_perm(const int32_t* __restrict__ init, int64_t n,
                                                       int32_t* __restrict__ counts,
                                                       int32_t* __restrict__ flag) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n; p += stride) {
    const int32_t v = init[p];
    if (v < 0 || v >= n)
      atomicOr(flag, 1);
    else
      atomicAdd(&counts[v], 1);
  }
}

__global__ __launch_bounds__(kBlock) void k_verify_counts(const int32_t* __restrict__ counts, int64_t n,
                                                          int32_t* __restrict__ flag) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n; p += stride)
    if (counts[p] != 1) atomicOr(flag, 1);
}

// G[p] = X[P[p]] (P NULL: identity), four channels per thread.
template <int DP, typename S>
__global__ __launch_bounds__(kBlock) void k_gather(const S* __restrict__ X, const int32_t* __restrict__ P,
                                                   S* __restrict__ G, int64_t n) {
  constexpr int LG = DP / 4;
  using Quad = typename Storage<S>::Quad;
  const Quad* __restrict__ src = reinterpret_cast<const Quad*>(X);
  Quad* __restrict__ dst = reinterpret_cast<Quad*>(G);
  const int64_t total = n * LG;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; e < total; e += stride) {
    const int64_t p = e / LG;
    const int j = static_cast<int>(e % LG);
    const int64_t from = P != nullptr ? static_cast<int64_t>(P[p]) : p;
    dst[e] = src[from * LG + j];
  }
}

// ------------------------------------------------------------------- blur

// The radius of a pass: st->r, or the fixed radius when st is NULL. Returns
// false when the sort has ended (every kernel queued after the end returns
// at once).
__device__ __forceinline__ bool pass_radius(const DevState* __restrict__ st, int radius, int& r) {
  if (st != nullptr && st->done) return false;
  r = st != nullptr ? st->r : radius;
  return true;
}

// table[t] = pi(t) packed as (ly << 16) | lx, pi the grouping bijection of
// a reorder over the beta^2 block-local cells, filled by all blocks of a
// launch (NT threads each). The first row pass of a reorder runs it after
// its lines, from the state's beta and keys.
template <int NT>
__device__ __forceinline__ void fill_group_table(int32_t* __restrict__ table, int beta, const uint64_t keys[4],
                                                 int64_t bid, int64_t nblocks) {
  const uint64_t cells = static_cast<uint64_t>(beta) * beta;
  const Bijection f(cells, keys);
  const uint64_t stride = static_cast<uint64_t>(nblocks) * NT;
  for (uint64_t t = static_cast<uint64_t>(bid) * NT + threadIdx.x; t < cells; t += stride) {
    const uint32_t v = static_cast<uint32_t>(f(t));
    const uint32_t ly = v / static_cast<uint32_t>(beta);
    const uint32_t lx = v - ly * static_cast<uint32_t>(beta);
    table[t] = static_cast<int32_t>((ly << 16) | lx);
  }
}

// Orders this wave's LDS writes before its later LDS reads (lanes of one
// wave exchange data through LDS without a block barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


// One separable box-blur pass. Lane = (line, channel): DP consecutive lanes
// walk one line, 64 / DP lines per wave. Along the line the window sum is
// kept as a running sum: it starts as the ascending sum of the first
// min(r, w-1) + 1 values; at each next position the entering value is added
// and then the leaving value subtracted, and the output is the running sum
// times float32(1 / count) for the window clipped to the grid.
//
// The running sum is a serial chain per (line, channel), so a wave cannot
// hide memory latency by switching lines. Instead each lane keeps the loads
// of the next kBlurUnroll positions in flight while it adds up the current
// ones (two register buffers used in turn). The line is cut into ranges where
// "a value enters" and "a value leaves" are fixed, which keeps the unrolled
// loops free of per-position tests; the position x is the same for all lanes
// of a wave, so every remaining branch is uniform.
#ifndef PLAS_BLUR_UNROLL
#define PLAS_BLUR_UNROLL 12
#endif
constexpr int kBlurUnroll = PLAS_BLUR_UNROLL;

template <typename S>
struct BlurLine {
  const S* __restrict__ src;
  S* __restrict__ dst;
  int64_t step;
  const float* __restrict__ inv;
  int w;
  int r;

  __device__ __forceinline__ float load(int t) const {
    return Storage<S>::widen(src[static_cast<int64_t>(t) * step]);
  }
  // float32(1/count) of output position x (window clipped to the line).
  __device__ __forceinline__ float mult(int x) const {
    const int hi = x + r < w - 1 ? x + r : w - 1;
    const int lo = x - r > 0 ? x - r : 0;
    return inv[hi - lo + 1];
  }
  __device__ __forceinline__ void store(int x, float s, float m) const {
    dst[static_cast<int64_t>(x) * step] = Storage<S>::narrow(s * m);
  }
  __device__ static __forceinline__ float widen(S v) { return Storage<S>::widen(v); }
  __device__ static __forceinline__ S narrow(float v) { return Storage<S>::narrow(v); }
};

// kBlurUnroll positions' entering values, leaving values and multipliers.
struct BlurBlock {
  float enter[kBlurUnroll];
  float leave[kBlurUnroll];
  float mult[kBlurUnroll];
};

// Addresses advance by one step per position (a 64-bit add) instead of
// being recomputed from the position (a 64-bit multiply each).
template <bool ENTER, bool LEAVE, typename L_t>
__device__ __forceinline__ void blur_fetch(const L_t& L, int x0, BlurBlock& B) {
  const auto* pe = L.src;
  const auto* pl = L.src;
  if (ENTER) pe += static_cast<int64_t>(x0 + L.r) * L.step;
  if (LEAVE) pl += static_cast<int64_t>(x0 - L.r - 1) * L.step;
#pragma unroll
  for (int i = 0; i < kBlurUnroll; ++i) {
    if (ENTER) {
      B.enter[i] = L.widen(*pe);
      pe += L.step;
    }
    if (LEAVE) {
      B.leave[i] = L.widen(*pl);
      pl += L.step;
    }
    B.mult[i] = L.mult(x0 + i);
  }
}

template <bool ENTER, bool LEAVE, typename L_t>
__device__ __forceinline__ void blur_apply(const L_t& L, int x0, const BlurBlock& B, float& s) {
  auto* pd = L.dst + static_cast<int64_t>(x0) * L.step;
#pragma unroll
  for (int i = 0; i < kBlurUnroll; ++i) {
    if (ENTER) s = s + B.enter[i];
    if (LEAVE) s = s - B.leave[i];
    *pd = L.narrow(s * B.mult[i]);
    pd += L.step;
  }
}

// Wait until every vector memory operation of this wave has completed
// (s_waitcnt vmcnt(0); expcnt and lgkmcnt left at their maxima).
__device__ __forceinline__ void wait_vmem() {
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __builtin_amdgcn_sched_barrier(0);
}


// Positions [xb, xe) where entering/leaving values exist as ENTER/LEAVE say.
// Loads and stores share one memory counter, so with the previous block's
// stores in flight the compiler can only wait for all outstanding memory
// operations before a block's values are used; left to itself it would do
// so after the next block's loads were issued and wait for those too. The
// explicit wait comes first, the next block's fetch is issued after it and
// flies while the current block is summed and stored.
template <bool ENTER, bool LEAVE, typename L_t>
__device__ __forceinline__ void blur_range(const L_t& L, int xb, int xe, float& s) {
  const int full = (xe - xb) / kBlurUnroll;
  int x = xb;
  if (full > 0) {
    BlurBlock next, cur;
    blur_fetch<ENTER, LEAVE>(L, x, next);
    for (int c = 0; c < full; ++c) {
      wait_vmem();
      cur = next;
      if (c + 1 < full) blur_fetch<ENTER, LEAVE>(L, x + kBlurUnroll, next);
      blur_apply<ENTER, LEAVE>(L, x, cur, s);
      x += kBlurUnroll;
    }
  }
  for (; x < xe; ++x) {
    if (ENTER) s = s + L.load(x + L.r);
    if (LEAVE) s = s - L.load(x - L.r - 1);
    L.store(x, s, L.mult(x));
  }
}

// Lines wave * 64/DP .. of one pass, by wave `wave` of the pass.
template <int DP, typename S>
__device__ __forceinline__ void blur_reg_lines(const S* __restrict__ in, S* __restrict__ out, int w, int r,
                                               int vertical, const float* __restrict__ inv, int64_t wave,
                                               int lane) {
  constexpr int LPW = 64 / DP;
  const int64_t line = wave * LPW + lane / DP;
  const int c = lane % DP;
  if (line >= w) return;
  const int64_t base = vertical ? line * DP + c : line * w * DP + c;
  BlurLine<S> L;
  L.src = in + base;
  L.dst = out + base;
  L.step = vertical ? static_cast<int64_t>(w) * DP : DP;
  L.inv = inv;
  L.w = w;
  L.r = r;
  if (r == 0) {
    for (int x = 0; x < w; ++x) L.dst[x * L.step] = L.src[x * L.step];
    return;
  }
  // Start: ascending sum of positions 0 .. first_hi, loaded kBlurUnroll at a time.
  const int first_hi = r < w - 1 ? r : w - 1;
  float s = L.load(0);
  int t = 1;
  for (; t + kBlurUnroll - 1 <= first_hi; t += kBlurUnroll) {
    float v[kBlurUnroll];
#pragma unroll
    for (int i = 0; i < kBlurUnroll; ++i) v[i] = L.load(t + i);
#pragma unroll
    for (int i = 0; i < kBlurUnroll; ++i) s = s + v[i];
  }
  for (; t <= first_hi; ++t) s = s + L.load(t);
  L.store(0, s, L.mult(0));
  // Position x has an entering value iff x + r <= w - 1 and a leaving value
  // iff x - r - 1 >= 0. Both bounds split [1, w) into at most three ranges.
  const int enter_end = w - r < 1 ? 1 : (w - r > w ? w : w - r);  // x < enter_end: entering
  const int leave_begin = r + 1 < w ? r + 1 : w;                 // x >= leave_begin: leaving
  if (enter_end <= leave_begin) {
    blur_range<true, false>(L, 1, enter_end, s);
    blur_range<false, false>(L, enter_end, leave_begin, s);
    blur_range<false, true>(L, leave_begin, w, s);
  } else {
    blur_range<true, false>(L, 1, leave_begin, s);
    blur_range<true, true>(L, leave_begin, enter_end, s);
    blur_range<false, true>(L, enter_end, w, s);
  }
}

// Waves of one pass for DP < 64 (64 / DP lines per wave).
template <int DP>
inline int64_t blur_reg_waves(int w) {
  return (w + 64 / DP - 1) / (64 / DP);
}

template <int DP, typename S>
__global__ __launch_bounds__(kBlock) void k_blur(const S* __restrict__ in, S* __restrict__ out,
                                                 int w, const DevState* __restrict__ st, int radius,
                                                 int vertical, const float* __restrict__ inv,
                                                 int32_t* __restrict__ table) {
  int r;
  if (!pass_radius(st, radius, r)) return;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) >> 6;
  blur_reg_lines<DP, S>(in, out, w, r, vertical, inv, wave, threadIdx.x & 63);
  if (table != nullptr) fill_group_table<kBlock>(table, st->beta, st->keys, blockIdx.x, gridDim.x);
}

// Cache hints, measured on whole sorts. The assignment reads every cell of G
// and T once per reorder, in random group order: streaming (non-temporal)
// loads keep those reads from evicting what the next blur pass reads (1024^2
// float32 with normal loads: assignment 109 -> 132 us). The staged blur
// stores its lines normally where the grid is about the size of the 256 MB
// Infinity Cache (the 128-row ring: 1024^2 float32 and 1448^2 bfloat16
// grids), as the next kernel reads them soon after: streaming stores made
// those sorts 3.7 % and 1.4 % slower. float32 grids of more than 1024 lines
// (the 64-row ring) are twice that size or more; there streaming stores are
// faster (1448^2: 5568 against 5668 ms; 2091^2: 15.5 against 16.3 s).
template <int RR>
constexpr bool blur_stream_stores() {
  return RR < 128;
}
constexpr bool kAssignStreamLoads = true;

typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

// 16-byte load / store with a streaming hint (the data is not used again
// from the cache) when `nt`.
template <bool nt>
__device__ __forceinline__ uint4 load16(const void* p) {
  if constexpr (nt) {
    const u32x4_t v = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
  } else {
    return *reinterpret_cast<const uint4*>(p);
  }
}
template <bool nt>
__device__ __forceinline__ void store16(void* p, uint4 v) {
  if constexpr (nt) {
    u32x4_t u = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(u, reinterpret_cast<u32x4_t*>(p));
  } else {
    *reinterpret_cast<uint4*>(p) = v;
  }
}

typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));

// Streaming-hint load / store of a Quad (float4 or uint2), as above.
template <bool nt, typename Q>
__device__ __forceinline__ Q load_quad(const Q* p) {
  if constexpr (nt && sizeof(Q) == 16) {
    const u32x4_t v = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(p));
    return __builtin_bit_cast(Q, v);
  } else if constexpr (nt && sizeof(Q) == 8) {
    const u32x2_t v = __builtin_nontemporal_load(reinterpret_cast<const u32x2_t*>(p));
    return __builtin_bit_cast(Q, v);
  } else {
    return *p;
  }
}

// Blur pass for cells of at least 16 bytes, staged through LDS. Same
// arithmetic as k_blur (one running sum per line and channel, same operation
// order); the memory side is built on gfx950's direct global -> LDS loads.
//
// A wave walks 64 / DP lines side by side (DP = 64: one line). LDS row p holds
// one position of all of them: element l * DP + c is channel c of line l, and
// lane l * DP + c runs that chain. A load instruction fills kPos consecutive
// rows (1 KB): load lane (q, j) moves the 16-byte piece j of position q, piece
// j belonging to line j / kPiecesPerCell, and the data goes straight to LDS
// without passing through registers, so several chunks can be in flight per
// wave. Outputs are summed into LDS rows and leave as 16-byte stores (cache
// hints: blur_stream_stores).
//
// Chunks are kChunk positions aligned to multiples of kChunk (a row walk then
// reads and writes whole aligned 4 KB blocks). The line is loaded chunk by
// chunk into a ring of rows (row = position modulo the ring). Step e takes
// chunk e: first its positions up to min(r, w - 1) go into the starting sum,
// then, from step A = ceil(r / kChunk) on, the outputs x of chunk e - A (x + r
// lies in chunk e or e - 1). While the ring also holds every leaving position
// x - r - 1 still to come beside the chunks in flight, leaving values are read
// back from it; otherwise the ring is split in two halves and the leaving
// chunks reach the upper half from KR register slots, where each chunk was
// kept since it entered (float32 over large working sets: 24 slots with the
// 128-row ring, 48 <= r <= 192; 8 with the 64-row ring, 16 <= r <= 64), or
// from a second load stream (the same positions again).
// Loads are issued at positions clamped into the line (a clamped load fetches
// a value the sums never use), so every chunk is exactly kVec load
// instructions.
//
// Waits. Vector memory operations of a wave complete in issue order, so
// "chunk c has arrived" is "at most n operations are outstanding", n being the
// number of loads and stores issued after chunk c's last load. Every step
// issues, in this order, the stores of the chunk it summed and then the loads
// of issue slot e + kDepth - 1 (entering chunk, then leaving chunk); n follows
// from that schedule (ops_after). The loads are written as asm so that the
// compiler does not add its own conservative wait (every load done) before
// each LDS read; M0 (the LDS base of a load) is set in the same asm statement,
// and no compiler-generated code of these kernels uses M0.
template <typename S, int RR, int KR = 0>
struct RingShape {
  static constexpr int kRowBytes = 64 * static_cast<int>(sizeof(S));  // one position of the wave's lines
  static constexpr int kLanesPerRow = kRowBytes / 16;
  static constexpr int kPos = 64 / kLanesPerRow;  // positions per load instruction: 4 (float32), 8 (bfloat16)
  static constexpr int kChunk = 16;               // positions per chunk
  static constexpr int kVec = kChunk / kPos;      // load instructions per chunk
#ifndef PLAS_BLUR_DEPTH
#define PLAS_BLUR_DEPTH 3
#endif
#ifndef PLAS_BLUR_EARLY
#define PLAS_BLUR_EARLY 0
#endif
  // issue slots in flight, the one being summed included (two with the
  // small ring, whose split halves hold two chunks)
  static constexpr int kDepth = RR >= 128 ? PLAS_BLUR_DEPTH : 2;
  static constexpr bool kEarly = PLAS_BLUR_EARLY;  // a step issues its loads before summing (else after)
  static constexpr int kRingRows = RR;
  static constexpr int kSlots = kRingRows / kChunk;
  static constexpr int kRegChunks = KR;  // register slots of leaving chunks (0: none)
  static constexpr int kRegWords = kChunk * static_cast<int>(sizeof(S)) / 4;  // registers per chunk
  static constexpr int kHalfRows = kRingRows / 2;  // rows of each stream when the ring is split
  static_assert(kRingRows % kChunk == 0 && (kRingRows & (kRingRows - 1)) == 0, "ring shape");
  static_assert(KR == 0 || sizeof(S) == 4, "register slots hold float32 chunks");
  static_assert(kHalfRows / kChunk >= kDepth + (kEarly ? 1 : 0), "a split half holds the chunks in use and in flight");
};

// LDS of one wave: (RR + 16) rows of 256 B (float32) or 128 B (bfloat16),
// 36 KB / 18 KB with the 128-row ring.
template <typename S, int RR>
struct alignas(16) RingLds {
  S ring[RingShape<S, RR>::kRingRows][64];
  S out[RingShape<S, RR>::kChunk][64];
};

// Leaving values come from the entering ring when, at every step, the chunk
// issued then does not overwrite a leaving position still to come: with A =
// ceil(r / kChunk) chunks between a step's chunk and its outputs and
// ceil((r + 1) / kChunk) between an output chunk and its leaving positions,
// A + ceil((r + 1) / kChunk) <= kSlots + 1 - kDepth.
template <typename S, int RR>
__device__ __forceinline__ bool ring_leave(int r) {
  using Sh = RingShape<S, RR>;
  const int a = (r + Sh::kChunk - 1) / Sh::kChunk;
  const int b = (r + Sh::kChunk) / Sh::kChunk;
  return a + b <= Sh::kSlots + (Sh::kEarly ? 0 : 1) - Sh::kDepth;
}

// One direct load: 16 bytes per lane from `src` to LDS byte address
// m0 + 16 * lane, with a streaming hint (the data is not read again through
// the cache) when `nt`. A preceding LDS read of the rows it overwrites must
// have completed: lgkmcnt(0) first.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"  // M0 is named as clobbered on purpose
template <bool nt>
__device__ __forceinline__ void dma16(const void* src, uint32_t m0) {
  if constexpr (nt)
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off nt"
                 :
                 : "v"(src), "s"(m0)
                 : "memory", "m0");
  else
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
                 :
                 : "v"(src), "s"(m0)
                 : "memory", "m0");
}
#pragma clang diagnostic pop

// Cache hints of the two load streams. The leaving stream (a second read of
// positions the entering stream read 2r + 1 positions earlier) streams
// through, so that it does not evict entering data the L2 still holds for
// it. The entering stream streams in the column pass when the grids in
// flight exceed 128 MiB (blur_large_working_set): its input H is dead after
// that pass, and keeping H out of the Infinity Cache leaves room for G and
// T, which the assignment reads next (1024^2 float32: column pass 98 -> 87
// us, assignment 110 -> 104 us at r <= 15). Streaming the row pass's loads
// of G as well made the column pass slower again (101 us); grids the cache
// holds whole ran 1-2 % slower with streaming column loads.
constexpr bool kBlurLeaveStream = true;

// s_waitcnt vmcnt(n) for a run-time n (rounded down, which only waits
// longer).
template <int N>
__device__ __forceinline__ void wait_vm() {
  asm volatile("s_waitcnt vmcnt(%0)" : : "n"(N) : "memory");
}
__device__ __forceinline__ void wait_vm_dyn(int n) {
  switch (n < 0 ? 0 : n) {
    case 0: wait_vm<0>(); break;
    case 1: wait_vm<1>(); break;
    case 2: wait_vm<2>(); break;
    case 3: wait_vm<3>(); break;
    case 4: wait_vm<4>(); break;
    case 5: wait_vm<5>(); break;
    case 6: wait_vm<6>(); break;
    case 7: wait_vm<7>(); break;
    case 8: wait_vm<8>(); break;
    case 9: wait_vm<9>(); break;
    case 10: wait_vm<10>(); break;
    case 11: wait_vm<11>(); break;
    case 12: wait_vm<12>(); break;
    case 13: wait_vm<13>(); break;
    case 14: wait_vm<14>(); break;
    case 15: wait_vm<15>(); break;
    default: wait_vm<16>(); break;
  }
}

template <typename S, int DP, int RR, int KR, bool NT>
struct RingLine {
  using Sh = RingShape<S, RR, KR>;
  static constexpr int kChunk = Sh::kChunk;
  static constexpr int kPiecesPerCell = DP * static_cast<int>(sizeof(S)) / 16;
  static_assert(kPiecesPerCell >= 1, "a cell must hold at least one 16-byte piece");
  const S* __restrict__ src;  // the pass's input grid
  S* __restrict__ dst;        // and output grid
  int64_t step;     // elements between consecutive positions of a line
  int64_t ld_off;   // element offset of this lane's load piece at position 0
  bool ld_ok;       // the load piece's line exists (else its loads are clamped and its stores skipped)
  int w, r, first_hi;
  int n_chunks;  // M: chunks of the line
  int ahead;     // A = ceil(r / kChunk): step e sums the outputs of chunk e - A
  int lag;       // the leaving chunk needed at step e is e - lag (split ring)
  int n_steps;   // A + M
  int q, j, lane;
  bool split;        // the leaving values have their own region (the ring's upper half)
  bool regs;         // split, and the leaving chunks come from registers instead of a second load stream
  int enter_mask;    // ring rows of the entering stream - 1
  uint32_t ring_m0;  // LDS byte address of ring row 0 (the same for all lanes)
  RingLds<S, RR>* lds;

  __device__ __forceinline__ int clamp_pos(int t) const { return t < 0 ? 0 : (t > w - 1 ? w - 1 : t); }

  // kVec loads of chunk m (positions kChunk m ..) into rows row0 ..
  template <bool nt>
  __device__ __forceinline__ void load_chunk(int m, int row0) const {
    const int pos0 = m * kChunk;
    const uint32_t m0 = ring_m0 + static_cast<uint32_t>(row0 * Sh::kRowBytes);
    if (pos0 + kChunk - 1 <= w - 1) {
      const S* p = src + ld_off + static_cast<int64_t>(pos0 + q) * step;
      const int64_t inc = static_cast<int64_t>(Sh::kPos) * step;
#pragma unroll
      for (int i = 0; i < Sh::kVec; ++i) dma16<nt>(p + i * inc, m0 + i * 1024u);
    } else {
#pragma unroll
      for (int i = 0; i < Sh::kVec; ++i)
        dma16<nt>(src + ld_off + static_cast<int64_t>(clamp_pos(pos0 + Sh::kPos * i + q)) * step, m0 + i * 1024u);
    }
  }

  // Issue slot u: entering chunk u and, when split, leaving chunk u - lag.
  __device__ __forceinline__ bool slot_enter(int u) const { return u < n_chunks; }
  __device__ __forceinline__ bool slot_leave(int u) const {
    return split && !regs && u - lag >= 0 && u - lag < n_chunks;
  }
  __device__ __forceinline__ void issue(int u) const {
    if (slot_enter(u)) load_chunk<NT>(u, (u * kChunk) & enter_mask);
    if (slot_leave(u))
      load_chunk<kBlurLeaveStream>(u - lag, Sh::kHalfRows + (((u - lag) * kChunk) & (Sh::kHalfRows - 1)));
  }
  __device__ __forceinline__ int slot_loads(int u) const {
    return Sh::kVec * ((slot_enter(u) ? 1 : 0) + (slot_leave(u) ? 1 : 0));
  }
  // Stores of step s: a whole output chunk (every output chunk but the last
  // lies inside the line, and only the last step stores the last one).
  __device__ __forceinline__ int step_stores(int s) const { return s >= ahead ? Sh::kVec : 0; }
  // Operations issued after slot e's loads, as of the start of step e: the
  // loads of slots e + 1 .. e + kDepth - 2 and the stores of the steps that
  // came after slot e was issued.
  __device__ __forceinline__ int ops_after(int e) const {
    int n = 0;
#pragma unroll
    for (int u = 1; u <= Sh::kDepth - 2; ++u) n += slot_loads(e + u);
    const int first = e - Sh::kDepth + (Sh::kEarly ? 1 : 2);
    const int s0 = first > 0 ? first : 0;
    for (int s = s0; s < e; ++s) n += step_stores(s);
    return n;
  }

  __device__ __forceinline__ int enter_row(int x) const { return (x + r) & enter_mask; }
  __device__ __forceinline__ int leave_row(int x) const {
    const int t = x - r - 1;
    return split ? Sh::kHalfRows + (t & (Sh::kHalfRows - 1)) : (t & (Sh::kRingRows - 1));
  }
  __device__ __forceinline__ float enter_val(int x) const {
    return Storage<S>::widen(lds->ring[enter_row(x)][lane]);
  }
  __device__ __forceinline__ float leave_val(int x) const {
    return Storage<S>::widen(lds->ring[leave_row(x)][lane]);
  }

  // Outputs x0 .. x0 + kChunk - 1, all inside the grid, all with (ENTER) or
  // without an entering value and all with (LEAVE) or without a leaving one:
  // no per-position tests. With both at every position the window holds
  // 2r + 1 cells, and with neither it is the whole line: one multiplier
  // serves all positions. Otherwise each position takes its own from lane p.
  template <bool ENTER, bool LEAVE>
  __device__ __forceinline__ void run_uniform(int x0, float mult, float& s) const {
    constexpr bool kConstMult = ENTER == LEAVE;
    const int mult_bits = __float_as_int(mult);
    float e[kChunk], l[kChunk];
    // The chunk's entering rows and its leaving rows are each kChunk
    // consecutive ring rows unless they wrap around the end of their region:
    // then one base address with constant offsets reads them.
    const int eb = enter_row(x0), lb = leave_row(x0);
    const bool e_flat = !ENTER || eb + kChunk <= enter_mask + 1;
    const bool l_flat = !LEAVE || (lb & (split ? Sh::kHalfRows - 1 : Sh::kRingRows - 1)) + kChunk <=
                                      (split ? Sh::kHalfRows : Sh::kRingRows);
    if (e_flat && l_flat) {
      const S* ep = &lds->ring[ENTER ? eb : 0][lane];
      const S* lp = &lds->ring[LEAVE ? lb : 0][lane];
#pragma unroll
      for (int p = 0; p < kChunk; ++p) {
        if (ENTER) e[p] = Storage<S>::widen(ep[p * 64]);
        if (LEAVE) l[p] = Storage<S>::widen(lp[p * 64]);
      }
    } else {
#pragma unroll
      for (int p = 0; p < kChunk; ++p) {
        if (ENTER) e[p] = enter_val(x0 + p);
        if (LEAVE) l[p] = leave_val(x0 + p);
      }
    }
    const float m_const = kConstMult ? __int_as_float(__builtin_amdgcn_readfirstlane(mult_bits)) : 0.0f;
#pragma unroll
    for (int p = 0; p < kChunk; ++p) {
      if (ENTER) s = s + e[p];
      if (LEAVE) s = s - l[p];
      const float m = kConstMult ? m_const : __int_as_float(__builtin_amdgcn_readlane(mult_bits, p));
      lds->out[p][lane] = Storage<S>::narrow(s * m);
    }
  }

  // Any outputs (x = 0 included: the starting sum as it is): the tests of
  // each position select the update.
  __device__ __forceinline__ void run_mixed(int x0, float mult, float& s) const {
    const int mult_bits = __float_as_int(mult);
    float e[kChunk], l[kChunk];
#pragma unroll
    for (int p = 0; p < kChunk; ++p) {
      e[p] = enter_val(x0 + p);
      l[p] = leave_val(x0 + p);
    }
#pragma unroll
    for (int p = 0; p < kChunk; ++p) {
      const int x = x0 + p;
      const bool inside = x >= 1 && x < w;
      const float with_enter = s + e[p];
      s = (inside && x + r <= w - 1) ? with_enter : s;
      const float with_leave = s - l[p];
      s = (inside && x - r - 1 >= 0) ? with_leave : s;
      lds->out[p][lane] = Storage<S>::narrow(s * __int_as_float(__builtin_amdgcn_readlane(mult_bits, p)));
    }
  }

  // The positions of chunk e up to first_hi, in ascending order, into the
  // starting sum (position 0 starts it).
  __device__ __forceinline__ void start_sum(int e, float& s) const {
    const int t0 = e * kChunk;
    float v[kChunk];
#pragma unroll
    for (int p = 0; p < kChunk; ++p) v[p] = Storage<S>::widen(lds->ring[(t0 + p) & enter_mask][lane]);
    if (t0 > 0 && t0 + kChunk - 1 <= first_hi) {
#pragma unroll
      for (int p = 0; p < kChunk; ++p) s = s + v[p];
    } else {
#pragma unroll
      for (int p = 0; p < kChunk; ++p) {
        const int t = t0 + p;
        const float added = t == 0 ? v[p] : s + v[p];
        s = t <= first_hi ? added : s;
      }
    }
  }

  // Output chunk k (positions x0 = k kChunk ..): sum, then store the chunk's
  // rows as 16-byte pieces.
  __device__ __forceinline__ void outputs(int k, float& s) const {
    const int x0 = k * kChunk;
    const int x1 = x0 + kChunk - 1;
    // Lane p < kChunk: float32(1 / count) of position x0 + p (correctly
    // rounded, as the host table 1.0f / c).
    float mult;
    {
      const int x = clamp_pos(x0 + (lane & (kChunk - 1)));
      const int hi = x + r < w - 1 ? x + r : w - 1;
      const int lo = x - r > 0 ? x - r : 0;
      mult = 1.0f / static_cast<float>(hi - lo + 1);
    }
    const bool all_in = x0 >= 1 && x1 < w;
    const bool enter_all = x1 + r <= w - 1, enter_none = x0 + r > w - 1;
    const bool leave_all = x0 - r - 1 >= 0, leave_none = x1 - r - 1 < 0;
    if (all_in && enter_all && leave_all)
      run_uniform<true, true>(x0, mult, s);
    else if (all_in && enter_all && leave_none)
      run_uniform<true, false>(x0, mult, s);
    else if (all_in && enter_none && leave_all)
      run_uniform<false, true>(x0, mult, s);
    else if (all_in && enter_none && leave_none)
      run_uniform<false, false>(x0, mult, s);
    else
      run_mixed(x0, mult, s);
#pragma unroll
    for (int i = 0; i < Sh::kVec; ++i) {
      const int x = x0 + Sh::kPos * i + q;
      if (x < w && ld_ok)
        store16<blur_stream_stores<RR>()>(dst + ld_off + static_cast<int64_t>(x) * step,
                                   *reinterpret_cast<const uint4*>(&lds->out[Sh::kPos * i + q][16 / sizeof(S) * j]));
    }
  }

  // Register ring of the leaving values: step e reads chunk e back from the
  // entering half and swaps it with register slot e mod lag, which holds
  // chunk e - lag, the newest leaving chunk of the step; that chunk goes to
  // its rows of the leaving half. A chunk is used as leaving values at steps
  // e and e + 1 only, and the leaving half holds four. A chunk's kChunk rows
  // are contiguous in both halves, so it moves as 16-byte pieces (lane l
  // holds bytes 16 l .. of each KB) in whatever order: only its place in the
  // leaving half matters. Past the last chunk the rows read are stale; what
  // they push is never popped (a chunk pushed at step e >= M would pop at
  // e + lag >= M + A, after the last step).
  using Word = uint32_t;
  static constexpr int kWords = Sh::kRegWords;  // per lane and chunk
  static constexpr int kPieces = kWords / 4;    // 16-byte pieces per lane and chunk
  template <int K>
  __device__ __forceinline__ void exchange(Word (&keep)[K][kWords], int slot, int e) const {
    Word in[kWords], out[kWords];
    const char* ep = reinterpret_cast<const char*>(&lds->ring[(e * kChunk) & enter_mask][0]) + 16 * lane;
#pragma unroll
    for (int i = 0; i < kPieces; ++i) {
      const uint4 v = *reinterpret_cast<const uint4*>(ep + 1024 * i);
      in[4 * i] = v.x;
      in[4 * i + 1] = v.y;
      in[4 * i + 2] = v.z;
      in[4 * i + 3] = v.w;
    }
    // The uniform slot is found in two levels of scalar branches: its group
    // of kGroup slots, then the slot.
    constexpr int kGroup = 6;
#pragma unroll
    for (int g = 0; g < K; g += kGroup) {
      if (slot >= g && slot < g + kGroup) {
#pragma unroll
        for (int k = g; k < g + kGroup && k < K; ++k) {
          if (k == slot) {
#pragma unroll
            for (int p = 0; p < kWords; ++p) {
              out[p] = keep[k][p];
              keep[k][p] = in[p];
            }
          }
        }
      }
    }
    if (e >= lag) {
      char* lp = reinterpret_cast<char*>(&lds->ring[Sh::kHalfRows + (((e - lag) * kChunk) & (Sh::kHalfRows - 1))][0]) +
                 16 * lane;
#pragma unroll
      for (int i = 0; i < kPieces; ++i)
        *reinterpret_cast<uint4*>(lp + 1024 * i) = make_uint4(out[4 * i], out[4 * i + 1], out[4 * i + 2], out[4 * i + 3]);
    }
  }

  __device__ __forceinline__ void run_regs() const {
    if constexpr (Sh::kRegChunks > 0) {
      // Zeroed: the first lag steps read a slot (and drop the value) before
      // its first chunk arrives.
      Word keep[Sh::kRegChunks][kWords] = {};
      for (int u = 0; u <= Sh::kDepth - 2; ++u) issue(u);
      float s = 0.0f;
      int slot = 0;
      for (int e = 0; e < n_steps; ++e) {
        if (slot_loads(e) > 0) wait_vm_dyn(ops_after(e));
        if (Sh::kEarly) issue(e + Sh::kDepth - 1);
        exchange<Sh::kRegChunks>(keep, slot, e);
        if (e * kChunk <= first_hi) start_sum(e, s);
        if (e >= ahead) outputs(e - ahead, s);
        if (!Sh::kEarly) issue(e + Sh::kDepth - 1);
        slot = slot + 1 == lag ? 0 : slot + 1;
      }
    }
  }

  __device__ __forceinline__ void run() const {
    if (regs) {
      run_regs();
      return;
    }
    for (int u = 0; u <= Sh::kDepth - 2; ++u) issue(u);
    float s = 0.0f;
    for (int e = 0; e < n_steps; ++e) {
      if (slot_loads(e) > 0) wait_vm_dyn(ops_after(e));
      if (Sh::kEarly) issue(e + Sh::kDepth - 1);
      if (e * kChunk <= first_hi) start_sum(e, s);
      if (e >= ahead) outputs(e - ahead, s);
      if (!Sh::kEarly) issue(e + Sh::kDepth - 1);
    }
  }
};

// Lines line0 .. line0 + 64/DP - 1 of a staged blur pass (those below w),
// by one wave.
template <typename S, int DP, int RR, int KR, bool NT>
__device__ __forceinline__ void blur_staged_line(const S* __restrict__ in, S* __restrict__ out, int w, int r,
                                                 int vertical, int64_t line0, int lane, RingLds<S, RR>* lds) {
  using Sh = RingShape<S, RR, KR>;
  using L_t = RingLine<S, DP, RR, KR, NT>;
  L_t L;
  // Element offset of line l at position 0, and between positions.
  auto line_off = [&](int64_t l) { return vertical ? l * DP : l * w * DP; };
  L.src = in;
  L.dst = out;
  L.step = vertical ? static_cast<int64_t>(w) * DP : DP;
  L.w = w;
  L.r = r;
  L.q = lane / Sh::kLanesPerRow;
  L.j = lane % Sh::kLanesPerRow;
  const int64_t ld_line = line0 + L.j / L_t::kPiecesPerCell;
  L.ld_ok = ld_line < w;
  L.ld_off = line_off(L.ld_ok ? ld_line : w - 1) + (L.j % L_t::kPiecesPerCell) * (16 / static_cast<int>(sizeof(S)));
  L.lane = lane;
  L.lds = lds;
  if (r == 0) {
    const int64_t own_line = line0 + lane / DP;
    const int64_t own_off = line_off(own_line < w ? own_line : w - 1) + lane % DP;
    if (own_line < w)
      for (int x = 0; x < w; ++x) L.dst[own_off + x * L.step] = L.src[own_off + x * L.step];
    return;
  }
  L.first_hi = r < w - 1 ? r : w - 1;
  L.n_chunks = (w + Sh::kChunk - 1) / Sh::kChunk;
  L.ahead = (r + Sh::kChunk - 1) / Sh::kChunk;
  L.n_steps = L.ahead + L.n_chunks;
  L.split = !ring_leave<S, RR>(r);
  // Step e sums outputs of chunk k = e - A, whose leaving positions reach
  // up to k kChunk + kChunk - 2 - r: chunk e - lag.
  L.lag = L.ahead - ((Sh::kChunk - 2 - r) >= 0 ? (Sh::kChunk - 2 - r) / Sh::kChunk
                                               : -((r - Sh::kChunk + 2 + Sh::kChunk - 1) / Sh::kChunk));
  L.regs = L.split && L.lag <= Sh::kRegChunks;
  L.enter_mask = (L.split ? Sh::kHalfRows : Sh::kRingRows) - 1;
  L.ring_m0 = __builtin_amdgcn_readfirstlane(
      static_cast<uint32_t>(reinterpret_cast<uintptr_t>((__attribute__((address_space(3))) S*)(&lds->ring[0][0]))));
  L.run();
}

// Waves per SIMD a staged kernel keeps room for in registers: one float32
// wave with the 128-row ring (its LDS allows no more), else two.
template <typename S, int RR>
constexpr int staged_waves_per_eu() {
  return sizeof(S) == 4 && RR >= 128 ? 1 : 2;
}

// One group of 64/DP lines per wave, WPB waves per block: block `bid` of
// `nblocks` takes groups bid * WPB + wave, and walks on with a stride if
// there are more groups than waves.
template <typename S, int DP, int WPB, int RR, int KR, bool NT>
__device__ __forceinline__ void blur_staged_lines(const S* __restrict__ in, S* __restrict__ out, int w, int r,
                                                  int vertical, int64_t bid, int64_t nblocks, RingLds<S, RR>* stage) {
  constexpr int kLinesPerWave = 64 / DP;
  const int wib = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  for (int64_t g = bid * WPB + wib; g * kLinesPerWave < w; g += nblocks * WPB)
    blur_staged_line<S, DP, RR, KR, NT>(in, out, w, r, vertical, g * kLinesPerWave, lane, stage + wib);
}

// Staged blur pass for cells of at least 16 bytes (DP * sizeof(S) >= 16),
// with a ring of RR rows per wave and KR register slots; NT: the entering
// loads stream.
template <typename S, int DP, int WPB, int RR, int KR, bool NT>
__global__ __launch_bounds__(WPB * 64) __attribute__((amdgpu_waves_per_eu(staged_waves_per_eu<S, RR>())))
void k_blur_staged(const S* __restrict__ in, S* __restrict__ out, int w, const DevState* __restrict__ st, int radius,
                   int vertical, int32_t* __restrict__ table) {
  __shared__ RingLds<S, RR> s_stage[WPB];
  int r;
  if (!pass_radius(st, radius, r)) return;
  blur_staged_lines<S, DP, WPB, RR, KR, NT>(in, out, w, r, vertical, blockIdx.x, gridDim.x, s_stage);
  if (table != nullptr) fill_group_table<WPB * 64>(table, st->beta, st->keys, blockIdx.x, gridDim.x);
}

// Register slots a wave keeps for the leaving values (float32): 24 with the
// 128-row ring (384 registers; one wave per SIMD, as the ring's LDS allows),
// 8 with the 64-row ring (128 registers; two waves per SIMD). bfloat16
// passes run two waves per SIMD and keep the second load stream: with 16
// slots they measured no faster (1448^2, r = 48..128: 146 / 144 us per
// row / column pass, against 138 / 148 us).
template <typename S, int RR>
constexpr int ring_register_chunks() {
  return sizeof(S) == 4 ? (RR >= 128 ? 24 : 8) : 0;
}

// Cells of DP * sizeof(S) bytes are moved in 16-byte pieces when they hold
// at least one (every float32 width, bfloat16 from 8 channels up).
template <typename S, int DP>
constexpr bool staged_cells() {
  return DP * static_cast<int>(sizeof(S)) >= 16;
}

// float32 waves of a staged pass with the 128-row ring (37 KB of LDS each)
// that fit on the chip at once: 4 per CU, 256 CUs.
constexpr int64_t kStagedWavesAtLargeRing = 1024;

// Wave groups (of 64/DP lines) of a staged pass over w lines.
template <int DP>
inline int64_t staged_groups(int w) {
  return (w + 64 / DP - 1) / (64 / DP);
}

// ---------------------------------------------------------- group table

__global__ __launch_bounds__(kBlock) void k_group_table(int32_t* __restrict__ table,
                                                        const DevState* __restrict__ st) {
  if (st->done) return;
  fill_group_table<kBlock>(table, st->beta, st->keys, blockIdx.x, gridDim.x);
}

// Squared distance partial over one lane's 4 channels, as the two lowest
// levels of the pairwise tree: (c0^2 + c1^2) + (c2^2 + c3^2).
__device__ inline float chunk_sq(const float4 a, const float4 b) {
  const float e0 = a.x - b.x, e1 = a.y - b.y, e2 = a.z - b.z, e3 = a.w - b.w;
  return (e0 * e0 + e1 * e1) + (e2 * e2 + e3 * e3);
}

// Channels per lane in the assignment: 8 bfloat16 channels (one 16-byte
// load) when a cell holds at least 8, else 4 (a float4, or 8 bytes of
// bfloat16). Eight channels per lane add the tree's third level, (first
// four) + (last four), inside the lane; the lanes then reduce the rest.
template <typename S, int DP>
constexpr int assign_channels() {
  return (sizeof(S) == 2 && DP >= 8) ? 8 : 4;
}

template <typename S, int DP>
struct AssignVec {
  using Quad = typename Storage<S>::Quad;
  using T = Quad;
  __device__ static __forceinline__ float sq(const T& a, const T& b) {
    return chunk_sq(Storage<S>::widen4(a), Storage<S>::widen4(b));
  }
};

template <>
struct AssignVec<uint16_t, 64> {
  using T = uint4;
  __device__ static __forceinline__ float sq(const T& a, const T& b) {
    const float lo = chunk_sq(Storage<uint16_t>::widen4(make_uint2(a.x, a.y)),
                              Storage<uint16_t>::widen4(make_uint2(b.x, b.y)));
    const float hi = chunk_sq(Storage<uint16_t>::widen4(make_uint2(a.z, a.w)),
                              Storage<uint16_t>::widen4(make_uint2(b.z, b.w)));
    return lo + hi;
  }
};
template <>
struct AssignVec<uint16_t, 32> : AssignVec<uint16_t, 64> {};
template <>
struct AssignVec<uint16_t, 16> : AssignVec<uint16_t, 64> {};
template <>
struct AssignVec<uint16_t, 8> : AssignVec<uint16_t, 64> {};

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}


// The 24 orderings of (0,1,2,3) in lexicographic order as position codes
// (sigma(i) in bits 2i..2i+1), eight codes per 64-bit word, ordering m in
// byte m mod 8 of word m / 8:
//   0123 0132 0213 0231 0312 0321 1023 1032 | 1203 1230 1302 1320 2013 2031
//   2103 2130 | 2301 2310 3012 3021 3102 3120 3201 3210
__device__ __forceinline__ uint32_t order_code(int m) {
  constexpr uint64_t kOrders0 = 0xB1E16C9C78D8B4E4ull;
  constexpr uint64_t kOrders1 = 0x36C672D22D8D39C9ull;
  constexpr uint64_t kOrders2 = 0x1B4B278763931E4Eull;
  const uint64_t word = m < 8 ? kOrders0 : (m < 16 ? kOrders1 : kOrders2);
  return static_cast<uint32_t>((word >> (8 * (m & 7))) & 0xff);
}

// One reorder's blockwise assignment. Items are the groups of every block
// (item < groups) followed by the cells in no group (singles), whose
// distance still counts towards the energy. LG = DP / C lanes serve one
// item, C = assign_channels<S, DP>() (4, or 8 for bfloat16 cells of 8 or
// more channels): lane `sub` holds channels C*sub .. C*sub+C-1 of the item's
// four grid cells and four target cells and forms all 16 pair partials as
// the lowest levels of the channel tree. The rest of the work is split
// across the LG lanes:
//  - a transposed butterfly: at tree level b each lane keeps the pairs whose
//    bit b matches its own lane bit, adds the partner's partial for them and
//    hands over the others, so after log2(LG) levels lane L holds the exact
//    distances of pairs q = t*LG + L (each still summed left half + right
//    half, level by level, as the channel tree prescribes);
//  - the quantised pair costs go to LDS; lane L evaluates orderings
//    L, L+LG, ... and the lanes pick the first minimum with a butterfly on
//    (cost, ordering index).
// Exact quotient a / d for 0 <= a < 2^31 and 1 <= d < 2^30 from a float64
// reciprocal: the estimate is off by at most one (relative error of the
// product below 2^-51), and the remainder's sign fixes it.
struct FastDiv {
  uint32_t d;
  double inv;
  __device__ __forceinline__ void init(uint32_t divisor) {
    d = divisor;
    inv = 1.0 / static_cast<double>(divisor);
  }
  __device__ __forceinline__ uint32_t div(uint32_t a) const {
    uint32_t q = static_cast<uint32_t>(static_cast<double>(a) * inv);
    const int32_t r = static_cast<int32_t>(a - q * d);
    if (r < 0)
      --q;
    else if (r >= static_cast<int32_t>(d))
      ++q;
    return q;
  }
};

// Geometry of one reorder's items, read once per thread. Item indices, cell
// indices and counts stay below 2^31 (side <= 46340).
struct ItemGeometry {
  const int32_t* __restrict__ table;
  int w, beta, nb, dy, dx, R;
  uint32_t groups, total, strip_rows, strip;
  FastDiv by_gpb, by_nb, by_w, by_rest;

  __device__ __forceinline__ void init(const DevState* __restrict__ st, const int32_t* __restrict__ tbl) {
    table = tbl;
    w = st->w;
    beta = st->beta;
    nb = st->nb;
    dy = st->dy;
    dx = st->dx;
    R = nb * beta;
    groups = static_cast<uint32_t>(st->groups);
    total = static_cast<uint32_t>(st->groups + st->singles);
    strip_rows = static_cast<uint32_t>(w - R) * static_cast<uint32_t>(w);
    strip = static_cast<uint32_t>(w) * w - static_cast<uint32_t>(R) * R;
    by_gpb.init(static_cast<uint32_t>(st->groups_per_block > 0 ? st->groups_per_block : 1));
    by_nb.init(static_cast<uint32_t>(nb));
    by_w.init(static_cast<uint32_t>(w));
    by_rest.init(static_cast<uint32_t>(w - R > 0 ? w - R : 1));
  }

  // The four cells of group `item`, or four times the cell of single `item`
  // (cells in no group: first the rolled-grid rows below the nb*beta square,
  // then the columns right of it, then the left-over cell pi(beta^2 - 1) of
  // each block when beta is odd). Inactive items map to cell 0.
  __device__ __forceinline__ void cells(uint32_t item, int32_t cell[4]) const {
    if (item < groups) {
      const uint32_t b = by_gpb.div(item);
      const uint32_t g = item - b * by_gpb.d;
      const int by = static_cast<int>(by_nb.div(b));
      const int bx = static_cast<int>(b) - by * nb;
      const int4 t4 = reinterpret_cast<const int4*>(table)[g];
      const int32_t t[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int y = dy + by * beta + (t[i] >> 16);
        int x = dx + bx * beta + (t[i] & 0xffff);
        if (y >= w) y -= w;
        if (x >= w) x -= w;
        cell[i] = y * w + x;
      }
      return;
    }
    int32_t p = 0;
    if (item < total) {
      const uint32_t t = item - groups;
      int u, v;
      if (t < strip) {
        if (t < strip_rows) {
          const uint32_t qy = by_w.div(t);
          u = R + static_cast<int>(qy);
          v = static_cast<int>(t - qy * by_w.d);
        } else {
          const uint32_t t2 = t - strip_rows;
          const uint32_t qy = by_rest.div(t2);
          u = static_cast<int>(qy);
          v = R + static_cast<int>(t2 - qy * by_rest.d);
        }
      } else {
        const uint32_t b = t - strip;
        const int by = static_cast<int>(by_nb.div(b));
        const int bx = static_cast<int>(b) - by * nb;
        const int32_t tt = table[static_cast<int64_t>(beta) * beta - 1];
        u = by * beta + (tt >> 16);
        v = bx * beta + (tt & 0xffff);
      }
      int y = u + dy, x = v + dx;
      if (y >= w) y -= w;
      if (x >= w) x -= w;
      p = y * w + x;
    }
    cell[0] = cell[1] = cell[2] = cell[3] = p;
  }
};

// Cross-lane moves within 16-lane rows (DPP): the value of lane i ^ (1 << b).
// Rows are rotated for b = 2 (i + 4 or i - 4 depending on bit 2) and b = 3.
template <int B>
__device__ __forceinline__ int dpp_xor(int v) {
  if constexpr (B == 0) {
    return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  } else if constexpr (B == 1) {
    return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  } else if constexpr (B == 2) {
    const int up = __builtin_amdgcn_update_dpp(0, v, 0x12C, 0xF, 0xF, false);    // row_ror 12: lane i + 4
    const int down = __builtin_amdgcn_update_dpp(0, v, 0x124, 0xF, 0xF, false);  // row_ror 4: lane i - 4
    return (__lane_id() & 4) ? down : up;
  } else {
    return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);  // row_ror 8: lane i ^ 8
  }
}

template <int B>
__device__ __forceinline__ float dpp_xor_f(float v) {
  return __int_as_float(dpp_xor<B>(__float_as_int(v)));
}

template <int B>
__device__ __forceinline__ unsigned long long dpp_xor_u64(unsigned long long v) {
  const int lo = dpp_xor<B>(static_cast<int>(v & 0xffffffffull));
  const int hi = dpp_xor<B>(static_cast<int>(v >> 32));
  return (static_cast<unsigned long long>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
}

// One level of the transposed butterfly over the item's pair partials: lanes
// with bit B clear keep the even pairs, the others the odd ones, each adding
// its partner's partial of the kept pair (partner = lane ^ (1 << B)).
template <int B, int N>
__device__ __forceinline__ void transpose_level(float* part, bool upper) {
#pragma unroll
  for (int t = 0; t < N; ++t) {
    const float lo = part[2 * t], hi = part[2 * t + 1];
    const float sum_lo = lo + dpp_xor_f<B>(lo);
    const float sum_hi = hi + dpp_xor_f<B>(hi);
    part[t] = upper ? sum_hi : sum_lo;
  }
}

// First minimum across the item's lanes at level B: smaller cost, then
// smaller ordering index.
template <int B>
__device__ __forceinline__ void argmin_level(unsigned long long& best, int& best_m) {
  const unsigned long long oc = dpp_xor_u64<B>(best);
  const int om = dpp_xor<B>(best_m);
  if (oc < best || (oc == best && om < best_m)) {
    best = oc;
    best_m = om;
  }
}

// Block `bid` of `nblocks` blocks that share one reorder's items.
template <int DP, typename S>
__device__ __forceinline__ void assign_items(S* __restrict__ G, const S* __restrict__ T, int32_t* __restrict__ P,
                                             const int32_t* __restrict__ table, DevState* __restrict__ st,
                                             int64_t bid, int64_t nblocks) {
  using V = AssignVec<S, DP>;
  using Vec = typename V::T;
  constexpr int LG = DP / assign_channels<S, DP>();
  static_assert(sizeof(Vec) * LG == DP * sizeof(S), "lane vectors must tile a cell");
  constexpr int IPW = 64 / LG;
  constexpr int LEVELS = LG == 1 ? 0 : LG == 2 ? 1 : LG == 4 ? 2 : LG == 8 ? 3 : 4;
  constexpr int KEEP = 16 / LG;  // pair distances held per lane after the reduction
  __shared__ unsigned long long s_q[kWavesPerBlock][IPW][16];
  ItemGeometry geo;
  geo.init(st, table);
  const double scale = ldexp(1.0, st->s);
  const int lane = threadIdx.x & 63;
  const int wib = threadIdx.x >> 6;
  const int sub = lane % LG, slot = lane / LG;
  unsigned long long* q_item = s_q[wib][slot];
  const int64_t wave = (bid * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = (nblocks * kBlock) >> 6;
  const Vec* __restrict__ G4 = reinterpret_cast<const Vec*>(G);
  const Vec* __restrict__ T4 = reinterpret_cast<const Vec*>(T);
  Vec* __restrict__ Gout = reinterpret_cast<Vec*>(G);
  unsigned long long e_acc = 0, m_acc = 0;

  // Software pipeline: the next item's cells (table reads) are resolved
  // while the current item's grid and target cells are in flight.
  int64_t first = wave * IPW;
  int32_t cell[4];
  geo.cells(static_cast<uint32_t>(first + slot), cell);
  for (; first < geo.total; first += nwaves * IPW) {
    const int64_t item = first + slot;
    const bool active = item < geo.total;
    const bool is_group = item < geo.groups;
    Vec g[4], tg[4];
    int32_t old_perm[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      g[i] = load_quad<kAssignStreamLoads>(G4 + static_cast<int64_t>(cell[i]) * LG + sub);
      tg[i] = load_quad<kAssignStreamLoads>(T4 + static_cast<int64_t>(cell[i]) * LG + sub);
    }
    if (sub == 0 && is_group) {
#pragma unroll
      for (int i = 0; i < 4; ++i) old_perm[i] = P[cell[i]];
    }
    int32_t next_cell[4];
    {
      const int64_t next = first + nwaves * IPW + slot;
      geo.cells(next < geo.total ? static_cast<uint32_t>(next) : geo.total, next_cell);
    }

    // Pair q = 4i + j: grid cell i against target cell j.
    float part[16];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) part[4 * i + j] = V::sq(g[i], tg[j]);
    if constexpr (LEVELS > 0) transpose_level<0, 8>(part, sub & 1);
    if constexpr (LEVELS > 1) transpose_level<1, 4>(part, sub & 2);
    if constexpr (LEVELS > 2) transpose_level<2, 2>(part, sub & 4);
    if constexpr (LEVELS > 3) transpose_level<3, 1>(part, sub & 8);
#pragma unroll
    for (int t = 0; t < KEEP; ++t)
      q_item[t * LG + sub] = static_cast<unsigned long long>(static_cast<double>(part[t]) * scale);
    wave_lds_sync();

    // Orderings sub, sub + LG, ...: this lane's first minimum.
    unsigned long long best = ~0ull;
    int best_m = 24;
#pragma unroll
    for (int m0 = 0; m0 < 24; m0 += LG) {
      const int m = m0 + sub;
      if (m < 24) {
        const uint32_t code = order_code(m);
        const unsigned long long cost = q_item[0 + (code & 3)] + q_item[4 + ((code >> 2) & 3)] +
                                        q_item[8 + ((code >> 4) & 3)] + q_item[12 + ((code >> 6) & 3)];
        if (cost < best) {
          best = cost;
          best_m = m;
        }
      }
    }
    // First minimum across the item's lanes: smaller cost, then smaller index.
    if constexpr (LEVELS > 0) argmin_level<0>(best, best_m);
    if constexpr (LEVELS > 1) argmin_level<1>(best, best_m);
    if constexpr (LEVELS > 2) argmin_level<2>(best, best_m);
    if constexpr (LEVELS > 3) argmin_level<3>(best, best_m);
    const unsigned long long self_cost = q_item[0];
    wave_lds_sync();

    if (is_group && best_m != 0) {
      const uint32_t code = order_code(best_m);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int to = (code >> (2 * i)) & 3;
        if (to != i) {
          const int32_t dst = to == 0 ? cell[0] : to == 1 ? cell[1] : to == 2 ? cell[2] : cell[3];
          Gout[static_cast<int64_t>(dst) * LG + sub] = g[i];
          if (sub == 0) {
            P[dst] = old_perm[i];
            ++m_acc;
          }
        }
      }
    }
    if (active && sub == 0) e_acc += is_group ? best : self_cost;
#pragma unroll
    for (int i = 0; i < 4; ++i) cell[i] = next_cell[i];
  }
  // One pair of atomics per block: waves reduce, then the block.
  __shared__ unsigned long long s_sum[2][kWavesPerBlock];
  e_acc = wave_sum_u64(e_acc);
  m_acc = wave_sum_u64(m_acc);
  if (lane == 0) {
    s_sum[0][wib] = e_acc;
    s_sum[1][wib] = m_acc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long e = 0, m = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) {
      e += s_sum[0][i];
      m += s_sum[1][i];
    }
    const int slot_acc = static_cast<int>(bid % kAccSlots);
    const unsigned long long e_old =
        __hip_atomic_fetch_add(&st->energy_acc[slot_acc], e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long m_old =
        __hip_atomic_fetch_add(&st->moved_acc[slot_acc], m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // Wait for both results (and every earlier memory operation of this
    // wave): once they have returned, both additions have been made where
    // every block's atomics meet, before anything this thread does next
    // (the control step's ticket).
    asm volatile("s_waitcnt vmcnt(0)" : : "v"(e_old), "v"(m_old) : "memory");
  }
}

// The preparation and the control step of a reorder's assignment (defined
// with the controller below).
__device__ void prepare_step(DevState* __restrict__ st, const LevelInfo* __restrict__ levels);
__device__ void reorder_done(DevState* __restrict__ st, const LevelInfo* __restrict__ levels,
                             plas_level_out* __restrict__ trace, uint32_t nblocks);

#ifndef PLAS_ASSIGN_WAVES_PER_EU
#define PLAS_ASSIGN_WAVES_PER_EU 4
#endif

// Occupancy target of the assignment kernels. One wave less per SIMD (more
// registers per lane) where the default would spill to scratch: 8-channel
// bfloat16 lanes hold twice the raw cell data, and with one or two lanes
// per item a lane keeps most of the 16 pair costs and orderings itself.
template <typename S, int DP>
constexpr int assign_waves_per_eu() {
  constexpr int lanes = DP / assign_channels<S, DP>();
  constexpr bool wide = lanes <= 2 || assign_channels<S, DP>() == 8;
  return wide && PLAS_ASSIGN_WAVES_PER_EU > 1 ? PLAS_ASSIGN_WAVES_PER_EU - 1 : PLAS_ASSIGN_WAVES_PER_EU;
}

template <int DP, typename S>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(assign_waves_per_eu<S, DP>())))
void k_assign(S* __restrict__ G, const S* __restrict__ T, int32_t* __restrict__ P,
              const int32_t* __restrict__ table, DevState* __restrict__ st,
              const LevelInfo* __restrict__ levels, plas_level_out* __restrict__ trace, int control) {
  if (st->done) return;
  if (control && blockIdx.x == 0 && threadIdx.x == 0) prepare_step(st, levels);
  assign_items<DP, S>(G, T, P, table, st, blockIdx.x, gridDim.x);
  if (control && threadIdx.x < 64) reorder_done(st, levels, trace, gridDim.x);
}

// ----------------------------------------------------------------- energy

template <int DP, typename S>
__global__ __launch_bounds__(kBlock) void k_energy(const S* __restrict__ G, const S* __restrict__ T,
                                                   int64_t n, double scale,
                                                   unsigned long long* __restrict__ out) {
  constexpr int LG = DP / 4;
  constexpr int IPW = 64 / LG;
  const int lane = threadIdx.x & 63;
  const int sub = lane % LG, slot = lane / LG;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * kBlock) >> 6;
  using Quad = typename Storage<S>::Quad;
  const Quad* __restrict__ G4 = reinterpret_cast<const Quad*>(G);
  const Quad* __restrict__ T4 = reinterpret_cast<const Quad*>(T);
  unsigned long long acc = 0;
  for (int64_t first = wave * IPW; first < n; first += nwaves * IPW) {
    const int64_t p = first + slot;
    const int64_t pc = p < n ? p : 0;
    float v = chunk_sq(Storage<S>::widen4(G4[pc * LG + sub]), Storage<S>::widen4(T4[pc * LG + sub]));
#pragma unroll
    for (int m = 1; m < LG; m <<= 1) v = v + __shfl_xor(v, m);
    if (p < n && sub == 0) acc += static_cast<unsigned long long>(static_cast<double>(v) * scale);
  }
  acc = wave_sum_u64(acc);
  if (lane == 0) atomicAdd(out, acc);
}

// -------------------------------------------------------------------- VAD

// The quality measure of App. C: the population variance of |a - b| over the
// right and down neighbour pairs of the arranged grid, every channel, in
// float64, in two passes (the mean, then the mean squared deviation). Each
// block writes its partial sum; one block adds the partials in a fixed
// order, so the result does not depend on scheduling.
template <typename SI>
__device__ __forceinline__ double feature(const SI* __restrict__ F, int64_t n, int d, int layout, int64_t i,
                                          int c) {
  const SI v = layout == 0 ? F[static_cast<int64_t>(c) * n + i] : F[i * d + c];
  return static_cast<double>(Storage<SI>::widen(v));
}

template <typename SI>
__global__ __launch_bounds__(kBlock) void k_vad_partial(const SI* __restrict__ F, const int32_t* __restrict__ perm,
                                                        int64_t n, int d, int w, int layout, int pass,
                                                        const double* __restrict__ mean_in,
                                                        double* __restrict__ part) {
  __shared__ double s_acc[kBlock];
  const double mean = pass == 0 ? 0.0 : mean_in[0];
  double acc = 0.0;
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int y = static_cast<int>(p / w), x = static_cast<int>(p - static_cast<int64_t>(y) * w);
    const int64_t a = perm != nullptr ? perm[p] : p;
    for (int dir = 0; dir < 2; ++dir) {
      const int yy = y + (dir == 1), xx = x + (dir == 0);
      if (yy >= w || xx >= w) continue;
      const int64_t q = static_cast<int64_t>(yy) * w + xx;
      const int64_t b = perm != nullptr ? perm[q] : q;
      for (int c = 0; c < d; ++c) {
        const double v = fabs(feature(F, n, d, layout, a, c) - feature(F, n, d, layout, b, c));
        acc += pass == 0 ? v : (v - mean) * (v - mean);
      }
    }
  }
  s_acc[threadIdx.x] = acc;
  __syncthreads();
  for (int stride = kBlock / 2; stride > 0; stride >>= 1) {
    if (threadIdx.x < stride) s_acc[threadIdx.x] += s_acc[threadIdx.x + stride];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s_acc[0];
}

// out[0] = sum of part[0 .. nparts) / count (one block of kBlock threads).
__global__ __launch_bounds__(kBlock) void k_vad_finish(const double* __restrict__ part, int nparts, double count,
                                                       double* __restrict__ out) {
  __shared__ double s_acc[kBlock];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kBlock) acc += part[i];
  s_acc[threadIdx.x] = acc;
  __syncthreads();
  for (int stride = kBlock / 2; stride > 0; stride >>= 1) {
    if (threadIdx.x < stride) s_acc[threadIdx.x] += s_acc[threadIdx.x + stride];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s_acc[0] / count;
}

// -------------------------------------------------------------- controller

// The control step after each reorder (Sec. 3.1), applied to a state copy:
// E is compared with the previous energy; an improvement of at least
// ceil(E_prev / M) keeps the level and its block shift; the first stall
// draws a new shift; a stall right after a new shift ends the level
// (phi <- decay * phi, precomputed in `levels`). The block shift number
// st.j, the grouping keys of reorder st.k + 1 and the next level come
// prepared in st.next_* (none depends on E). trace may be NULL.
__device__ void control_step(DevState& st, const LevelInfo* __restrict__ levels,
                             plas_level_out* __restrict__ trace) {
  unsigned long long E = 0, moved = 0;
  for (int i = 0; i < kAccSlots; ++i) {
    E += st.energy_acc[i];
    moved += st.moved_acc[i];
    st.energy_acc[i] = 0;
    st.moved_acc[i] = 0;
  }
  st.blocks_done = 0;
  st.k += 1;
  st.level_reorders += 1;
  st.level_moved += moved;
  st.energy_last = E;
  if (st.level_reorders == 1) st.levels_run += 1;
  const int L = st.level;
  if (trace != nullptr) {
    plas_level_out& tr = trace[L];
    tr.phi = levels[L].phi;
    tr.r = levels[L].r;
    tr.beta = levels[L].beta;
    tr.reorders = st.level_reorders;
    tr.energy_fixed = E;
    tr.moved = st.level_moved;
  }
  const uint64_t M = st.inv_threshold;
  const uint64_t prev = st.energy_prev;
  const bool improved = !st.has_prev || (E < prev && prev - E >= (prev + M - 1) / M);
  if (improved) {
    st.energy_prev = E;
    st.has_prev = 1;
    st.just_shifted = 0;
  } else if (st.just_shifted) {
    const int next = L + 1;
    if (next >= st.nlevels) {
      st.done = 1;
      st.ended = 1;
    } else {
      const LevelInfo lv = st.next_level;
      st.level = next;
      st.r = lv.r;
      st.beta = lv.beta;
      st.nb = lv.nb;
      st.groups_per_block = lv.groups_per_block;
      st.groups = lv.groups;
      st.singles = lv.singles;
      st.dy = st.next_dy;
      st.dx = st.next_dx;
      st.j += 1;
      st.has_prev = 0;
      st.just_shifted = 0;
      st.level_reorders = 0;
      st.level_moved = 0;
    }
  } else {
    st.dy = st.next_dy;
    st.dx = st.next_dx;
    st.j += 1;
    st.just_shifted = 1;
    st.energy_prev = E;
  }
  if (st.max_reorders > 0 && st.k >= st.max_reorders) st.done = 1;
  if (!st.done)
    for (int i = 0; i < 4; ++i) st.keys[i] = st.next_keys[i];
}

// What the control step of the running reorder may need, prepared by one
// thread of the assignment's first block before its items: block shift
// number j, the grouping keys of reorder k + 1, the next level. Written
// with device-scope atomic exchanges, made where every block's atomics meet
// and complete (their results returned) before that thread takes its
// block's ticket, so the last block, which reads the state after every
// ticket, sees them.
__device__ void prepare_step(DevState* __restrict__ st, const LevelInfo* __restrict__ levels) {
  int32_t dy, dx;
  block_shift(st->seed, st->j, st->w, &dy, &dx);
  const Words4 keys = draw(st->seed, kDrawGrouping, static_cast<uint64_t>(st->k + 1));
  __hip_atomic_exchange(&st->next_dy, dy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_exchange(&st->next_dx, dx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int i = 0; i < 4; ++i)
    __hip_atomic_exchange(&st->next_keys[i], keys.v[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int next = st->level + 1;
  if (next < st->nlevels) {
    static_assert(sizeof(LevelInfo) % 4 == 0, "level copied as 32-bit words");
    const uint32_t* src = reinterpret_cast<const uint32_t*>(levels + next);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&st->next_level);
    for (int i = 0; i < static_cast<int>(sizeof(LevelInfo) / 4); ++i)
      __hip_atomic_exchange(dst + i, src[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// The end of a reorder's assignment launch, run by the first wave of every
// block after the block has added its sums to the state (nblocks blocks of
// this sort; the block's other waves have ended). Its first thread takes a
// ticket (an atomic increment, made after the sums were added); the wave
// that draws the last ticket sees every block's sums and runs the control
// step on the state in place: no block of the launch reads the state after
// taking its ticket, and the next launch of the sort starts after this one
// ends. Device-scope fences are not needed and would be costly here (each
// writes back the L2 of its chiplet): the sums, the tickets, the prepared
// values and the last wave's reads are all device-scope atomics.
__device__ void reorder_done(DevState* __restrict__ st, const LevelInfo* __restrict__ levels,
                             plas_level_out* __restrict__ trace, uint32_t nblocks) {
  static_assert(sizeof(DevState) % 4 == 0, "state is copied as 32-bit words");
  constexpr int kWords = sizeof(DevState) / 4;
  __shared__ DevState s_st;
  const int lane = threadIdx.x & 63;
  uint32_t last = 0;
  if (lane == 0)
    last = __hip_atomic_fetch_add(&st->blocks_done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == nblocks - 1
               ? 1u
               : 0u;
  if (__builtin_amdgcn_readfirstlane(last) == 0) return;
  uint32_t* words = reinterpret_cast<uint32_t*>(&s_st);
  uint32_t* gwords = reinterpret_cast<uint32_t*>(st);
  for (int i = lane; i < kWords; i += 64)
    words[i] = __hip_atomic_load(gwords + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  wave_lds_sync();
  if (lane == 0) control_step(s_st, levels, trace);
  wave_lds_sync();
  for (int i = lane; i < kWords; i += 64) gwords[i] = words[i];
}

// ------------------------------------------------------------------ batch
//
// Many independent sorts advance together, one reorder per launch sequence.
// grids[i] holds sort i's buffers and state pair; a launch covers several
// sorts, and its block map gives each block its sort and its index among
// that sort's blocks: map[b] = (grid index << 16) | block index. Every block
// then runs exactly the code of a single-sort launch of that sort's shape,
// so each sort's result does not depend on the batch it runs in.

// The kernels' view of BatchGrid: the same layout, with every pointer
// declared as device (global) memory. Pointers read from memory are
// otherwise generic to the compiler, which then emits flat instructions.
#define PLAS_GLOBAL __attribute__((address_space(1)))
struct BatchGridView {
  void PLAS_GLOBAL* G;
  void PLAS_GLOBAL* H;
  void PLAS_GLOBAL* T;
  int32_t PLAS_GLOBAL* P;
  int32_t PLAS_GLOBAL* table;
  const float PLAS_GLOBAL* inv;
  const LevelInfo PLAS_GLOBAL* levels;
  plas_level_out PLAS_GLOBAL* trace;
  DevState PLAS_GLOBAL* state;
  int32_t w;
  int32_t blur_blocks;
  int32_t assign_blocks;
  int32_t pad;
};
static_assert(sizeof(BatchGridView) == sizeof(BatchGrid), "descriptor view layout");
static_assert(offsetof(BatchGridView, w) == offsetof(BatchGrid, w), "descriptor view layout");

__device__ __forceinline__ const BatchGridView& batch_grid(const BatchGrid* __restrict__ grids,
                                                           const uint32_t* __restrict__ map, uint32_t& local) {
  const uint32_t e = map[blockIdx.x];
  local = e & 0xffffu;
  return reinterpret_cast<const BatchGridView*>(grids)[e >> 16];
}

// A global pointer of the view as a plain pointer of type T (the compiler
// keeps track of where it points).
template <typename T, typename U>
__device__ __forceinline__ T* global_ptr(U PLAS_GLOBAL* p) {
  return (T*)((T PLAS_GLOBAL*)p);
}

// A batch blur pass's route (see launch_blur_batch): its axis, source and
// destination grids (0 G, 1 H, 2 T) and whether it fills the grouping table
// afterwards (the first row pass of a reorder).
__host__ __device__ __forceinline__ int route_vertical(int route) { return route & 1; }
__device__ __forceinline__ bool route_table(int route) { return (route >> 5) & 1; }
template <typename S>
__device__ __forceinline__ S* route_grid(const BatchGridView& g, int sel) {
  return global_ptr<S>(sel == 0 ? g.G : sel == 1 ? g.H : g.T);
}

// Ring rows of the batched staged pass (grids of a batch take whole lines
// by the thousand; the larger ring keeps leaving values on chip up to r = 47).
constexpr int kBatchRingRows = 128;

template <typename S, int DP, int WPB, int KR, bool NT>
__global__ __launch_bounds__(WPB * 64) __attribute__((amdgpu_waves_per_eu(staged_waves_per_eu<S, kBatchRingRows>())))
void k_blur_staged_batch(const BatchGrid* __restrict__ grids, const uint32_t* __restrict__ map, int route) {
  __shared__ RingLds<S, kBatchRingRows> s_stage[WPB];
  uint32_t local;
  const BatchGridView& g = batch_grid(grids, map, local);
  const DevState* st = global_ptr<const DevState>(g.state);
  int r;
  if (!pass_radius(st, 0, r)) return;
  const int vertical = route_vertical(route);
  const S* in = route_grid<S>(g, (route >> 1) & 3);
  S* out = route_grid<S>(g, (route >> 3) & 3);
  blur_staged_lines<S, DP, WPB, kBatchRingRows, KR, NT>(in, out, g.w, r, vertical, local, g.blur_blocks, s_stage);
  if (route_table(route))
    fill_group_table<WPB * 64>(global_ptr<int32_t>(g.table), st->beta, st->keys, local, g.blur_blocks);
}

template <int DP, typename S>
__global__ __launch_bounds__(kBlock) void k_blur_batch(const BatchGrid* __restrict__ grids,
                                                       const uint32_t* __restrict__ map, int route) {
  uint32_t local;
  const BatchGridView& g = batch_grid(grids, map, local);
  const DevState* st = global_ptr<const DevState>(g.state);
  int r;
  if (!pass_radius(st, 0, r)) return;
  const int vertical = route_vertical(route);
  const S* in = route_grid<S>(g, (route >> 1) & 3);
  S* out = route_grid<S>(g, (route >> 3) & 3);
  const int64_t wave = (static_cast<int64_t>(local) * kBlock + threadIdx.x) >> 6;
  blur_reg_lines<DP, S>(in, out, g.w, r, vertical, global_ptr<const float>(g.inv), wave, threadIdx.x & 63);
  if (route_table(route))
    fill_group_table<kBlock>(global_ptr<int32_t>(g.table), st->beta, st->keys, local, g.blur_blocks);
}

// Every block of a sort adds its sums; the last one of the sort runs its
// control step.
template <int DP, typename S>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(assign_waves_per_eu<S, DP>())))
void k_assign_batch(const BatchGrid* __restrict__ grids, const uint32_t* __restrict__ map) {
  uint32_t local;
  const BatchGridView& g = batch_grid(grids, map, local);
  DevState* st = global_ptr<DevState>(g.state);
  if (st->done) return;
  if (local == 0 && threadIdx.x == 0) prepare_step(st, global_ptr<const LevelInfo>(g.levels));
  assign_items<DP, S>(global_ptr<S>(g.G), global_ptr<const S>(g.T), global_ptr<int32_t>(g.P),
                      global_ptr<const int32_t>(g.table), st, local, g.assign_blocks);
  if (threadIdx.x < 64)
    reorder_done(st, global_ptr<const LevelInfo>(g.levels), global_ptr<plas_level_out>(g.trace),
                 static_cast<uint32_t>(g.assign_blocks));
}

// (done, k) of each listed sort's state, for the host's check between
// chunks.
__global__ __launch_bounds__(kBlock) void k_batch_status(const BatchGrid* __restrict__ grids,
                                                         const int32_t* __restrict__ list, int count,
                                                         HostStatus* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= count) return;
  const DevState* st = global_ptr<const DevState>(reinterpret_cast<const BatchGridView*>(grids)[list[i]].state);
  HostStatus hs;
  hs.done = st->done;
  hs.pad = 0;
  hs.k = st->k;
  out[i] = hs;
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t* __restrict__ p, int64_t count, uint32_t value) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < count; i += stride) p[i] = value;
}

__global__ __launch_bounds__(kBlock) void k_inverse_counts(float* __restrict__ inv, int w) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c <= w) inv[c] = c == 0 ? 0.0f : 1.0f / static_cast<float>(c);
}

}  // namespace

// ------------------------------------------------- no-allocation scratch

// The device memory of plas_grid_energy_noalloc: its three grids, the range
// pass scratch, an accumulator and a flag, and the 1/c table. Host code
// must not pass `scratch` itself to a kernel (it names a host-side stand-in):
// noalloc_scratch gives its address on the current device.
static __device__ __align__(256) unsigned char scratch[NoAllocLayout::kBytes];
static_assert(NoAllocLayout::kRangePartBytes == static_cast<size_t>(kRangeBlocks) * 3 * 64 * sizeof(float),
              "range scratch of the widest cell");
static_assert((kNoAllocMaxSide + 1) * sizeof(float) <= 4096, "1/c table");

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_address[kMaxScratchDevices] = {};
}  // namespace

hipError_t noalloc_scratch(int device, void** out) {
  if (out == nullptr || device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_address[device] == nullptr) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_address[device] = ptr;
  }
  *out = g_scratch_address[device];
  return hipSuccess;
}

// --------------------------------------------------------------- launchers

hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t value, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  k_fill_u32<<<blocks_for(count, 1024), kBlock, 0, stream>>>(p, count, value);
  return hipGetLastError();
}

hipError_t launch_inverse_counts(float* inv, int w, hipStream_t stream) {
  if (w < 0) return hipErrorInvalidValue;
  k_inverse_counts<<<(w + kBlock) / kBlock, kBlock, 0, stream>>>(inv, w);
  return hipGetLastError();
}

#define PLAS_DISPATCH_DP(dp, CALL) \
  switch (dp) {                    \
    case 4: { constexpr int DPV = 4; CALL; } break;   \
    case 8: { constexpr int DPV = 8; CALL; } break;   \
    case 16: { constexpr int DPV = 16; CALL; } break; \
    case 32: { constexpr int DPV = 32; CALL; } break; \
    case 64: { constexpr int DPV = 64; CALL; } break; \
    default: return hipErrorInvalidValue;             \
  }

// The body sees SV = the storage element type (float, or uint16_t holding
// bfloat16 bits).
#define PLAS_DISPATCH_STORAGE(storage, ...)                \
  if ((storage) == kStorageF32) {                          \
    using SV = float;                                      \
    __VA_ARGS__;                                           \
  } else if ((storage) == kStorageBF16) {                  \
    using SV = uint16_t;                                   \
    __VA_ARGS__;                                           \
  } else {                                                 \
    return hipErrorInvalidValue;                           \
  }

hipError_t launch_ingest(const void* features, int input_bf16, int64_t n, int d, int layout, int dp, int storage,
                         void* X, hipStream_t stream) {
  if (layout == 0) {
    const int blocks = static_cast<int>((n + 63) / 64);
    PLAS_DISPATCH_STORAGE(storage, {
      if (input_bf16) {
        PLAS_DISPATCH_DP(dp, (k_ingest_cn<DPV, uint16_t, SV><<<blocks, kBlock, 0, stream>>>(
                                 static_cast<const uint16_t*>(features), n, d, static_cast<SV*>(X))));
      } else {
        PLAS_DISPATCH_DP(dp, (k_ingest_cn<DPV, float, SV><<<blocks, kBlock, 0, stream>>>(
                                 static_cast<const float*>(features), n, d, static_cast<SV*>(X))));
      }
    });
  } else {
    const int blocks = blocks_for(n * dp, 65536);
    PLAS_DISPATCH_STORAGE(storage, {
      if (input_bf16) {
        PLAS_DISPATCH_DP(dp, (k_ingest_nc<DPV, uint16_t, SV><<<blocks, kBlock, 0, stream>>>(
                                 static_cast<const uint16_t*>(features), n, d, static_cast<SV*>(X))));
      } else {
        PLAS_DISPATCH_DP(dp, (k_ingest_nc<DPV, float, SV><<<blocks, kBlock, 0, stream>>>(
                                 static_cast<const float*>(features), n, d, static_cast<SV*>(X))));
      }
    });
  }
  return hipGetLastError();
}

size_t range_partial_floats(int dp) { return static_cast<size_t>(kRangeBlocks) * 3 * dp; }

hipError_t launch_range(const void* X, int64_t n, int d, int dp, int storage, float* part, float* out,
                        hipStream_t stream) {
  PLAS_DISPATCH_STORAGE(storage, {
    PLAS_DISPATCH_DP(dp, (k_range_partial<DPV, SV><<<kRangeBlocks, kBlock, 0, stream>>>(
                             static_cast<const SV*>(X), n, part)));
  });
  PLAS_DISPATCH_DP(dp, (k_range_finish<DPV><<<1, 64, 0, stream>>>(part, kRangeBlocks, d, out)));
  return hipGetLastError();
}

hipError_t launch_start_perm(int32_t* P, int64_t n, const uint64_t keys[4], hipStream_t stream) {
  Words4 k;
  for (int i = 0; i < 4; ++i) k.v[i] = keys[i];
  k_start_perm<<<blocks_for(n), kBlock, 0, stream>>>(P, n, k);
  return hipGetLastError();
}

hipError_t launch_check_perm(const int32_t* init, int64_t n, int32_t* counts, int32_t* flag,
                             hipStream_t stream) {
  k_count_perm<<<blocks_for(n), kBlock, 0, stream>>>(init, n, counts, flag);
  k_verify_counts<<<blocks_for(n), kBlock, 0, stream>>>(counts, n, flag);
  return hipGetLastError();
}

hipError_t launch_gather(const void* X, const int32_t* P, void* G, int64_t n, int dp, int storage,
                         hipStream_t stream) {
  const int blocks = blocks_for(n * (dp / 4), 65536);
  PLAS_DISPATCH_STORAGE(storage, {
    PLAS_DISPATCH_DP(dp, (k_gather<DPV, SV><<<blocks, kBlock, 0, stream>>>(static_cast<const SV*>(X), P,
                                                                          static_cast<SV*>(G), n)));
  });
  return hipGetLastError();
}

// A staged pass with ring RR: over a large working set with register slots
// (float32) and, in the column pass, streaming entering loads; else with
// neither.
template <typename S, int DP, int WPB, int RR>
hipError_t staged_launch(int blocks, bool large, int vertical, hipStream_t stream, const S* src, S* dst, int w,
                         const DevState* st, int radius, int32_t* table) {
  constexpr int kR = ring_register_chunks<S, RR>();
  constexpr int kThreads = WPB * 64;
  if (!large)
    k_blur_staged<S, DP, WPB, RR, 0, false><<<blocks, kThreads, 0, stream>>>(src, dst, w, st, radius, vertical, table);
  else if (vertical)
    k_blur_staged<S, DP, WPB, RR, kR, true><<<blocks, kThreads, 0, stream>>>(src, dst, w, st, radius, vertical, table);
  else
    k_blur_staged<S, DP, WPB, RR, kR, false><<<blocks, kThreads, 0, stream>>>(src, dst, w, st, radius, vertical,
                                                                             table);
  return hipGetLastError();
}

// One pass for storage S and DP channels: the staged kernel when cells
// hold whole 16-byte pieces, else the register kernel.
template <typename S, int DP>
hipError_t blur_pass_dp(const void* in, void* out, int w, const DevState* st, int radius, int vertical,
                        const float* inv, hipStream_t stream, const TableArgs& ta) {
  // With the table, also enough blocks to fill it at about one entry per
  // thread (blocks beyond the lines only do that).
  auto with_table = [&](int64_t blocks, int threads) {
    if (ta.table == nullptr) return static_cast<int>(blocks);
    const int64_t need = std::min<int64_t>(1024, (ta.max_cells + threads - 1) / threads);
    return static_cast<int>(std::max<int64_t>(blocks, need));
  };
  if constexpr (staged_cells<S, DP>()) {
    constexpr int kThreads = kBlurWavesPerBlock * 64;
    const int64_t groups = staged_groups<DP>(w);
    const int blocks = with_table((groups + kBlurWavesPerBlock - 1) / kBlurWavesPerBlock, kThreads);
    // The 128-row ring while every wave of the pass fits on the chip at
    // once with it (4 float32 waves per CU), else the 64-row ring (8 per CU);
    // register slots for the leaving values and streaming column loads on
    // grids the Infinity Cache does not hold twice over.
    const bool large = blur_large_working_set(static_cast<int64_t>(w) * w * DP * static_cast<int64_t>(sizeof(S)));
    const S* src = static_cast<const S*>(in);
    S* dst = static_cast<S*>(out);
    if (sizeof(S) == 2 || groups <= kStagedWavesAtLargeRing)
      return staged_launch<S, DP, kBlurWavesPerBlock, 128>(blocks, large, vertical, stream, src, dst, w, st, radius,
                                                           ta.table);
    return staged_launch<S, DP, kBlurWavesPerBlock, 64>(blocks, large, vertical, stream, src, dst, w, st, radius,
                                                        ta.table);
  } else {
    const int blocks = with_table((blur_reg_waves<DP>(w) + kWavesPerBlock - 1) / kWavesPerBlock, kBlock);
    k_blur<DP, S><<<blocks, kBlock, 0, stream>>>(static_cast<const S*>(in), static_cast<S*>(out), w, st, radius,
                                                 vertical, inv, ta.table);
  }
  return hipGetLastError();
}

hipError_t launch_blur_pass(const void* in, void* out, int w, int dp, int storage, const DevState* st,
                            int radius, int vertical, const float* inv, hipStream_t stream, const TableArgs* table) {
  const TableArgs ta = table != nullptr ? *table : TableArgs{};
  PLAS_DISPATCH_STORAGE(storage, {
    PLAS_DISPATCH_DP(dp, return (blur_pass_dp<SV, DPV>(in, out, w, st, radius, vertical, inv, stream, ta)));
  });
  return hipSuccess;
}

hipError_t launch_group_table(int32_t* table, const DevState* st, int64_t max_cells,
                              hipStream_t stream) {
  k_group_table<<<blocks_for(max_cells), kBlock, 0, stream>>>(table, st);
  return hipGetLastError();
}

// Items per wave of the assignment kernel: 64 lanes over DP / C lanes per
// item (C from assign_channels).
inline int64_t assign_items_per_wave(int dp, int storage) {
  const int c = (storage == kStorageBF16 && dp >= 8) ? 8 : 4;
  return 64 / (dp / c);
}

hipError_t launch_assign(void* G, const void* T, int32_t* P, const int32_t* table, DevState* st, int dp,
                         int storage, int64_t max_items, hipStream_t stream, const ControlArgs* control) {
  const int64_t items_per_wave = assign_items_per_wave(dp, storage);
  const int64_t waves = (max_items + items_per_wave - 1) / items_per_wave;
  const int blocks = blocks_for(waves * 64, assign_blocks_cap(storage));
  const ControlArgs ca = control != nullptr ? *control : ControlArgs{};
  const int with_control = control != nullptr ? 1 : 0;
  PLAS_DISPATCH_STORAGE(storage, {
    PLAS_DISPATCH_DP(dp, (k_assign<DPV, SV><<<blocks, kBlock, 0, stream>>>(
                             static_cast<SV*>(G), static_cast<const SV*>(T), P, table, st, ca.levels, ca.trace,
                             with_control)));
  });
  return hipGetLastError();
}

hipError_t launch_energy(const void* G, const void* T, int64_t n, int dp, int storage, int s,
                         unsigned long long* energy_out, hipStream_t stream) {
  const int64_t items_per_wave = 64 / (dp / 4);
  const int64_t waves = (n + items_per_wave - 1) / items_per_wave;
  const int blocks = blocks_for(waves * 64);
  const double scale = ldexp(1.0, s);
  PLAS_DISPATCH_STORAGE(storage, {
    PLAS_DISPATCH_DP(dp, (k_energy<DPV, SV><<<blocks, kBlock, 0, stream>>>(
                             static_cast<const SV*>(G), static_cast<const SV*>(T), n, scale, energy_out)));
  });
  return hipGetLastError();
}

// ---- VAD

size_t vad_partial_doubles() { return kMaxGridBlocks; }

hipError_t launch_vad(const void* features, int input_bf16, const int32_t* perm, int64_t n, int d, int w,
                      int layout, double* part, double* out, hipStream_t stream) {
  const int blocks = blocks_for(n);
  const double count = static_cast<double>(d) * 2.0 * w * (w - 1);
  // out[0]: mean |a - b|; out[1]: the variance.
  for (int pass = 0; pass < 2; ++pass) {
    if (input_bf16)
      k_vad_partial<uint16_t><<<blocks, kBlock, 0, stream>>>(static_cast<const uint16_t*>(features), perm, n, d, w,
                                                             layout, pass, out, part);
    else
      k_vad_partial<float><<<blocks, kBlock, 0, stream>>>(static_cast<const float*>(features), perm, n, d, w,
                                                          layout, pass, out, part);
    k_vad_finish<<<1, kBlock, 0, stream>>>(part, blocks, count, out + pass);
  }
  return hipGetLastError();
}

// ---- batch

bool staged_blur(int dp, int storage) { return dp * (storage == kStorageBF16 ? 2 : 4) >= 16; }

// The second read of a pass's leaving values comes from the 256 MB Infinity
// Cache when the grids in flight are well inside it, and there the register
// slots only add work: measured on float32 sorts, single 4-64 MiB grids ran
// 2-4 % faster without them; single 256 MiB and larger grids, and a batch
// of 64 grids of up to 121 MiB (3 GB together), ran 3-8 % faster with them.
// The same bound decides the column pass's streaming loads.
constexpr int64_t kLargeWorkingSetBytes = int64_t(128) << 20;

bool blur_large_working_set(int64_t working_bytes) { return working_bytes > kLargeWorkingSetBytes; }

int batch_blur_blocks(int w, int dp, int storage, int waves_per_block, int64_t max_cells) {
  int64_t blocks = 0, threads = 0;
  int64_t groups = 0, waves = 0;
  switch (dp) {
    case 4: groups = staged_groups<4>(w); waves = blur_reg_waves<4>(w); break;
    case 8: groups = staged_groups<8>(w); waves = blur_reg_waves<8>(w); break;
    case 16: groups = staged_groups<16>(w); waves = blur_reg_waves<16>(w); break;
    case 32: groups = staged_groups<32>(w); waves = blur_reg_waves<32>(w); break;
    default: groups = staged_groups<64>(w); waves = blur_reg_waves<64>(w); break;
  }
  if (staged_blur(dp, storage)) {
    blocks = (groups + waves_per_block - 1) / waves_per_block;
    threads = 64 * waves_per_block;
  } else {
    blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    threads = kBlock;
  }
  const int64_t need = std::min<int64_t>(1024, (max_cells + threads - 1) / threads);
  return static_cast<int>(std::max(blocks, need));
}

int batch_assign_blocks(int64_t max_items, int dp, int storage, int cap) {
  const int64_t items_per_wave = assign_items_per_wave(dp, storage);
  const int64_t waves = (max_items + items_per_wave - 1) / items_per_wave;
  return blocks_for(waves * 64, cap > 0 ? cap : assign_blocks_cap(storage));
}

int assign_blocks_cap(int storage) {
  (void)storage;
  return PLAS_ASSIGN_MAX_BLOCKS;
}

template <typename S, int DP, int KR, bool NT>
hipError_t blur_batch_staged(const BatchGrid* grids, const uint32_t* map, int blocks, int waves_per_block,
                             int route, hipStream_t stream) {
  switch (waves_per_block) {
    case 1:
      k_blur_staged_batch<S, DP, 1, KR, NT><<<blocks, 64, 0, stream>>>(grids, map, route);
      break;
    case 2:
      k_blur_staged_batch<S, DP, 2, KR, NT><<<blocks, 128, 0, stream>>>(grids, map, route);
      break;
    case 4:
      k_blur_staged_batch<S, DP, 4, KR, NT><<<blocks, 256, 0, stream>>>(grids, map, route);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipSuccess;
}

template <typename S, int DP>
hipError_t blur_batch_dp(const BatchGrid* grids, const uint32_t* map, int blocks, int waves_per_block,
                         int route, int large, hipStream_t stream) {
  if constexpr (staged_cells<S, DP>()) {
    constexpr int kR = ring_register_chunks<S, kBatchRingRows>();
    const hipError_t e =
        large == 0 ? blur_batch_staged<S, DP, 0, false>(grids, map, blocks, waves_per_block, route, stream)
        : route_vertical(route) ? blur_batch_staged<S, DP, kR, true>(grids, map, blocks, waves_per_block, route, stream)
                                : blur_batch_staged<S, DP, kR, false>(grids, map, blocks, waves_per_block, route, stream);
    if (e != hipSuccess) return e;
  } else {
    k_blur_batch<DP, S><<<blocks, kBlock, 0, stream>>>(grids, map, route);
  }
  return hipGetLastError();
}

int blur_route(int vertical, int src, int dst, int with_table) {
  return (vertical & 1) | ((src & 3) << 1) | ((dst & 3) << 3) | ((with_table & 1) << 5);
}

hipError_t launch_blur_batch(const BatchGrid* grids, const uint32_t* map, int blocks, int dp, int storage,
                             int waves_per_block, int route, int large, hipStream_t stream) {
  const int src = (route >> 1) & 3, dst = (route >> 3) & 3;
  if (src > 2 || dst < 1 || dst > 2 || src == dst) return hipErrorInvalidValue;
  PLAS_DISPATCH_STORAGE(storage, {
    PLAS_DISPATCH_DP(dp, return (blur_batch_dp<SV, DPV>(grids, map, blocks, waves_per_block, route, large, stream)));
  });
  return hipSuccess;
}

hipError_t launch_assign_batch(const BatchGrid* grids, const uint32_t* map, int blocks, int dp, int storage,
                               hipStream_t stream) {
  PLAS_DISPATCH_STORAGE(storage, {
    PLAS_DISPATCH_DP(dp, (k_assign_batch<DPV, SV><<<blocks, kBlock, 0, stream>>>(grids, map)));
  });
  return hipGetLastError();
}

hipError_t launch_batch_status(const BatchGrid* grids, const int32_t* list, int count, HostStatus* out,
                               hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  k_batch_status<<<(count + kBlock - 1) / kBlock, kBlock, 0, stream>>>(grids, list, count, out);
  return hipGetLastError();
}

#undef PLAS_DISPATCH_STORAGE
#undef PLAS_DISPATCH_DP

}  // namespace plas
