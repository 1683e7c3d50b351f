// plas_host.h -- host-side internals of libplas.so shared by the single-sort
// engine (plas_engine.cpp) and the batch engine (plas_batch.cpp): the
// context, device buffers, argument checks, feature preparation and the
// radius schedule. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "plas.h"
#include "plas_device.h"
#include "plas_launch.h"
#include "plas_random.h"

using plas::DevState;
using plas::HostStatus;
using plas::LevelInfo;
using plas::plas_level_out;

struct plas_batch_state;

namespace plas_host {

constexpr int kDefaultReordersPerSync = 32;
// With profiling, every kProfileEvery-th reorder slot of a chunk is timed
// (three events: before the blur passes, between them and the assignment,
// after it). A HIP event record between two launches costs about 5 us of
// device time: timing every reorder slows the sort it measures by ~4 %,
// every 32nd by ~0.15 %.
constexpr int kProfileEvery = 32;

struct DeviceBuffer {
  void* ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace plas_host

struct plas_context {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string error;
  // Device workspace, grown on demand and kept.
  plas_host::DeviceBuffer grid_g, grid_h, grid_t;  // [n][dp] each, float32 or bfloat16
  plas_host::DeviceBuffer perm;                    // int32[n]
  plas_host::DeviceBuffer table;                   // int32[beta^2]
  plas_host::DeviceBuffer inv;                     // float32 1/c, c = 0..w
  plas_host::DeviceBuffer range_part, range_out;   // range pass scratch and result
  plas_host::DeviceBuffer levels;                  // LevelInfo[levels]
  plas_host::DeviceBuffer trace;                   // plas_level_out[levels]
  plas_host::DeviceBuffer state;                   // DevState of a sort
  plas_host::DeviceBuffer stage_state;             // DevState of a stage call
  plas_host::DeviceBuffer scratch;                 // u64 accumulators and flags
  plas_host::DeviceBuffer vad;                     // VAD partial sums and results
  void* noalloc = nullptr;                         // the device's scratch of plas_grid_energy_noalloc
  // Pinned host memory for small read-backs.
  HostStatus* status_host = nullptr;
  float* range_host = nullptr;
  unsigned long long* u64_host = nullptr;
  DevState* state_host = nullptr;
  std::vector<hipEvent_t> events;
  // Batch engine resources (plas_batch.cpp), created on first use.
  plas_batch_state* batch = nullptr;
};

// Frees h->batch (defined in plas_batch.cpp).
void release_batch_state(plas_context* h);

namespace plas_host {

// ---------------------------------------------------------------- helpers

inline int32_t fail(plas_context* h, int32_t status, const std::string& msg) {
  if (h != nullptr) h->error = msg;
  return status;
}

inline int32_t hip_fail(plas_context* h, hipError_t e, const char* what) {
  std::string msg = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(h, PLAS_ERR_OUT_OF_MEMORY, msg);
  return fail(h, PLAS_ERR_HIP, msg);
}

#define PLAS_HIP(h, call)                                  \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hip_fail((h), e_, #call); \
  } while (0)

// Keeps the caller's current device and restores it on exit.
class DeviceScope {
 public:
  explicit DeviceScope(int device) {
    if (hipGetDevice(&saved_) != hipSuccess) saved_ = -1;
    ok_ = hipSetDevice(device) == hipSuccess;
  }
  ~DeviceScope() {
    if (saved_ >= 0) (void)hipSetDevice(saved_);
  }
  bool ok() const { return ok_; }

 private:
  int saved_ = -1;
  bool ok_ = false;
};

inline hipError_t reserve(DeviceBuffer& b, size_t bytes) {
  if (bytes <= b.bytes && b.ptr != nullptr) return hipSuccess;
  if (b.ptr != nullptr) {
    hipError_t e = hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipMalloc(&b.ptr, bytes);
  if (e != hipSuccess) {
    b.ptr = nullptr;
    return e;
  }
  b.bytes = bytes;
  return hipSuccess;
}

inline void release(DeviceBuffer& b) {
  if (b.ptr != nullptr) (void)hipFree(b.ptr);
  b.ptr = nullptr;
  b.bytes = 0;
}

template <typename T>
inline T* as(DeviceBuffer& b) {
  return static_cast<T*>(b.ptr);
}

inline size_t storage_bytes(int32_t storage) { return storage == PLAS_STORAGE_BF16 ? 2 : 4; }

inline bool valid_storage(int32_t storage) { return storage == PLAS_STORAGE_F32 || storage == PLAS_STORAGE_BF16; }

inline int padded_channels(int d) {
  int dp = 4;
  while (dp < d) dp *= 2;
  return dp;
}

// The radius schedule of Sec. 3.1 with the block geometry of each level.
inline int32_t build_schedule(int32_t w, double decay, int32_t min_block, double start_radius,
                       std::vector<LevelInfo>* out) {
  if (w < 1 || !(decay > 0.0 && decay < 1.0) || min_block < 1) return PLAS_ERR_INVALID_ARGUMENT;
  double phi = start_radius > 0.0 ? start_radius : static_cast<double>(w) / 2.0 - 1.0;
  if (!(phi >= 1.0)) phi = 1.0;  // also catches NaN
  out->clear();
  while (phi >= 1.0) {
    LevelInfo lv{};
    lv.phi = phi;
    // r beyond w - 1 blurs whole lines; the cap only keeps x + r in range.
    const double rf = std::floor(phi);
    lv.r = rf > 1073741824.0 ? 1073741824 : static_cast<int32_t>(rf);
    lv.beta = std::min(w, std::max(min_block, lv.r + 1));
    lv.nb = w / lv.beta;
    const int64_t cells = static_cast<int64_t>(lv.beta) * lv.beta;
    lv.groups_per_block = cells / 4;
    lv.groups = static_cast<int64_t>(lv.nb) * lv.nb * lv.groups_per_block;
    const int64_t covered = static_cast<int64_t>(lv.nb) * lv.beta;
    lv.singles = static_cast<int64_t>(w) * w - covered * covered +
                 static_cast<int64_t>(lv.nb) * lv.nb * (cells % 4);
    out->push_back(lv);
    phi = phi * decay;
  }
  return PLAS_OK;
}

inline int32_t scale_shift(const float* mins, const float* maxs, int32_t d, int64_t n) {
  double dmax = 0.0;
  for (int32_t c = 0; c < d; ++c) {
    const double span = static_cast<double>(maxs[c]) - static_cast<double>(mins[c]);
    dmax += span * span;
  }
  if (!(dmax > 0.0)) return 0;
  int e = 0;
  (void)std::frexp(static_cast<double>(n) * dmax, &e);
  return 61 - e;
}

inline bool valid_layout(int32_t layout) { return layout == PLAS_LAYOUT_CN || layout == PLAS_LAYOUT_NC; }

// Shared argument checks of plas_sort and plas_grid_energy.
inline int32_t check_features(plas_context* h, const void* features, int64_t n, int32_t d, int32_t side,
                       int32_t layout, int32_t dtype) {
  if (h == nullptr) return PLAS_ERR_INVALID_ARGUMENT;
  if (features == nullptr) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "features is NULL");
  if (side < 2 || side > 46340) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "side must be in [2, 46340]");
  if (n != static_cast<int64_t>(side) * side)
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "n must equal side * side");
  if (d < 1) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "d must be >= 1");
  if (!valid_layout(layout)) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "unknown layout");
  if (dtype != PLAS_DTYPE_F32 && dtype != PLAS_DTYPE_BF16) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "unknown dtype");
  if (d > PLAS_MAX_CHANNELS)
    return fail(h, PLAS_ERR_UNSUPPORTED, "d above PLAS_MAX_CHANNELS is not supported");
  return PLAS_OK;
}

// Ingest + range + scale shift into X (device [n][dp] in `storage`, cell-major
// padded features). Returns NONFINITE if a value is not finite.
inline int32_t ingest_features(plas_context* h, const void* features, int32_t dtype, int64_t n, int32_t d,
                               int32_t layout, int dp, int32_t storage, void* X, int32_t* s_out) {
  PLAS_HIP(h, reserve(h->range_part, plas::range_partial_floats(dp) * sizeof(float)));
  PLAS_HIP(h, reserve(h->range_out, (2 * 64 + 1) * sizeof(float)));
  PLAS_HIP(h, plas::launch_ingest(features, dtype == PLAS_DTYPE_BF16, n, d, layout, dp, storage, X, h->stream));
  PLAS_HIP(h, plas::launch_range(X, n, d, dp, storage, as<float>(h->range_part), as<float>(h->range_out),
                                 h->stream));
  PLAS_HIP(h, hipMemcpyAsync(h->range_host, h->range_out.ptr, (2 * dp + 1) * sizeof(float),
                             hipMemcpyDeviceToHost, h->stream));
  PLAS_HIP(h, hipStreamSynchronize(h->stream));
  if (h->range_host[2 * dp] != 0.0f)
    return fail(h, PLAS_ERR_NONFINITE, "features contain NaN or infinity");
  *s_out = scale_shift(h->range_host, h->range_host + dp, d, n);
  return PLAS_OK;
}

// The context's three working grids, with X in grid_t.
inline int32_t prepare_features(plas_context* h, const void* features, int32_t dtype, int64_t n, int32_t d,
                                int32_t layout, int dp, int32_t storage, int32_t* s_out) {
  const size_t grid_bytes = static_cast<size_t>(n) * dp * storage_bytes(storage);
  PLAS_HIP(h, reserve(h->grid_g, grid_bytes));
  PLAS_HIP(h, reserve(h->grid_h, grid_bytes));
  PLAS_HIP(h, reserve(h->grid_t, grid_bytes));
  return ingest_features(h, features, dtype, n, d, layout, dp, storage, h->grid_t.ptr, s_out);
}

// Validate a caller permutation (device int32[n]); counts: device scratch of
// n int32.
inline int32_t check_permutation(plas_context* h, const int32_t* perm, int64_t n, int32_t* counts) {
  int32_t* flag = reinterpret_cast<int32_t*>(as<unsigned long long>(h->scratch) + 8);
  PLAS_HIP(h, hipMemsetAsync(counts, 0, static_cast<size_t>(n) * sizeof(int32_t), h->stream));
  PLAS_HIP(h, hipMemsetAsync(flag, 0, sizeof(int32_t), h->stream));
  PLAS_HIP(h, plas::launch_check_perm(perm, n, counts, flag, h->stream));
  PLAS_HIP(h, hipMemcpyAsync(h->u64_host, flag, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
  PLAS_HIP(h, hipStreamSynchronize(h->stream));
  int32_t bad = 0;
  std::memcpy(&bad, h->u64_host, sizeof(int32_t));
  if (bad != 0) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "permutation is not a bijection of [0, n)");
  return PLAS_OK;
}

// float32 1/c for c = 0..w (0 for c = 0), correctly rounded.
inline std::vector<float> inverse_counts(int32_t w) {
  std::vector<float> inv(static_cast<size_t>(w) + 1);
  inv[0] = 0.0f;
  for (int32_t c = 1; c <= w; ++c) inv[c] = 1.0f / static_cast<float>(c);
  return inv;
}

inline int32_t upload_inverse_counts(plas_context* h, int32_t w) {
  PLAS_HIP(h, reserve(h->inv, static_cast<size_t>(w + 1) * sizeof(float)));
  const std::vector<float> inv = inverse_counts(w);
  PLAS_HIP(h, hipMemcpyAsync(h->inv.ptr, inv.data(), inv.size() * sizeof(float), hipMemcpyHostToDevice,
                             h->stream));
  // The source vector dies at return; make the copy complete first.
  PLAS_HIP(h, hipStreamSynchronize(h->stream));
  return PLAS_OK;
}

inline int32_t ensure_events(plas_context* h, size_t count) {
  while (h->events.size() < count) {
    hipEvent_t e;
    PLAS_HIP(h, hipEventCreate(&e));
    h->events.push_back(e);
  }
  return PLAS_OK;
}

inline void fill_state_for_level(DevState* s, const LevelInfo& lv) {
  s->r = lv.r;
  s->beta = lv.beta;
  s->nb = lv.nb;
  s->groups_per_block = lv.groups_per_block;
  s->groups = lv.groups;
  s->singles = lv.singles;
}

// The state before a sort's first reorder: level 0 with its block shift
// (draw (seed, 2, 0)) and the grouping keys of reorder 0 (draw (seed, 1, 0)).
inline void init_sort_state(DevState* S, int32_t w, int32_t s, const std::vector<LevelInfo>& levels,
                            const plas_sort_params& prm, uint64_t seed) {
  std::memset(S, 0, sizeof(DevState));
  S->w = w;
  S->s = s;
  fill_state_for_level(S, levels[0]);
  S->nlevels = static_cast<int32_t>(levels.size());
  S->inv_threshold = prm.inv_threshold;
  S->max_reorders = prm.max_reorders;
  S->seed = seed;
  plas::block_shift(seed, 0, w, &S->dy, &S->dx);
  S->j = 1;
  const plas::Words4 keys = plas::draw(seed, plas::kDrawGrouping, 0);
  for (int i = 0; i < 4; ++i) S->keys[i] = keys.v[i];
}

// The checkpoint of a sort's final state S (schedule of nlevels levels). The
// device counts a level in levels_run from its first reorder; the checkpoint
// counts the levels before the current one.
inline void fill_checkpoint(const DevState& S, int32_t nlevels, plas_sort_checkpoint* ck) {
  std::memset(ck, 0, sizeof(*ck));
  ck->struct_size = sizeof(plas_sort_checkpoint);
  ck->done = S.ended;
  ck->reorders = S.k;
  ck->shift_draws = S.j;
  ck->level = S.ended ? nlevels : S.level;
  ck->levels_done = S.levels_run - (!S.ended && S.level_reorders > 0 ? 1 : 0);
  ck->dy = S.dy;
  ck->dx = S.dx;
  ck->has_prev = S.has_prev;
  ck->just_shifted = S.just_shifted;
  ck->energy_prev = S.energy_prev;
  ck->energy_last = S.energy_last;
  ck->level_reorders = S.level_reorders;
  ck->level_moved = S.level_moved;
}

// Set up S (made by init_sort_state) to continue from a checkpoint.
inline int32_t apply_checkpoint(plas_context* h, DevState* S, const plas_sort_checkpoint& ck,
                                const std::vector<LevelInfo>& levels) {
  const int32_t nlevels = static_cast<int32_t>(levels.size());
  if (ck.struct_size != sizeof(plas_sort_checkpoint))
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "resume->struct_size does not match this library");
  if (ck.reorders < 0 || ck.levels_done < 0 || ck.level_reorders < 0 || ck.level < 0 ||
      (ck.done ? ck.level != nlevels : ck.level >= nlevels) || ck.levels_done > ck.level ||
      ck.dy < 0 || ck.dy >= S->w || ck.dx < 0 || ck.dx >= S->w)
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "resume does not fit this sort's schedule");
  if (!ck.done) fill_state_for_level(S, levels[ck.level]);
  S->level = ck.done ? nlevels - 1 : ck.level;
  S->k = ck.reorders;
  S->j = ck.shift_draws;
  S->levels_run = ck.levels_done + (!ck.done && ck.level_reorders > 0 ? 1 : 0);
  S->dy = ck.dy;
  S->dx = ck.dx;
  S->has_prev = ck.has_prev != 0;
  S->just_shifted = ck.just_shifted != 0;
  S->energy_prev = ck.energy_prev;
  S->energy_last = ck.energy_last;
  S->level_reorders = ck.level_reorders;
  S->level_moved = ck.level_moved;
  S->blocks_done = 0;
  S->ended = ck.done != 0;
  S->done = S->ended || (S->max_reorders > 0 && S->k >= S->max_reorders);
  const plas::Words4 keys = plas::draw(S->seed, plas::kDrawGrouping, static_cast<uint64_t>(S->k));
  for (int i = 0; i < 4; ++i) S->keys[i] = keys.v[i];
  return PLAS_OK;
}

// Shared checks of the sort parameters (plas_sort and plas_sort_batch).
inline int32_t check_params(plas_context* h, const plas_sort_params* params, plas_sort_params* prm) {
  plas_sort_params_init(prm);
  if (params != nullptr) {
    if (params->struct_size != sizeof(plas_sort_params))
      return fail(h, PLAS_ERR_INVALID_ARGUMENT, "params->struct_size does not match this library");
    *prm = *params;
  }
  if (!(prm->radius_decay > 0.0 && prm->radius_decay < 1.0))
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "radius_decay must be in (0, 1)");
  if (prm->inv_threshold < 1) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "inv_threshold must be >= 1");
  if (prm->min_block < 1) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "min_block must be >= 1");
  if (prm->max_reorders < 0) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "max_reorders must be >= 0");
  if (!valid_storage(prm->storage)) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "unknown storage");
  if (prm->filter != PLAS_FILTER_BOX && prm->filter != PLAS_FILTER_BOX3)
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "unknown filter");
  if (prm->resume != nullptr && prm->init_perm == nullptr)
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "resume needs init_perm (the stopped sort's permutation)");
  return PLAS_OK;
}

// Improvements per level are at most about M * ln(2^62) (each one lowers the
// energy by at least 1/M of it); two stalls end a level.
inline int64_t reorder_bound(size_t levels, uint32_t inv_threshold) {
  return static_cast<int64_t>(levels) * (static_cast<int64_t>(inv_threshold) * 44 + 3);
}

inline double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace plas_host

