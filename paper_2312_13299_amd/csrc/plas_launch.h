// plas_launch.h -- host-side launchers of the PLAS kernels (plas_kernels.hip).
// Each enqueues work on `stream` and returns the launch status; none
// synchronises. `dp` is the padded channel stride of the working layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plas_device.h"

namespace plas {

struct plas_level_out {  // same layout as plas_level_stat in plas.h
  double phi;
  int32_t r;
  int32_t beta;
  int64_t reorders;
  uint64_t energy_fixed;
  uint64_t moved;
};

// Storage of the working grids.
constexpr int kStorageF32 = 0;
constexpr int kStorageBF16 = 1;

// features (layout CN [d][n] or NC [n][d]; float32, or bfloat16 bits if
// input_bf16) -> X [n][dp] in `storage`, channels >= d zero.
hipError_t launch_ingest(const void* features, int input_bf16, int64_t n, int d, int layout, int dp, int storage,
                         void* X, hipStream_t stream);
// Per-channel min/max of X[n][dp] over the first d channels, and a flag set
// if any value is NaN or infinite. out: [dp] mins, [dp] maxs, then the flag
// (as a float slot holding 0 or 1). part: scratch of range_partial_floats().
size_t range_partial_floats(int dp);
hipError_t launch_range(const void* X, int64_t n, int d, int dp, int storage, float* part, float* out,
                        hipStream_t stream);
// P[p] = bijection(n, keys)(p).
hipError_t launch_start_perm(int32_t* P, int64_t n, const uint64_t keys[4], hipStream_t stream);
// Check that init (int32[n]) is a bijection of [0, n): counts is scratch
// int32[n], flag (device int32) is set to 1 when it is not. counts and flag
// must be zeroed beforehand.
hipError_t launch_check_perm(const int32_t* init, int64_t n, int32_t* counts, int32_t* flag,
                             hipStream_t stream);
// G[p] = X[P[p]] over dp channels (P NULL: identity).
hipError_t launch_gather(const void* X, const int32_t* P, void* G, int64_t n, int dp, int storage,
                         hipStream_t stream);
// The grouping table a reorder's first row pass fills after its lines, from
// the state's beta and keys.
struct TableArgs {
  int32_t* table;
  int64_t max_cells;  // largest beta^2 of the sort: the pass launches enough blocks to fill it quickly
};

// One blur pass (vertical = 0: rows, 1: columns) with radius st->r, or
// `radius` if st is NULL (a pass queued after the end of the sort returns at
// once). inv: float32 1/c for c = 0..w (the register kernel's multipliers).
hipError_t launch_blur_pass(const void* in, void* out, int w, int dp, int storage, const DevState* st,
                            int radius, int vertical, const float* inv, hipStream_t stream,
                            const TableArgs* table = nullptr);
// Grouping table of the current reorder: table[t] = packed pi(t), t < beta^2.
hipError_t launch_group_table(int32_t* table, const DevState* st, int64_t max_cells,
                              hipStream_t stream);
// What the control step at the end of a sort's assignment needs: the level
// table and the per-level trace (may be NULL).
struct ControlArgs {
  const LevelInfo* levels;
  plas_level_out* trace;
};

// One blockwise assignment with the parameters in st. max_items bounds
// groups + singles over every level this launch may see. With `control`,
// the last block to finish runs the control step of the reorder on st in
// place (the energy and moved sums, the stall test, the schedule, the next
// shift and grouping keys); without it, st keeps the sums for the caller.
hipError_t launch_assign(void* G, const void* T, int32_t* P, const int32_t* table, DevState* st, int dp,
                         int storage, int64_t max_items, hipStream_t stream, const ControlArgs* control = nullptr);
// VAD (App. C) of features[perm] on a w x w grid: out[0] receives the mean
// |a - b| over neighbour pairs and channels, out[1] the variance. part:
// device scratch of vad_partial_doubles() doubles; out: device double[2].
size_t vad_partial_doubles();
hipError_t launch_vad(const void* features, int input_bf16, const int32_t* perm, int64_t n, int d, int w,
                      int layout, double* part, double* out, hipStream_t stream);

// ---- batches of sorts (BatchGrid in plas_device.h). A launch's block map
// (device uint32[blocks]) holds (grid index << 16) | block index within the
// grid's blocks; a grid's entries run from 0 to its block count - 1.
// Blocks each grid takes per launch kind.
// Whether blur passes of this shape use the staged kernel (cells of at
// least 16 bytes); waves_per_block applies to those only.
bool staged_blur(int dp, int storage);
// Whether the grids in flight (the one grid of a sort, every running grid
// of a batch) are a large working set, more than 128 MiB: then staged
// float32 passes keep the leaving values in registers rather than reading
// them a second time, and column passes stream their loads.
bool blur_large_working_set(int64_t working_bytes);
// Blur blocks: enough for every line, and for filling a grouping table of
// max_cells entries at about one entry per thread.
int batch_blur_blocks(int w, int dp, int storage, int waves_per_block, int64_t max_cells);  // wpb: 1, 2, 4
int batch_assign_blocks(int64_t max_items, int dp, int storage, int cap);  // cap <= 0: the single-sort default
int assign_blocks_cap(int storage);  // blocks of an assignment launch without a tuned value
// A batch blur pass's route: its axis (vertical 0: rows, 1: columns), its
// source and destination grids (0 G, 1 H, 2 T; the destination H or T, not
// the source) and whether it fills each grid's grouping table after its
// lines (the first row pass of a reorder).
int blur_route(int vertical, int src, int dst, int with_table);
// One blur pass along `route` of every mapped grid, all of dp channels and
// `storage`; large: blur_large_working_set holds for the running grids.
hipError_t launch_blur_batch(const BatchGrid* grids, const uint32_t* map, int blocks, int dp, int storage,
                             int waves_per_block, int route, int large, hipStream_t stream);
// One assignment of every mapped grid; each grid's last block runs its
// control step.
hipError_t launch_assign_batch(const BatchGrid* grids, const uint32_t* map, int blocks, int dp, int storage,
                               hipStream_t stream);
// out[i] = (done, k) of grids[list[i]]'s state, i < count.
hipError_t launch_batch_status(const BatchGrid* grids, const int32_t* list, int count, HostStatus* out,
                               hipStream_t stream);

// energy_out (device u64) += sum over cells of floor(d(G[p], T[p]) * 2^s).
hipError_t launch_energy(const void* G, const void* T, int64_t n, int dp, int storage, int s,
                         unsigned long long* energy_out, hipStream_t stream);

// p[i] = value for i < count (a kernel, not a memset: callers may capture the
// stream in a graph).
hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t value, hipStream_t stream);
// inv[c] = float32 1/c (correctly rounded) for c = 1..w, inv[0] = 0.
hipError_t launch_inverse_counts(float* inv, int w, hipStream_t stream);

// ---- the device scratch of the no-allocation energy query. One array per
// GPU, allocated with the code object and held until the process ends;
// every call on a GPU shares it.
constexpr int64_t kNoAllocMaxCells = 65536;  // side <= 256
constexpr int kNoAllocMaxSide = 256;
struct NoAllocLayout {
  static constexpr size_t kGrid = static_cast<size_t>(kNoAllocMaxCells) * 64 * 4;  // widest cell, float32
  static constexpr size_t kG = 0, kH = kGrid, kT = 2 * kGrid;
  static constexpr size_t kRangePart = 3 * kGrid;
  static constexpr size_t kRangePartBytes = 256 * 3 * 64 * 4;  // range_partial_floats(64) floats
  static constexpr size_t kRangeOut = kRangePart + kRangePartBytes;
  static constexpr size_t kFlags = kRangeOut + 1024;  // u64 accumulator, then an int32 flag
  static constexpr size_t kInv = kFlags + 256;
  static constexpr size_t kBytes = kInv + 4096;  // (kNoAllocMaxSide + 1) floats, rounded up
};
// The array's device address on `device`, which must be current (looked up
// once per device, then remembered).
hipError_t noalloc_scratch(int device, void** out);

}  // namespace plas
