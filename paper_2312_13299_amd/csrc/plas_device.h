// plas_device.h -- data shared by the PLAS kernels and the host engine.
#pragma once

#include <stdint.h>

namespace plas {

// Number of separate energy accumulators the assignment kernel spreads its
// atomics over (the controller adds them up).
constexpr int kAccSlots = 32;

// One radius level, prepared on the host (Sec. 3.1): real radius phi, blur
// half-width r = floor(phi), block side beta = clamp(r + 1, min_block, w),
// nb = floor(w / beta) blocks per side, floor(beta^2 / 4) groups per block.
struct LevelInfo {
  double phi;
  int32_t r;
  int32_t beta;
  int32_t nb;
  int32_t pad;
  int64_t groups_per_block;
  int64_t groups;   // nb^2 * groups_per_block
  int64_t singles;  // cells in no group: w^2 - (nb*beta)^2 + nb^2 * (beta^2 mod 4)
};

// Device-resident state of one sort. The parameters block is what every
// kernel of a reorder reads; the control block is updated once after each
// reorder, by the last block of its assignment launch to finish.
struct DevState {
  // ---- parameters of the current reorder
  int32_t done;
  int32_t w;
  int32_t r;
  int32_t beta;
  int32_t nb;
  int32_t dy;
  int32_t dx;
  int32_t s;  // energy scale shift
  int64_t groups_per_block;
  int64_t groups;
  int64_t singles;
  uint64_t keys[4];  // round keys of the grouping bijection
  // ---- written by the assignment kernel
  unsigned long long energy_acc[kAccSlots];
  unsigned long long moved_acc[kAccSlots];
  // ---- control
  int32_t level;
  int32_t nlevels;
  int32_t has_prev;
  int32_t just_shifted;
  int32_t levels_run;
  uint32_t inv_threshold;
  uint32_t blocks_done;  // assignment blocks of the running reorder that have added their sums
  int32_t ended;    // the schedule ended (done for another reason: max_reorders)
  int64_t k;  // reorders done
  int64_t max_reorders;
  int64_t level_reorders;
  uint64_t j;  // shift draws done
  uint64_t seed;
  uint64_t energy_prev;
  uint64_t energy_last;
  uint64_t level_moved;
  // ---- prepared during a reorder's assignment for its control step (by
  // the first block, so that the last block's step draws nothing and reads
  // no table): block shift number j, the grouping keys of reorder k + 1 and
  // the next level's parameters (unset at the last level)
  int32_t next_dy;
  int32_t next_dx;
  uint64_t next_keys[4];
  LevelInfo next_level;
};

// Small status block copied to pinned host memory at each sync.
struct HostStatus {
  int32_t done;
  int32_t pad;
  int64_t k;
};

struct plas_level_out;

// One sort of a batch: its buffers, its state, and how many blocks of each
// launch kind it takes. Grids G, H, T are [w*w][dp] in the batch's
// storage.
struct BatchGrid {
  void* G;
  void* H;
  void* T;
  int32_t* P;
  int32_t* table;
  const float* inv;
  const LevelInfo* levels;
  plas_level_out* trace;
  DevState* state;
  int32_t w;
  int32_t blur_blocks;
  int32_t assign_blocks;
  int32_t pad;
};

}  // namespace plas
