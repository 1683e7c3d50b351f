/*
 * plas_stages.h -- the individual steps of one PLAS reorder, exported so that
 * each kernel can be driven and checked on its own, plus the library's
 * host-side helpers (random draws, schedule, energy scale).
 *
 * Working layout of a grid: device [n][dp], n = side^2, cell-major, dp a
 * power of two in {4, 8, 16, 32, 64} (channels padded with zeros; the
 * library uses dp = max(4, next power of two >= d)), elements float32
 * (storage PLAS_STORAGE_F32) or bfloat16 bit patterns (PLAS_STORAGE_BF16).
 * Pointers called device pointers are caller-owned device memory of the
 * handle's device. Status codes and threading rules are those of plas.h.
 * Every call returns after its work has finished on the handle's stream.
 */
#ifndef PLAS_STAGES_H
#define PLAS_STAGES_H

#include <stdint.h>

#include "plas.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Target of Sec. 3.1: the grid low-pass filtered by a box of half-width
 * `radius` (>= 0), rows then columns; each window is clipped to the grid and
 * the sum is taken as a sliding sum along the line (add the entering value,
 * then subtract the leaving one) times float32(1/count). radius 0 copies.
 * grid, target: device [n][dp] grids in `storage`; they must not overlap.
 */
int32_t plas_stage_blur(plas_handle h, const void* grid, void* target, int32_t side, int32_t dp,
                        int32_t storage, int32_t radius);

/*
 * The shared grouping of one reorder (Sec. 3.1, "Blockwise Linear
 * Assignment"): table[t] = pi(t) for t < beta^2, pi the keyed bijection of
 * [0, beta^2) (4-round Feistel, cycle walking) under round_keys, stored as
 * (ly << 16) | lx with pi(t) = ly * beta + lx. table: device int32[beta^2].
 * 1 <= beta <= 65535.
 */
int32_t plas_stage_group_table(plas_handle h, int32_t beta, const uint64_t round_keys[4],
                               int32_t* table);

/*
 * One blockwise linear assignment (Sec. 3.1; Fig. "swapping_pixels"): the
 * grid rolled by (dy, dx) is cut into floor(side/beta)^2 blocks; group g of
 * every block holds the block-local cells pi(4g..4g+3); each group moves its
 * four cells by the permutation of least integer cost
 * sum_i floor(d(grid[c_i], target[c_sigma(i)]) * 2^scale_shift) (first in
 * lexicographic order on ties). grid (device [n][dp] in `storage`) and perm
 * (device int32[n]) are updated in place; target is read only. energy (host,
 * may be NULL) receives the integer energy of the new arrangement against
 * target over all cells; moved (host, may be NULL) the cells that moved.
 * 2 <= beta <= side, 0 <= dy, dx < side.
 */
int32_t plas_stage_assign(plas_handle h, void* grid, const void* target, int32_t* perm,
                          int32_t side, int32_t dp, int32_t storage, int32_t beta, int32_t dy,
                          int32_t dx, const uint64_t round_keys[4], int32_t scale_shift,
                          uint64_t* energy, uint64_t* moved);

/* Integer energy of grid against target: sum over cells of
 * floor(d(grid[p], target[p]) * 2^scale_shift). Both device [n][dp] in `storage`. */
int32_t plas_stage_energy(plas_handle h, const void* grid, const void* target, int32_t side,
                          int32_t dp, int32_t storage, int32_t scale_shift, uint64_t* energy);

/* out[i] = pi(i) for i < n, pi the keyed bijection of [0, n) (the random
 * start arrangement of Sec. 3.1 uses the keys of draw (seed, 0, 0)).
 * out: device int32[n], 1 <= n <= 2^31 - 1. */
int32_t plas_stage_bijection(plas_handle h, int64_t n, const uint64_t round_keys[4],
                             int32_t* out);

/* ---- host-side helpers (no device work) ---- */

/* Philox4x64-10 block (Salmon et al., SC'11) computed on the host. */
void plas_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* The library's draw (seed, purpose, index): Philox with counter
 * (purpose, index, 0, 0) and key (seed, 0). Purposes: 0 start arrangement,
 * 1 grouping of reorder k, 2 block shift j. */
void plas_draw(uint64_t seed, uint64_t purpose, uint64_t index, uint64_t out[4]);

/* The radius schedule of Sec. 3.1 for a grid of `side`: fills up to cap
 * levels (phi, r, beta; any pointer may be NULL) and returns the number of
 * levels, or a negative status. */
int32_t plas_schedule(int32_t side, double decay, int32_t min_block, double start_radius,
                      double* phi, int32_t* r, int32_t* beta, int32_t cap);

/* Energy scale from per-channel ranges: D_max = sum_c (max_c - min_c)^2 in
 * float64 (channels in order); s = 61 - e where n * D_max = m * 2^e,
 * m in [0.5, 1); s = 0 if D_max = 0. */
int32_t plas_scale_shift_from_ranges(const float* mins, const float* maxs, int32_t d, int64_t n,
                                     int32_t* scale_shift);

#ifdef __cplusplus
}
#endif
#endif
