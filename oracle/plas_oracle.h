/*
 * plas_oracle.h -- reference CPU implementation of Parallel Linear Assignment
 * Sorting (PLAS), the sort of Sec. 3.1 of "Compact 3D Scene Representation via
 * Self-Organizing Gaussian Grids" (arXiv 2312.13299).
 *
 * TEST INFRASTRUCTURE ONLY. This library exists to check the GPU library.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it. It shares no code with the GPU library.
 *
 * Parity: every function here is pinned by tests against the mathematics
 * (closed forms, brute force, a library Philox, invariants); see each
 * function's comment. Nothing in this file is "parity unpinned" except where
 * a comment says so.
 *
 * Conventions.
 *  - A grid of side w holds N = w*w cells; cell p = y*w + x (row-major).
 *  - Feature matrices are float32, either channel-major ("CN", [d][n]) or
 *    cell-major ("NC", [n][d]). The oracle's working grid is always [N][d].
 *  - A permutation is in gather form: perm[p] is the index of the Gaussian
 *    that sits at cell p, so the arranged grid is features[perm].
 */
#ifndef PLAS_ORACLE_H
#define PLAS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PLAS_REF_OK 0
#define PLAS_REF_INVALID (-1)
#define PLAS_REF_NONFINITE (-5)
#define PLAS_REF_MAX_D 256

#define PLAS_REF_LAYOUT_CN 0
#define PLAS_REF_LAYOUT_NC 1

/* Where a sort stopped (at max_reorders, before the next reorder), so that
 * a later call can resume it: with this state and the stopped call's
 * permutation as init_perm, the resumed sort ends with the permutation,
 * reorder count, energy and trace of the uninterrupted one. */
typedef struct {
    int64_t k;               /* reorders done */
    uint64_t j;              /* shift draws done */
    int32_t level;           /* schedule levels entered (phi = phi0 * decay^level) */
    int32_t levels_run;      /* levels finished that ran a reorder (the current one excluded) */
    int32_t dy, dx;          /* the current level's block shift */
    int32_t has_prev;        /* the current level has an energy to compare with */
    int32_t just_shifted;    /* the last reorder stalled and a new shift was drawn */
    uint64_t E_prev;         /* the energy compared with */
    uint64_t E_last;         /* energy after the last reorder */
    int64_t level_reorders;  /* reorders of the current level so far */
    uint64_t level_moved;    /* cells moved in the current level so far */
    int32_t done;            /* nonzero: the schedule has ended */
    int32_t reserved;
} plas_ref_state;

typedef struct {
    uint64_t seed;
    double radius_decay;      /* 0.95 (Sec. 3.1) */
    uint32_t inv_threshold;   /* 10000: stall below a 0.01 % improvement (Sec. 3.1) */
    int32_t min_block;        /* 16 (Sec. 3.1) */
    double start_radius;      /* <= 0: w/2 - 1 (Sec. 3.1) */
    int64_t max_reorders;     /* 0: run to the end of the schedule */
    const int32_t* init_perm; /* NULL: random start (Sec. 3.1) */
    int32_t storage_bf16;     /* nonzero: features and blurred grids held in bfloat16 */
    int32_t filter;           /* PLAS_REF_FILTER_BOX (0) or PLAS_REF_FILTER_BOX3 (1) */
    const plas_ref_state* resume; /* NULL: a new sort; else continue from this state, init_perm
                                     holding the stopped sort's permutation */
} plas_ref_params;

/* The low-pass filter of the target. BOX: one box pass per axis. BOX3: the
 * box pass three times per axis (rows three times, then columns three
 * times), a Gaussian-like filter of variance r(r+1) per axis. */
#define PLAS_REF_FILTER_BOX 0
#define PLAS_REF_FILTER_BOX3 1

typedef struct {
    double phi;
    int32_t r;
    int32_t beta;
    int64_t reorders;
    uint64_t energy;  /* integer energy after the level's last reorder */
    uint64_t moved;   /* cells that changed place over the level */
} plas_ref_level;

typedef struct {
    int64_t reorders;
    int32_t levels;
    int32_t scale_shift;
    uint64_t energy;
    double energy_mean;
    plas_ref_level* trace;      /* caller-owned, may be NULL */
    int32_t trace_cap;
    int32_t trace_len;
    uint64_t* reorder_energy;   /* caller-owned, may be NULL: E after each reorder */
    int64_t reorder_energy_cap;
    plas_ref_state* state;      /* caller-owned, may be NULL: where the sort stopped */
} plas_ref_result;

/* Philox4x64-10 block: out = Philox(ctr, key). */
void plas_ref_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
/* The four words drawn for (seed, purpose, index): ctr = (purpose, index, 0, 0), key = (seed, 0). */
void plas_ref_draw(uint64_t seed, uint64_t purpose, uint64_t index, uint64_t out[4]);
/* MurmurHash3 64-bit finaliser. */
uint64_t plas_ref_fmix64(uint64_t k);
/* Keyed bijection of [0, n): 4-round Feistel network with cycle walking. */
uint64_t plas_ref_bijection(uint64_t n, const uint64_t round_keys[4], uint64_t i);
void plas_ref_bijection_table(uint64_t n, const uint64_t round_keys[4], int64_t* out);
/* Block shift for shift draw j on a grid of side w. */
void plas_ref_shift(uint64_t seed, uint64_t j, int32_t w, int32_t* dy, int32_t* dx);

/* Energy scale: s such that per-cell quantised distances sum below 2^61. */
int32_t plas_ref_scale_shift(const float* F, int64_t n, int32_t d, int32_t layout,
                             int32_t* s_out, double* dmax_out);
/* Separable box blur with clamped windows: T = V_r(H_r(G)), G and T [N][d]. */
int32_t plas_ref_blur(const float* G, float* T, int32_t w, int32_t d, int32_t r);
/* The same, with each pass's output rounded to bfloat16 when storage_bf16. */
int32_t plas_ref_blur_storage(const float* G, float* T, int32_t w, int32_t d, int32_t r,
                              int32_t storage_bf16);
/* The same for either filter: BOX3 runs the row pass three times and then
 * the column pass three times, each pass's output rounded as stored. */
int32_t plas_ref_blur_filter(const float* G, float* T, int32_t w, int32_t d, int32_t r,
                             int32_t storage_bf16, int32_t filter);
/* x rounded to the nearest bfloat16 (ties to even), returned as float. */
float plas_ref_round_bf16(float x);
/* Squared L2 distance, pairwise tree over channels padded to a power of two. */
float plas_ref_distance(const float* a, const float* b, int32_t d);
/* floor(dist * 2^s) as an exact unsigned integer. */
uint64_t plas_ref_quantise(float dist, int32_t s);
/* sum over cells of quantise(distance(G[p], T[p])). */
uint64_t plas_ref_energy_fixed(const float* G, const float* T, int64_t N, int32_t d, int32_t s);
/* The 24 permutations of (0,1,2,3) in lexicographic order, as out[24][4]. */
void plas_ref_perms24(int32_t* out);
/* One blockwise linear assignment (one reorder): regroups, swaps G and P in
 * place, returns the integer energy of the new arrangement against T. */
uint64_t plas_ref_assign(float* G, const float* T, int32_t* P, int32_t w, int32_t d,
                         int32_t beta, int32_t dy, int32_t dx, const uint64_t round_keys[4],
                         int32_t s, uint64_t* moved_out);
/* The radius schedule: fills phi/r/beta for each level, returns the count. */
int32_t plas_ref_schedule(int32_t w, double decay, int32_t min_block, double start_radius,
                          double* phi, int32_t* r, int32_t* beta, int32_t cap);
/* Arranged grid G[p] = F[perm[p]] as [N][d] (perm NULL = identity). */
int32_t plas_ref_gather(const float* F, const int32_t* perm, int64_t n, int32_t d,
                        int32_t layout, float* G);

/* Progress control inside one radius level (Sec. 3.1). */
typedef struct {
    int32_t has_prev;      /* the level has an energy to compare the next one with */
    int32_t just_shifted;  /* the last reorder stalled and a new shift was drawn */
    uint64_t E_prev;       /* the energy the next reorder is compared with */
} plas_ref_ctl;

#define PLAS_REF_CTL_KEEP 0  /* improved: the next reorder keeps the block shift */
#define PLAS_REF_CTL_SHIFT 1 /* first stall: draw a new block shift */
#define PLAS_REF_CTL_END 2   /* stall right after a new shift: the level ends */

/* 1 iff a reorder with energy E improves on E_prev by at least 1/M of it
 * (always 1 when there is no previous energy), else 0. */
int32_t plas_ref_improved(uint64_t E, uint64_t E_prev, int32_t has_prev, uint32_t M);
/* Applies a reorder's energy E to the level's control state c and returns
 * the action: KEEP, SHIFT or END. A new level starts from {0, 0, 0}. */
int32_t plas_ref_control(plas_ref_ctl* c, uint64_t E, uint32_t M);

/* The whole sort. */
int32_t plas_ref_sort(const float* F, int64_t n, int32_t d, int32_t side, int32_t layout,
                      const plas_ref_params* params, int32_t* perm_out, plas_ref_result* res);
/* Integer grid energy of an arrangement at radius r. */
int32_t plas_ref_grid_energy(const float* F, const int32_t* perm, int64_t n, int32_t d,
                             int32_t side, int32_t layout, int32_t r, uint64_t* energy,
                             int32_t* s_out, double* energy_mean);
/* The same with bfloat16 storage of the features and the blurred grid. */
int32_t plas_ref_grid_energy_storage(const float* F, const int32_t* perm, int64_t n, int32_t d,
                                     int32_t side, int32_t layout, int32_t r, int32_t storage_bf16,
                                     uint64_t* energy, int32_t* s_out, double* energy_mean);
/* The same energy in float64 with direct window means and no quantisation:
 * mean over cells of the squared distance to the blurred grid. */
double plas_ref_grid_energy_f64(const float* F, const int32_t* perm, int64_t n, int32_t d,
                                int32_t side, int32_t layout, int32_t r);
/* Variance of the absolute differences between 4-neighbours (App. C). */
double plas_ref_vad(const float* F, const int32_t* perm, int64_t n, int32_t d, int32_t side,
                    int32_t layout);

/* Thread count for the parallel loops; returns the count now in effect. */
int32_t plas_ref_set_threads(int32_t threads);

#ifdef __cplusplus
}
#endif
#endif
