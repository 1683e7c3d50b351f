/*
 * plas_oracle.c -- reference CPU implementation of Parallel Linear Assignment
 * Sorting (PLAS), Sec. 3.1 of "Compact 3D Scene Representation via
 * Self-Organizing Gaussian Grids" (arXiv 2312.13299).
 *
 * TEST INFRASTRUCTURE ONLY: it checks the GPU library and is loaded only by
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark.
 * It shares no code with the GPU library.
 *
 * It is written to be read against the paper, not to be fast. Each step is a
 * plain loop in the order the method states it. OpenMP threads split
 * independent lines, groups and cells; they never change the order of a
 * floating-point operation, and the only cross-thread sums are exact integer
 * sums, so the result is the same at any thread count.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 * No FMA contraction, IEEE single precision with round-to-nearest-even and
 * denormals kept.
 *
 * What the paper states and where (Sec. 3.1, "Sorting High Dimensional
 * Gaussians into 2D Grids", and Fig. "blockwise_assignment"/"swapping_pixels"):
 *  - start from a random arrangement;
 *  - low-pass filter the grid into a target, reassign elements towards it,
 *    repeat with a shrinking filter, starting at radius w/2 - 1 and shrinking
 *    by phi <- 0.95 phi until the radius would fall below 1;
 *  - blocks of side beta = phi + 1, never below 16, shifted together by a
 *    random (dy, dx), processed independently;
 *  - groups of 4 from one random permutation of a block's elements, shared by
 *    all blocks; each group takes the best of its 24 permutations;
 *  - after each assignment, compare the mean L2 distance to the previous one;
 *    below a 0.01 % improvement draw a new block position, and if that does
 *    not improve either, shrink the radius.
 * Where the paper is silent this file takes the readings listed beside each
 * function (box filter, arithmetic order, integer energy, RNG).
 */
#include "plas_oracle.h"

#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* Loops over fewer items than this run on one thread: the work is too small
 * to repay starting a parallel region. Thread count never changes results. */
#define PAR_MIN_ITEMS 16384

/* ------------------------------------------------------------------------ */
/* Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel      */
/* Random Numbers: As Easy as 1, 2, 3", SC'11). The paper does not name a   */
/* generator (Sec. 3.1); a counter-based one lets every draw be named        */
/* by (seed, purpose, index). Pinned against numpy.random.Philox.            */
/* ------------------------------------------------------------------------ */

#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

static void mul_hi_lo(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void plas_ref_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mul_hi_lo(PHILOX_M0, x0, &hi0, &lo0);
        mul_hi_lo(PHILOX_M1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* Purposes: 0 = initial arrangement, 1 = grouping of reorder k, 2 = block
 * shift draw j. */
void plas_ref_draw(uint64_t seed, uint64_t purpose, uint64_t index, uint64_t out[4])
{
    uint64_t ctr[4] = {purpose, index, 0, 0};
    uint64_t key[2] = {seed, 0};
    plas_ref_philox4x64_10(ctr, key, out);
}

/* MurmurHash3's 64-bit finaliser (Austin Appleby, public domain). */
uint64_t plas_ref_fmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb53fe1a85ec3ULL;
    k ^= k >> 33;
    return k;
}

/* ------------------------------------------------------------------------ */
/* Random permutations. Each block's elements are split into groups of four */
/* along one random permutation of the block (Sec. 3.1, Blockwise Linear     */
/* Assignment), and the sort starts from a random arrangement (Sec. 3.1).    */
/* Reading: a keyed bijection of [0, n) evaluated per element: a balanced    */
/* 4-round Feistel network on 2h bits, h = max(1, ceil(ceil(log2 n) / 2)),   */
/* round function                                                            */
/* F(R, K) = fmix64(R xor K) mod 2^h, and cycle walking (Black and Rogaway,  */
/* "Ciphers with Arbitrary Finite Domains", 2002) down to [0, n).            */
/* Pinned: bijective for every n up to 2^16 and sampled larger n; key        */
/* dependent; statistically uniform.                                         */
/* ------------------------------------------------------------------------ */

static int half_width(uint64_t n)
{
    int bits = 0;
    while (bits < 64 && ((uint64_t)1 << bits) < n)
        bits++;
    int h = (bits + 1) / 2;
    return h < 1 ? 1 : h;
}

static uint64_t feistel4(uint64_t x, int h, const uint64_t rk[4])
{
    uint64_t mask = ((uint64_t)1 << h) - 1;
    uint64_t left = x >> h;
    uint64_t right = x & mask;
    for (int i = 0; i < 4; i++) {
        uint64_t f = plas_ref_fmix64(right ^ rk[i]) & mask;
        uint64_t new_left = right;
        uint64_t new_right = left ^ f;
        left = new_left;
        right = new_right;
    }
    return (left << h) | right;
}

uint64_t plas_ref_bijection(uint64_t n, const uint64_t rk[4], uint64_t i)
{
    int h = half_width(n);
    uint64_t y = feistel4(i, h, rk);
    while (y >= n)
        y = feistel4(y, h, rk);
    return y;
}

void plas_ref_bijection_table(uint64_t n, const uint64_t rk[4], int64_t* out)
{
#pragma omp parallel for schedule(static) if (n >= PAR_MIN_ITEMS)
    for (int64_t i = 0; i < (int64_t)n; i++)
        out[i] = (int64_t)plas_ref_bijection(n, rk, (uint64_t)i);
}

/* All blocks move together by one random offset (dy, dx) per draw (Sec.
 * 3.1). Reading: a torus
 * roll with dy, dx uniform in [0, w), taken from the top 32 bits of the first
 * two words of the shift draw: (hi32 * w) >> 32. */
void plas_ref_shift(uint64_t seed, uint64_t j, int32_t w, int32_t* dy, int32_t* dx)
{
    uint64_t u[4];
    plas_ref_draw(seed, 2, j, u);
    *dy = (int32_t)(((u[0] >> 32) * (uint64_t)w) >> 32);
    *dx = (int32_t)(((u[1] >> 32) * (uint64_t)w) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Feature access                                                            */
/* ------------------------------------------------------------------------ */

static float feature_at(const float* F, int64_t n, int32_t d, int32_t layout, int64_t i, int32_t c)
{
    if (layout == PLAS_REF_LAYOUT_CN)
        return F[(int64_t)c * n + i];
    return F[i * d + c];
}

/* ------------------------------------------------------------------------ */
/* Energy scale. The paper tracks progress by the mean L2 distance of the    */
/* sorted grid to its target (Sec. 3.1) and compares it with a relative     */
/* threshold. Reading: the stall test runs on an exact integer energy, the   */
/* sum over cells of floor(d * 2^s), with s fixed once per input so that the */
/* sum over all N cells stays below 2^61:                                    */
/*   D_max = sum_c (max_c - min_c)^2 in float64, channels in order;          */
/*   N * D_max = m * 2^e with m in [0.5, 1) (frexp); s = 61 - e;             */
/*   s = 0 when D_max = 0.                                                   */
/* Any cell's distance to a target of window means is at most about D_max,   */
/* because every target value is a mean of grid values of the same channel. */
/* Non-finite features are rejected.                                         */
/* ------------------------------------------------------------------------ */

int32_t plas_ref_scale_shift(const float* F, int64_t n, int32_t d, int32_t layout,
                             int32_t* s_out, double* dmax_out)
{
    if (F == NULL || n < 1 || d < 1)
        return PLAS_REF_INVALID;
    double dmax = 0.0;
    for (int32_t c = 0; c < d; c++) {
        float lo = INFINITY, hi = -INFINITY;
        for (int64_t i = 0; i < n; i++) {
            float v = feature_at(F, n, d, layout, i, c);
            if (!isfinite(v))
                return PLAS_REF_NONFINITE;
            if (v < lo)
                lo = v;
            if (v > hi)
                hi = v;
        }
        double span = (double)hi - (double)lo;
        dmax += span * span;
    }
    int32_t s = 0;
    if (dmax > 0.0) {
        int e = 0;
        frexp((double)n * dmax, &e);
        s = 61 - e;
    }
    if (s_out)
        *s_out = s;
    if (dmax_out)
        *dmax_out = dmax;
    return PLAS_REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Target: the low-pass filtered grid (Sec. 3.1; Fig. "blockwise_assignment" */
/* caption). Readings, the paper naming a Gaussian filter of shrinking size  */
/* without giving its kernel:                                                */
/*  - a box (mean) filter of half-width r = floor(phi), separable, rows      */
/*    first then columns;                                                    */
/*  - at the borders the window is clipped to the grid and the sum divided   */
/*    by the number of cells inside, i.e. the mean over the clipped window;  */
/*  - each pass runs per line as a sliding sum: start with the ascending sum */
/*    of line[0..min(r, w-1)]; at each next position add the entering value  */
/*    (if inside) and then subtract the leaving one (if inside); the output  */
/*    is the running sum times float32(1/count), the correctly rounded       */
/*    reciprocal of the window's cell count;                                 */
/*  - r = 0 is the identity (a window of one cell).                          */
/* Pinned: constant and linear-ramp closed forms, exact small-integer sums,  */
/* a float64 brute-force mean within the rounding bound, grid symmetries.    */
/* ------------------------------------------------------------------------ */

/* Round to bfloat16 (8 exponent bits, 7 stored mantissa bits) to nearest,
 * ties to even: add half an ulp of the kept part, plus one if the kept part
 * is odd, then drop the low 16 bits. Infinities and NaNs pass unchanged.
 * Pinned against torch's float32 -> bfloat16 conversion. */
float plas_ref_round_bf16(float x)
{
    uint32_t u;
    memcpy(&u, &x, sizeof(u));
    if ((u & 0x7f800000u) == 0x7f800000u)
        return x;
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
    float y;
    memcpy(&y, &u, sizeof(y));
    return y;
}

static int32_t window_count(int32_t x, int32_t r, int32_t w)
{
    int32_t lo = x - r < 0 ? 0 : x - r;
    int32_t hi = x + r > w - 1 ? w - 1 : x + r;
    return hi - lo + 1;
}

/* The window mean as stored: float32, or rounded to bfloat16 (the inputs of
 * a bfloat16 grid are already bfloat16 values; sums stay float32). */
static float stored(float v, int32_t bf16)
{
    return bf16 ? plas_ref_round_bf16(v) : v;
}

static void box_line(const float* in, ptrdiff_t step, float* out, int32_t w, int32_t r,
                     const float* inv, int32_t bf16)
{
    if (r == 0) {
        for (int32_t x = 0; x < w; x++)
            out[x * step] = in[x * step];
        return;
    }
    int32_t first_hi = r < w - 1 ? r : w - 1;
    float s = in[0];
    for (int32_t t = 1; t <= first_hi; t++)
        s = s + in[t * step];
    out[0] = stored(s * inv[window_count(0, r, w)], bf16);
    for (int32_t x = 1; x < w; x++) {
        if (x + r <= w - 1)
            s = s + in[(ptrdiff_t)(x + r) * step];
        if (x - r - 1 >= 0)
            s = s - in[(ptrdiff_t)(x - r - 1) * step];
        out[x * step] = stored(s * inv[window_count(x, r, w)], bf16);
    }
}

int32_t plas_ref_blur(const float* G, float* T, int32_t w, int32_t d, int32_t r)
{
    return plas_ref_blur_storage(G, T, w, d, r, 0);
}

int32_t plas_ref_blur_storage(const float* G, float* T, int32_t w, int32_t d, int32_t r,
                              int32_t storage_bf16)
{
    return plas_ref_blur_filter(G, T, w, d, r, storage_bf16, PLAS_REF_FILTER_BOX);
}

/* One box pass over every line of one axis: rows (horizontal) or columns. */
static void box_pass(const float* in, float* out, int32_t w, int32_t d, int32_t r, const float* inv,
                     int32_t bf16, int vertical)
{
    int64_t N = (int64_t)w * w;
    (void)N;
#pragma omp parallel for schedule(static) if (N >= PAR_MIN_ITEMS)
    for (int32_t l = 0; l < w; l++)
        for (int32_t c = 0; c < d; c++) {
            if (vertical)
                box_line(in + (int64_t)l * d + c, (ptrdiff_t)w * d, out + (int64_t)l * d + c, w, r, inv,
                         bf16);
            else
                box_line(in + (int64_t)l * w * d + c, d, out + (int64_t)l * w * d + c, w, r, inv, bf16);
        }
}

/* Gaussian-like variant (BOX3): the paper names a Gaussian filter without
 * its kernel. Repeating a box filter approaches a Gaussian (the sum of
 * three uniform variables; Wells, "Efficient synthesis of Gaussian filters
 * by cascaded uniform filters", IEEE TPAMI 1986): three passes of
 * half-width r per axis give a piecewise-quadratic kernel of support 3r
 * and variance 3 * r(r+1)/3 = r(r+1) per axis. Rows first, three times,
 * then columns three times; every pass is the clipped box pass above.
 * Pinned: the response to a single impulse against the three-fold
 * convolution of box kernels (interior and at a border), its variance,
 * r = 0 and constant grids. */
int32_t plas_ref_blur_filter(const float* G, float* T, int32_t w, int32_t d, int32_t r,
                             int32_t storage_bf16, int32_t filter)
{
    if (G == NULL || T == NULL || w < 1 || d < 1 || r < 0 ||
        (filter != PLAS_REF_FILTER_BOX && filter != PLAS_REF_FILTER_BOX3))
        return PLAS_REF_INVALID;
    const int passes = filter == PLAS_REF_FILTER_BOX3 ? 3 : 1;
    int64_t N = (int64_t)w * w;
    float* inv = (float*)malloc(sizeof(float) * (size_t)(w + 1));
    float* A = (float*)malloc(sizeof(float) * (size_t)(N * d));
    float* B = passes > 1 ? (float*)malloc(sizeof(float) * (size_t)(N * d)) : NULL;
    if (inv == NULL || A == NULL || (passes > 1 && B == NULL)) {
        free(inv);
        free(A);
        free(B);
        return PLAS_REF_INVALID;
    }
    inv[0] = 0.0f;
    for (int32_t c = 1; c <= w; c++)
        inv[c] = 1.0f / (float)c;
    float* bufs[2] = {A, B};
    const float* src = G;
    /* Horizontal passes: every row, every channel. */
    for (int p = 0; p < passes; p++) {
        float* dst = bufs[p & 1];
        box_pass(src, dst, w, d, r, inv, storage_bf16, 0);
        src = dst;
    }
    /* Vertical passes on the result: every column, every channel; the last
     * one writes T. */
    for (int p = 0; p < passes; p++) {
        float* dst = p == passes - 1 ? T : bufs[(passes + p) & 1];
        box_pass(src, dst, w, d, r, inv, storage_bf16, 1);
        src = dst;
    }
    free(B);
    free(A);
    free(inv);
    return PLAS_REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Distance. Each group keeps the ordering with the smallest summed         */
/* distance (Fig. "swapping_pixels"), and progress is measured by the mean   */
/* L2 distance to the target (Sec. 3.1). Reading: the squared Euclidean      */
/* distance, as in linear assignment sorting (Sec. 2.2). Its channel sum is  */
/* a balanced pairwise tree over the channels padded with zeros to the next  */
/* power of two m: sum(v[0..m)) = sum(v[0..m/2)) + sum(v[m/2..m)). Each term */
/* is the rounded difference times itself (no FMA).                          */
/* Pinned: d(x, x) = 0, one channel, a float64 dot product within the        */
/* pairwise bound, and a hand-computed case that separates tree from         */
/* sequential order.                                                         */
/* ------------------------------------------------------------------------ */

static float pairwise_sum(const float* v, int32_t m)
{
    if (m == 1)
        return v[0];
    int32_t half = m / 2;
    float left = pairwise_sum(v, half);
    float right = pairwise_sum(v + half, half);
    return left + right;
}

float plas_ref_distance(const float* a, const float* b, int32_t d)
{
    float sq[PLAS_REF_MAX_D];
    int32_t m = 1;
    while (m < d)
        m *= 2;
    for (int32_t c = 0; c < m; c++) {
        if (c < d) {
            float delta = a[c] - b[c];
            sq[c] = delta * delta;
        } else {
            sq[c] = 0.0f;
        }
    }
    return pairwise_sum(sq, m);
}

/* floor(dist * 2^s): exact, since scaling by a power of two is exact in
 * float64 and the cast truncates a non-negative value. */
uint64_t plas_ref_quantise(float dist, int32_t s)
{
    return (uint64_t)ldexp((double)dist, s);
}

uint64_t plas_ref_energy_fixed(const float* G, const float* T, int64_t N, int32_t d, int32_t s)
{
    uint64_t E = 0;
#pragma omp parallel for schedule(static) reduction(+ : E) if (N >= PAR_MIN_ITEMS)
    for (int64_t p = 0; p < N; p++)
        E += plas_ref_quantise(plas_ref_distance(G + p * d, T + p * d, d), s);
    return E;
}

/* ------------------------------------------------------------------------ */
/* Blockwise linear assignment (Sec. 3.1, "Blockwise Linear Assignment";     */
/* Fig. "swapping_pixels").                                                  */
/* ------------------------------------------------------------------------ */

/* The 24 orderings of four elements, lexicographic: (0,1,2,3) first. */
void plas_ref_perms24(int32_t* out)
{
    int k = 0;
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++)
            for (int c = 0; c < 4; c++)
                for (int e = 0; e < 4; e++) {
                    if (a == b || a == c || a == e || b == c || b == e || c == e)
                        continue;
                    out[4 * k + 0] = a;
                    out[4 * k + 1] = b;
                    out[4 * k + 2] = c;
                    out[4 * k + 3] = e;
                    k++;
                }
}

/*
 * One reorder. Readings:
 *  - the grid is rolled by (dy, dx) and cut into nb x nb blocks of side beta,
 *    nb = floor(w / beta); cells of the rolled grid outside the nb*beta
 *    square are not grouped this time (a later shift moves them in);
 *  - the shared block permutation pi is the keyed bijection of [0, beta^2);
 *    group g of every block takes block-local cells pi(4g .. 4g+3), row-major
 *    inside the block; the beta^2 mod 4 left-over cells stay put;
 *  - group cell i moves to place sigma(i) for the permutation sigma with the
 *    smallest cost sum_i floor(d(G[c_i], T[c_sigma(i)]) * 2^s), computed in
 *    exact integers; the first minimum in lexicographic order wins, so ties
 *    keep the current places;
 *  - the returned energy covers every cell: each group's minimum cost plus
 *    floor(d(G[p], T[p]) * 2^s) for every ungrouped cell.
 * Pinned: each group's choice equals an exhaustive search over the 24
 * orderings; on a 2x2 grid with a given target one reorder reaches the best
 * of all 24 arrangements; the energy never rises within a reorder and equals
 * a recomputation from the new grid.
 */
uint64_t plas_ref_assign(float* G, const float* T, int32_t* P, int32_t w, int32_t d,
                         int32_t beta, int32_t dy, int32_t dx, const uint64_t rk[4],
                         int32_t s, uint64_t* moved_out)
{
    int64_t N = (int64_t)w * w;
    int32_t nb = w / beta;
    int64_t cells_per_block = (int64_t)beta * beta;
    int64_t groups_per_block = cells_per_block / 4;
    int64_t* pi = (int64_t*)malloc(sizeof(int64_t) * (size_t)cells_per_block);
    unsigned char* grouped = (unsigned char*)calloc((size_t)N, 1);
    int32_t perms[24 * 4];
    plas_ref_perms24(perms);
    plas_ref_bijection_table((uint64_t)cells_per_block, rk, pi);

    uint64_t E = 0, moved = 0;
    const int64_t total_groups = (int64_t)nb * nb * groups_per_block;
#pragma omp parallel for schedule(static) reduction(+ : E, moved) if (N >= PAR_MIN_ITEMS)
    for (int64_t item = 0; item < total_groups; item++) {
        int64_t blk = item / groups_per_block, g = item % groups_per_block;
        int64_t by = blk / nb, bx = blk % nb;
        int64_t cell[4];
        for (int i = 0; i < 4; i++) {
            int64_t local = pi[4 * g + i];
            int64_t ly = local / beta, lx = local % beta;
            int64_t y = (dy + by * beta + ly) % w;
            int64_t x = (dx + bx * beta + lx) % w;
            cell[i] = y * w + x;
        }
        uint64_t q[4][4];
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++)
                q[i][j] = plas_ref_quantise(
                    plas_ref_distance(G + cell[i] * d, T + cell[j] * d, d), s);
        int best = 0;
        uint64_t best_cost = 0;
        for (int m = 0; m < 24; m++) {
            const int32_t* sg = perms + 4 * m;
            uint64_t cost = q[0][sg[0]] + q[1][sg[1]] + q[2][sg[2]] + q[3][sg[3]];
            if (m == 0 || cost < best_cost) {
                best = m;
                best_cost = cost;
            }
        }
        E += best_cost;
        const int32_t* sg = perms + 4 * best;
        float saved[4 * PLAS_REF_MAX_D];
        int32_t saved_perm[4];
        for (int i = 0; i < 4; i++) {
            memcpy(saved + i * d, G + cell[i] * d, sizeof(float) * (size_t)d);
            saved_perm[i] = P[cell[i]];
        }
        for (int i = 0; i < 4; i++) {
            int64_t dst = cell[sg[i]];
            memcpy(G + dst * d, saved + i * d, sizeof(float) * (size_t)d);
            P[dst] = saved_perm[i];
            if (sg[i] != i)
                moved++;
            grouped[cell[i]] = 1;
        }
    }
    /* Cells that were in no group keep their place; their distance still
     * counts, because the energy covers the whole grid. */
#pragma omp parallel for schedule(static) reduction(+ : E) if (N >= PAR_MIN_ITEMS)
    for (int64_t p = 0; p < N; p++)
        if (!grouped[p])
            E += plas_ref_quantise(plas_ref_distance(G + p * d, T + p * d, d), s);
    free(grouped);
    free(pi);
    if (moved_out)
        *moved_out = moved;
    return E;
}

/* ------------------------------------------------------------------------ */
/* Radius schedule (Sec. 3.1): phi starts at w/2 - 1 and shrinks by 0.95     */
/* until it would fall below 1. Readings: r = floor(phi); block side         */
/* beta = r + 1 clamped to [min_block, w]; for w <= 3 the start is raised to */
/* 1 so that tiny grids run one level.                                       */
/* Pinned: level counts against the closed form 1 + floor(ln phi0 /          */
/* ln(1/0.95)) for several w.                                                */
/* ------------------------------------------------------------------------ */

int32_t plas_ref_schedule(int32_t w, double decay, int32_t min_block, double start_radius,
                          double* phi, int32_t* r, int32_t* beta, int32_t cap)
{
    if (w < 1 || !(decay > 0.0 && decay < 1.0))
        return PLAS_REF_INVALID;
    double f = start_radius > 0.0 ? start_radius : (double)w / 2.0 - 1.0;
    if (f < 1.0)
        f = 1.0;
    int32_t count = 0;
    while (f >= 1.0) {
        if (count < cap) {
            int32_t rr = (int32_t)floor(f);
            int32_t b = rr + 1;
            if (b < min_block)
                b = min_block;
            if (b > w)
                b = w;
            if (phi)
                phi[count] = f;
            if (r)
                r[count] = rr;
            if (beta)
                beta[count] = b;
        }
        count++;
        f = f * decay;
    }
    return count;
}

int32_t plas_ref_gather(const float* F, const int32_t* perm, int64_t n, int32_t d,
                        int32_t layout, float* G)
{
    if (F == NULL || G == NULL || n < 1 || d < 1)
        return PLAS_REF_INVALID;
    for (int64_t p = 0; p < n; p++) {
        int64_t src = perm ? (int64_t)perm[p] : p;
        if (src < 0 || src >= n)
            return PLAS_REF_INVALID;
        for (int32_t c = 0; c < d; c++)
            G[p * d + c] = feature_at(F, n, d, layout, src, c);
    }
    return PLAS_REF_OK;
}

static int is_bijection(const int32_t* perm, int64_t n)
{
    unsigned char* seen = (unsigned char*)calloc((size_t)n, 1);
    int ok = 1;
    for (int64_t p = 0; p < n && ok; p++) {
        if (perm[p] < 0 || perm[p] >= n || seen[perm[p]])
            ok = 0;
        else
            seen[perm[p]] = 1;
    }
    free(seen);
    return ok;
}

/* ------------------------------------------------------------------------ */
/* Progress control between reorders of one radius level (Sec. 3.1): after  */
/* each assignment the distance to the target is compared with the previous */
/* one; an improvement of less than 0.01 % counts as none. Then a new block */
/* position is drawn, and if the reorder with that position does not        */
/* improve either, the level ends and the radius shrinks.                   */
/* Readings: the distance is the integer energy E; with M = 10^4 a reorder  */
/* improves iff E < E_prev and E_prev - E >= ceil(E_prev / M), which for    */
/* integers is exactly (E_prev - E) / E_prev >= 1 / M, evaluated without a  */
/* 128-bit product. The first reorder of a level has nothing to compare     */
/* with and counts as an improvement. After a stall the stalled energy is   */
/* the one the next reorder must beat.                                      */
/* Pinned: against exact rational arithmetic at and around the threshold,  */
/* on hand-worked energy sequences, and by replaying whole sorts' energies. */
/* ------------------------------------------------------------------------ */

int32_t plas_ref_improved(uint64_t E, uint64_t E_prev, int32_t has_prev, uint32_t M)
{
    if (!has_prev)
        return 1;
    if (M < 1 || E >= E_prev)
        return 0;
    uint64_t need = E_prev / M + (E_prev % M != 0); /* ceil(E_prev / M) */
    return E_prev - E >= need;
}

int32_t plas_ref_control(plas_ref_ctl* c, uint64_t E, uint32_t M)
{
    if (plas_ref_improved(E, c->E_prev, c->has_prev, M)) {
        c->E_prev = E;
        c->has_prev = 1;
        c->just_shifted = 0;
        return PLAS_REF_CTL_KEEP;
    }
    if (c->just_shifted)
        return PLAS_REF_CTL_END;
    c->just_shifted = 1;
    c->E_prev = E;
    return PLAS_REF_CTL_SHIFT;
}

/* ------------------------------------------------------------------------ */
/* The sort (Sec. 3.1). Control, per level:                                  */
/*  - draw a block shift; no previous energy yet;                            */
/*  - each reorder: target = blur(grid), then one blockwise assignment;      */
/*  - after it, plas_ref_control: improved (see above) keeps the shift;      */
/*    a first stall draws a new shift; a stall right after a new shift ends  */
/*    the level.                                                             */
/* The grouping permutation is drawn anew for every reorder k (purpose 1),   */
/* the shift for every shift draw j (purpose 2), the start arrangement once  */
/* (purpose 0).                                                              */
/* ------------------------------------------------------------------------ */

int32_t plas_ref_sort(const float* F, int64_t n, int32_t d, int32_t side, int32_t layout,
                      const plas_ref_params* prm, int32_t* perm_out, plas_ref_result* res)
{
    if (F == NULL || prm == NULL || perm_out == NULL || side < 2 || d < 1 ||
        d > PLAS_REF_MAX_D || n != (int64_t)side * side ||
        (layout != PLAS_REF_LAYOUT_CN && layout != PLAS_REF_LAYOUT_NC) ||
        !(prm->radius_decay > 0.0 && prm->radius_decay < 1.0) || prm->inv_threshold < 1 ||
        prm->min_block < 1 || (prm->filter != PLAS_REF_FILTER_BOX && prm->filter != PLAS_REF_FILTER_BOX3))
        return PLAS_REF_INVALID;
    const int32_t w = side;
    const int64_t N = n;
    const int32_t bf16 = prm->storage_bf16 != 0;
    /* bfloat16 storage: the sort sees the features rounded to bfloat16. */
    float* rounded = NULL;
    if (bf16) {
        rounded = (float*)malloc(sizeof(float) * (size_t)(n * d));
        if (rounded == NULL)
            return PLAS_REF_INVALID;
        for (int64_t i = 0; i < n * d; i++)
            rounded[i] = plas_ref_round_bf16(F[i]);
        F = rounded;
    }
    int32_t s = 0;
    int32_t st = plas_ref_scale_shift(F, n, d, layout, &s, NULL);
    if (st == PLAS_REF_OK && prm->init_perm && !is_bijection(prm->init_perm, N))
        st = PLAS_REF_INVALID;
    if (st == PLAS_REF_OK && prm->resume &&
        (prm->init_perm == NULL || prm->resume->k < 0 || prm->resume->level < 0 ||
         prm->resume->levels_run < 0 || prm->resume->levels_run > prm->resume->level))
        st = PLAS_REF_INVALID;
    if (st != PLAS_REF_OK) {
        free(rounded);
        return st;
    }

    int32_t* P = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
    float* G = (float*)malloc(sizeof(float) * (size_t)(N * d));
    float* T = (float*)malloc(sizeof(float) * (size_t)(N * d));
    if (P == NULL || G == NULL || T == NULL) {
        free(P);
        free(G);
        free(T);
        free(rounded);
        return PLAS_REF_INVALID;
    }
    /* Start: random positions (Sec. 3.1) or the caller's arrangement. */
    if (prm->init_perm) {
        memcpy(P, prm->init_perm, sizeof(int32_t) * (size_t)N);
    } else {
        uint64_t rk[4];
        plas_ref_draw(prm->seed, 0, 0, rk);
        for (int64_t p = 0; p < N; p++)
            P[p] = (int32_t)plas_ref_bijection((uint64_t)N, rk, (uint64_t)p);
    }
    plas_ref_gather(F, P, n, d, layout, G);

    const uint64_t M = prm->inv_threshold;
    int64_t k = 0;      /* reorders done */
    uint64_t j = 0;     /* shift draws done */
    int32_t levels = 0;
    uint64_t E_last = 0;
    int stop = 0;
    int32_t level_index = 0;
    double phi = prm->start_radius > 0.0 ? prm->start_radius : (double)w / 2.0 - 1.0;
    if (phi < 1.0)
        phi = 1.0;
    /* Resume: the counters, and phi after the levels already entered. */
    const plas_ref_state* R = prm->resume;
    int resume_in_level = 0;
    if (R) {
        k = R->k;
        j = R->j;
        levels = R->levels_run;
        E_last = R->E_last;
        for (level_index = 0; level_index < R->level; level_index++)
            phi = phi * prm->radius_decay;
        resume_in_level = !R->done;
        if (R->done)
            phi = 0.0;
    }
    plas_ref_state at = {0};
    while (phi >= 1.0 && !stop) {
        int32_t r = (int32_t)floor(phi);
        int32_t beta = r + 1;
        if (beta < prm->min_block)
            beta = prm->min_block;
        if (beta > w)
            beta = w;
        int32_t dy, dx;
        plas_ref_ctl ctl = {0, 0, 0};
        int64_t level_reorders = 0;
        uint64_t level_moved = 0;
        if (resume_in_level) {
            /* Inside a level: its shift and stall state as they were. */
            dy = R->dy;
            dx = R->dx;
            ctl.has_prev = R->has_prev != 0;
            ctl.just_shifted = R->just_shifted != 0;
            ctl.E_prev = R->E_prev;
            level_reorders = R->level_reorders;
            level_moved = R->level_moved;
            resume_in_level = 0;
        } else {
            plas_ref_shift(prm->seed, j, w, &dy, &dx);
            j++;
        }
        for (;;) {
            if (prm->max_reorders > 0 && k >= prm->max_reorders) {
                stop = 1;
                at.level = level_index;
                at.levels_run = levels;
                at.dy = dy;
                at.dx = dx;
                at.has_prev = ctl.has_prev;
                at.just_shifted = ctl.just_shifted;
                at.E_prev = ctl.E_prev;
                at.level_reorders = level_reorders;
                at.level_moved = level_moved;
                break;
            }
            plas_ref_blur_filter(G, T, w, d, r, bf16, prm->filter);
            uint64_t rk[4];
            plas_ref_draw(prm->seed, 1, (uint64_t)k, rk);
            uint64_t moved = 0;
            uint64_t E = plas_ref_assign(G, T, P, w, d, beta, dy, dx, rk, s, &moved);
            if (res && res->reorder_energy && k < res->reorder_energy_cap)
                res->reorder_energy[k] = E;
            k++;
            level_reorders++;
            level_moved += moved;
            E_last = E;
            int32_t act = plas_ref_control(&ctl, E, M);
            if (act == PLAS_REF_CTL_END)
                break;
            if (act == PLAS_REF_CTL_SHIFT) {
                plas_ref_shift(prm->seed, j, w, &dy, &dx);
                j++;
            }
        }
        if (level_reorders > 0) {
            if (res && res->trace && levels < res->trace_cap) {
                plas_ref_level* L = &res->trace[levels];
                L->phi = phi;
                L->r = r;
                L->beta = beta;
                L->reorders = level_reorders;
                L->energy = E_last;
                L->moved = level_moved;
            }
            levels++;
        }
        if (!stop) {
            phi = phi * prm->radius_decay;
            level_index++;
        }
    }
    if (!stop) {
        at.level = level_index;
        at.levels_run = levels;
        at.done = 1;
    }
    at.k = k;
    at.j = j;
    at.E_last = E_last;
    if (res && res->state)
        *res->state = at;
    memcpy(perm_out, P, sizeof(int32_t) * (size_t)N);
    if (res) {
        res->reorders = k;
        res->levels = levels;
        res->scale_shift = s;
        res->energy = E_last;
        res->energy_mean = ldexp((double)E_last, -s) / (double)N;
        res->trace_len = levels < res->trace_cap ? levels : res->trace_cap;
    }
    free(P);
    free(G);
    free(T);
    free(rounded);
    return PLAS_REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Energy of a given arrangement (the distance of Sec. 3.1).                 */
/* ------------------------------------------------------------------------ */

int32_t plas_ref_grid_energy(const float* F, const int32_t* perm, int64_t n, int32_t d,
                             int32_t side, int32_t layout, int32_t r, uint64_t* energy,
                             int32_t* s_out, double* energy_mean)
{
    return plas_ref_grid_energy_storage(F, perm, n, d, side, layout, r, 0, energy, s_out,
                                        energy_mean);
}

int32_t plas_ref_grid_energy_storage(const float* F, const int32_t* perm, int64_t n, int32_t d,
                                     int32_t side, int32_t layout, int32_t r, int32_t storage_bf16,
                                     uint64_t* energy, int32_t* s_out, double* energy_mean)
{
    if (F == NULL || side < 1 || n != (int64_t)side * side || d < 1 || d > PLAS_REF_MAX_D ||
        r < 0 || (layout != PLAS_REF_LAYOUT_CN && layout != PLAS_REF_LAYOUT_NC))
        return PLAS_REF_INVALID;
    if (perm && !is_bijection(perm, n))
        return PLAS_REF_INVALID;
    float* rounded = NULL;
    if (storage_bf16) {
        rounded = (float*)malloc(sizeof(float) * (size_t)(n * d));
        for (int64_t i = 0; i < n * d; i++)
            rounded[i] = plas_ref_round_bf16(F[i]);
        F = rounded;
    }
    int32_t s = 0;
    int32_t st = plas_ref_scale_shift(F, n, d, layout, &s, NULL);
    if (st != PLAS_REF_OK) {
        free(rounded);
        return st;
    }
    float* G = (float*)malloc(sizeof(float) * (size_t)(n * d));
    float* T = (float*)malloc(sizeof(float) * (size_t)(n * d));
    plas_ref_gather(F, perm, n, d, layout, G);
    plas_ref_blur_storage(G, T, side, d, r, storage_bf16 != 0);
    uint64_t E = plas_ref_energy_fixed(G, T, n, d, s);
    free(G);
    free(T);
    free(rounded);
    if (energy)
        *energy = E;
    if (s_out)
        *s_out = s;
    if (energy_mean)
        *energy_mean = ldexp((double)E, -s) / (double)n;
    return PLAS_REF_OK;
}

/* Float64 form: window means summed directly over the clipped window, rows
 * then columns, and squared distances without quantisation; returns the mean
 * over cells of the squared distance. Used to compare arrangements across
 * precisions; its blur is pinned by the same brute-force checks. */
double plas_ref_grid_energy_f64(const float* F, const int32_t* perm, int64_t n, int32_t d,
                                int32_t side, int32_t layout, int32_t r)
{
    if (F == NULL || side < 1 || n != (int64_t)side * side || d < 1 || r < 0)
        return NAN;
    const int32_t w = side;
    double* G = (double*)malloc(sizeof(double) * (size_t)(n * d));
    double* H = (double*)malloc(sizeof(double) * (size_t)(n * d));
    double* T = (double*)malloc(sizeof(double) * (size_t)(n * d));
    for (int64_t p = 0; p < n; p++) {
        int64_t src = perm ? (int64_t)perm[p] : p;
        for (int32_t c = 0; c < d; c++)
            G[p * d + c] = (double)feature_at(F, n, d, layout, src, c);
    }
#pragma omp parallel for schedule(static) if (n >= PAR_MIN_ITEMS)
    for (int32_t y = 0; y < w; y++)
        for (int32_t x = 0; x < w; x++) {
            int32_t lo = x - r < 0 ? 0 : x - r, hi = x + r > w - 1 ? w - 1 : x + r;
            for (int32_t c = 0; c < d; c++) {
                double acc = 0.0;
                for (int32_t t = lo; t <= hi; t++)
                    acc += G[((int64_t)y * w + t) * d + c];
                H[((int64_t)y * w + x) * d + c] = acc / (double)(hi - lo + 1);
            }
        }
#pragma omp parallel for schedule(static) if (n >= PAR_MIN_ITEMS)
    for (int32_t y = 0; y < w; y++)
        for (int32_t x = 0; x < w; x++) {
            int32_t lo = y - r < 0 ? 0 : y - r, hi = y + r > w - 1 ? w - 1 : y + r;
            for (int32_t c = 0; c < d; c++) {
                double acc = 0.0;
                for (int32_t t = lo; t <= hi; t++)
                    acc += H[((int64_t)t * w + x) * d + c];
                T[((int64_t)y * w + x) * d + c] = acc / (double)(hi - lo + 1);
            }
        }
    double total = 0.0;
    for (int64_t p = 0; p < n; p++) {
        double acc = 0.0;
        for (int32_t c = 0; c < d; c++) {
            double delta = G[p * d + c] - T[p * d + c];
            acc += delta * delta;
        }
        total += acc;
    }
    free(G);
    free(H);
    free(T);
    return total / (double)n;
}

/* VAD, the sort-quality measure of App. C: the variance of |a - b| over
 * neighbouring cells, every channel counted. Reading: right and down
 * neighbours, no wrap-around; population variance in float64. */
double plas_ref_vad(const float* F, const int32_t* perm, int64_t n, int32_t d, int32_t side,
                    int32_t layout)
{
    if (F == NULL || side < 2 || n != (int64_t)side * side || d < 1)
        return NAN;
    const int32_t w = side;
    double sum = 0.0;
    int64_t count = 0;
    for (int pass = 0; pass < 2; pass++) {
        double mean = pass == 0 ? 0.0 : sum / (double)count;
        double acc = 0.0;
        for (int32_t y = 0; y < w; y++)
            for (int32_t x = 0; x < w; x++) {
                int64_t p = (int64_t)y * w + x;
                int64_t a = perm ? perm[p] : p;
                for (int dir = 0; dir < 2; dir++) {
                    int32_t yy = y + (dir == 1), xx = x + (dir == 0);
                    if (yy >= w || xx >= w)
                        continue;
                    int64_t q = (int64_t)yy * w + xx;
                    int64_t b = perm ? perm[q] : q;
                    for (int32_t c = 0; c < d; c++) {
                        double v = fabs((double)feature_at(F, n, d, layout, a, c) -
                                        (double)feature_at(F, n, d, layout, b, c));
                        if (pass == 0) {
                            acc += v;
                            count++;
                        } else {
                            acc += (v - mean) * (v - mean);
                        }
                    }
                }
            }
        if (pass == 0)
            sum = acc;
        else
            return acc / (double)count;
    }
    return NAN;
}

int32_t plas_ref_set_threads(int32_t threads)
{
    if (threads > 0)
        omp_set_num_threads(threads);
    return omp_get_max_threads();
}
