/*
 * plas.h -- C ABI of the MI355X (gfx950) PLAS library, libplas.so.
 *
 * PLAS (Parallel Linear Assignment Sorting) arranges N feature vectors on a
 * side x side grid (N = side^2) so that neighbouring cells hold similar
 * vectors. It is the sort of Sec. 3.1 ("Sorting High Dimensional Gaussians
 * into 2D Grids") of "Compact 3D Scene Representation via Self-Organizing
 * Gaussian Grids" (arXiv 2312.13299): starting from a random arrangement it
 * repeatedly blurs the grid into a target and reassigns random groups of four
 * cells by the best of their 24 permutations, with a shrinking blur radius.
 *
 * Every step runs in HIP kernels on the device; the host only validates
 * arguments, sequences launches and copies small results back.
 *
 * Conventions for every entry point:
 *  - Pointers named as device pointers must point to device memory of the
 *    handle's device (e.g. a torch CUDA tensor's data_ptr()); the library
 *    never frees them. Host pointers (stats, trace, scalar outputs) are
 *    caller-owned host memory.
 *  - Cells are row-major: cell p = y * side + x.
 *  - A permutation is in gather form: perm[p] is the index of the vector
 *    that sits at cell p (arranged = features[perm]).
 *  - Functions return PLAS_OK (0) or a negative status; they never throw
 *    across the ABI. plas_last_error() gives a message for the last failure
 *    on a handle.
 *  - Work is ordered on the handle's stream (plas_set_stream). Calls that
 *    fill host outputs synchronise that stream before returning.
 *  - One handle per host thread; a handle is not thread-safe.
 */
#ifndef PLAS_H
#define PLAS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PLAS_ABI_VERSION 2

/* Status codes. */
#define PLAS_OK 0
#define PLAS_ERR_INVALID_ARGUMENT (-1) /* NULL pointer, n != side^2, side < 2, bad d/layout/radius, init_perm not a bijection */
#define PLAS_ERR_UNSUPPORTED (-2)      /* a dtype or channel count the library does not handle */
#define PLAS_ERR_OUT_OF_MEMORY (-3)    /* the device workspace could not be allocated */
#define PLAS_ERR_HIP (-4)              /* a HIP runtime call failed; see plas_last_error */
#define PLAS_ERR_NONFINITE (-5)        /* a feature value is NaN or infinite */

/* Feature layouts. */
#define PLAS_LAYOUT_CN 0 /* channel-major: features[c * n + i] */
#define PLAS_LAYOUT_NC 1 /* vector-major:  features[i * d + c] */

/* Feature element types (of the caller's features array). */
#define PLAS_DTYPE_F32 0
#define PLAS_DTYPE_BF16 1 /* bfloat16 as uint16 bit patterns */

/* Storage of the working grids. Arithmetic is float32 either way; with
 * PLAS_STORAGE_BF16 the features are rounded to bfloat16 (nearest, ties to
 * even) on entry and every blurred grid is rounded when stored, which halves
 * the bytes each reorder moves. */
#define PLAS_STORAGE_F32 0
#define PLAS_STORAGE_BF16 1

/* The target's low-pass filter (Sec. 3.1 names a Gaussian filter of radius
 * phi without its kernel). PLAS_FILTER_BOX: one box (mean) pass of
 * half-width r = floor(phi) per axis, the window clipped to the grid.
 * PLAS_FILTER_BOX3: the same box pass three times per axis, rows then
 * columns: a Gaussian-like kernel of variance r(r+1) per axis and support
 * 3r (repeated uniform filters, Wells 1986); three times the blur work.
 * Sorts, batches and servers take either; the energy query uses the box. */
#define PLAS_FILTER_BOX 0
#define PLAS_FILTER_BOX3 1

/* Largest channel count d. */
#define PLAS_MAX_CHANNELS 64

typedef struct plas_context* plas_handle;

/*
 * Where a sort stopped: after params->max_reorders reorders, or at the end of
 * its schedule (done). Passed back as params->resume, with the stopped sort's
 * permutation as params->init_perm and the same features, side, seed and
 * other parameters, it continues the sort, which then ends with the
 * permutation, reorder count, energy and per-level statistics of the sort run
 * without a stop. The resumed sort's trace is indexed by level from level 0:
 * entries levels_done onwards hold the levels it ran (the level it resumed in
 * with its whole count, the reorders before the stop included), the entries
 * before them are zero, so stitching the first levels_done entries of the
 * earlier trace in front gives the uninterrupted sort's trace. The fields are
 * the state of the Sec. 3.1 controller (radius level, block shift and stall
 * test); a caller stores and returns them unchanged.
 */
typedef struct {
    uint32_t struct_size;    /* sizeof(plas_sort_checkpoint) */
    int32_t done;            /* nonzero: the schedule has ended, nothing is left to run */
    int64_t reorders;        /* reorders run so far */
    uint64_t shift_draws;    /* block shifts drawn so far */
    int32_t level;           /* radius level the next reorder belongs to */
    int32_t levels_done;     /* levels before it that ran at least one reorder */
    int32_t dy, dx;          /* that level's current block shift */
    int32_t has_prev;        /* the level has an energy to compare the next one with */
    int32_t just_shifted;    /* the last reorder stalled and the shift was redrawn */
    uint64_t energy_prev;    /* the energy compared with */
    uint64_t energy_last;    /* integer energy after the last reorder */
    int64_t level_reorders;  /* reorders of the current level so far */
    uint64_t level_moved;    /* cells moved in the current level so far */
} plas_sort_checkpoint;

/*
 * Sort parameters. Defaults (plas_sort_params_init) follow Sec. 3.1:
 * radius decay 0.95, a 0.01 % improvement threshold, blocks of at least 16,
 * start radius side/2 - 1.
 */
typedef struct {
    uint32_t struct_size;    /* sizeof(plas_sort_params); set by plas_sort_params_init */
    uint32_t inv_threshold;  /* M: a reorder improves if E_prev - E >= ceil(E_prev / M); 10000 */
    uint64_t seed;           /* names every random draw (start, grouping, shifts) */
    double radius_decay;     /* phi <- decay * phi at each level; 0.95; must be in (0, 1) */
    double start_radius;     /* <= 0: side/2 - 1; raised to 1 if below */
    int64_t max_reorders;    /* 0: run the whole schedule; > 0: stop after this many reorders */
    const int32_t* init_perm;/* device int32[n] start arrangement (gather form), or NULL for the seeded random start */
    int32_t min_block;       /* smallest block side; 16 */
    int32_t profile;         /* nonzero: time the blur and assignment kernels of every 32nd reorder with HIP events (fills *_ms and *_launches in stats) */
    int32_t reorders_per_sync; /* reorders queued between checks of the device's done flag; 0: library default */
    int32_t storage;         /* PLAS_STORAGE_F32 (default) or PLAS_STORAGE_BF16 */
    int32_t filter;          /* PLAS_FILTER_BOX (default) or PLAS_FILTER_BOX3 */
    int32_t reserved;        /* 0 */
    const plas_sort_checkpoint* resume; /* host, or NULL for a new sort; needs init_perm (plas_sort only) */
} plas_sort_params;

/* One radius level of a finished sort. */
typedef struct {
    double phi;            /* real radius */
    int32_t r;             /* blur half-width floor(phi) */
    int32_t beta;          /* block side */
    int64_t reorders;      /* reorders run at this level */
    uint64_t energy_fixed; /* integer energy after the level's last reorder */
    uint64_t moved;        /* cells that changed place over the level */
} plas_level_stat;

typedef struct {
    uint32_t struct_size;   /* sizeof(plas_sort_stats); the caller sets it */
    int32_t levels;         /* levels that ran at least one reorder */
    int64_t reorders;       /* blockwise assignments run in total */
    uint64_t energy_fixed;  /* integer energy after the last reorder */
    int32_t scale_shift;    /* s: energies are sums of floor(d * 2^s) */
    int32_t trace_len;      /* entries written to trace */
    double energy;          /* energy_fixed * 2^-s / n: mean squared distance to the target */
    plas_level_stat* trace; /* caller-owned host array, may be NULL */
    int32_t trace_cap;      /* its capacity */
    int32_t reserved;
    /* With params->profile: device time summed over the timed launches (every
     * 32nd reorder slot of each chunk; each event costs device time, so not
     * every one is timed),
     * and how many launches that was. Average = *_ms / *_launches. */
    double blur_ms;         /* both blur passes */
    int64_t blur_launches;  /* passes (two per reorder, six with PLAS_FILTER_BOX3) */
    double assign_ms;       /* assignment kernel */
    int64_t assign_launches;
    double total_ms;        /* wall time of the whole call */
    plas_sort_checkpoint* checkpoint; /* caller-owned host struct, or NULL: where the sort stopped */
} plas_sort_stats;

int32_t plas_get_abi_version(void);

/* Fill p with the defaults above. Returns PLAS_ERR_INVALID_ARGUMENT for NULL. */
int32_t plas_sort_params_init(plas_sort_params* p);

/* Create a context on HIP device `device`. The device workspace is allocated
 * on first use and kept, grown as needed, until plas_destroy. */
int32_t plas_create(plas_handle* out, int32_t device);

/* Release the context and its workspace. NULL is allowed. */
int32_t plas_destroy(plas_handle h);

/* Order all further work on `stream` (a hipStream_t; NULL = the null
 * stream). Python passes torch.cuda.current_stream().cuda_stream. */
int32_t plas_set_stream(plas_handle h, void* stream);

/*
 * Sort (Sec. 3.1). features: device array of n = side^2 vectors of d
 * channels (1 <= d <= PLAS_MAX_CHANNELS) in `layout`, element type `dtype`;
 * read only. perm_out: device int32[n], written in gather form. stats: host
 * memory or NULL. The call returns when the sort has finished on the device.
 * Deterministic: the same inputs, seed and storage give the same permutation,
 * equal bit for bit to the CPU oracle's for that storage.
 */
int32_t plas_sort(plas_handle h, const void* features, int64_t n, int32_t d, int32_t side,
                  int32_t layout, int32_t dtype, const plas_sort_params* params,
                  int32_t* perm_out, plas_sort_stats* stats);

/*
 * Energy of an arrangement (the distance of Sec. 3.1 that the sort
 * minimises): arranged = features[perm] (perm: device int32[n] in gather
 * form, or NULL for the identity), target = box blur of half-width `radius`
 * (>= 0), energy = sum over cells of floor(d(arranged[p], target[p]) * 2^s),
 * with s derived from the (stored) features' per-channel ranges, grids held
 * in `storage`. Host outputs may be NULL. energy_mean = energy * 2^-s / n.
 */
int32_t plas_grid_energy(plas_handle h, const void* features, const int32_t* perm, int64_t n,
                         int32_t d, int32_t side, int32_t layout, int32_t dtype, int32_t storage,
                         int32_t radius, uint64_t* energy_fixed, int32_t* scale_shift,
                         double* energy_mean);

/*
 * plas_grid_energy for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid hipMalloc): the same arguments and
 * results, computed in a static device
 * array of about 50 MB that the library holds on each GPU it runs on until
 * the process ends. Limit: n <= 65536 cells (side <= 256), else
 * PLAS_ERR_INVALID_ARGUMENT. The call allocates nothing (no hipMalloc,
 * hipFree or memset; it does synchronise h's stream to read its results).
 * Every call on one GPU shares that array: calls that overlap on a GPU (other
 * threads, other streams) race; each call leaves its data there.
 */
int32_t plas_grid_energy_noalloc(plas_handle h, const void* features, const int32_t* perm, int64_t n,
                                 int32_t d, int32_t side, int32_t layout, int32_t dtype, int32_t storage,
                                 int32_t radius, uint64_t* energy_fixed, int32_t* scale_shift,
                                 double* energy_mean);

/*
 * VAD, the sort-quality measure of App. C: the population variance of the
 * absolute differences |a - b| between the values of right and down
 * neighbouring cells (no wrap-around) of the arranged grid
 * features[perm] (perm: device int32[n] in gather form, or NULL for the
 * identity), over every channel, computed in float64 in two passes (mean,
 * then mean squared deviation). Lower is smoother. vad: host output.
 */
int32_t plas_vad(plas_handle h, const void* features, const int32_t* perm, int64_t n, int32_t d,
                 int32_t side, int32_t layout, int32_t dtype, double* vad);

/* A static string naming a status code. */
const char* plas_status_string(int32_t status);

/* The message of the last failure on h (empty if none). Valid until the next call on h. */
const char* plas_last_error(plas_handle h);

#ifdef __cplusplus
}
#endif
#endif
