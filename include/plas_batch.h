/*
 * plas_batch.h -- many PLAS sorts advanced together on one device.
 *
 * A batch runs independent sorts (each one the sort of Sec. 3.1 on its own
 * grid, with its own seed) in lock step: every reorder is one launch of each
 * kernel kind -- controller, blur rows, blur columns, assignment -- covering
 * every sort still running. Small grids then share the device instead of each
 * leaving most of it idle, and the launch count no longer grows with the
 * number of sorts. Each sort keeps its own device-resident state machine
 * (stall test, block shifts, radius schedule); a sort that has finished is
 * dropped from the launches at the next status check.
 *
 * Results: each sort's permutation, reorder count, per-level trace and
 * energy equal, bit for bit, what plas_sort returns for the same features,
 * seed, storage and parameters, whatever else runs in the batch and however
 * the launches are shaped (the tuning table only changes launch shapes).
 *
 * Conventions of plas.h apply (device/host pointers, status codes, one handle
 * per host thread). A batch call is synchronous: it returns when every sort
 * has finished or one has failed.
 */
#ifndef PLAS_BATCH_H
#define PLAS_BATCH_H

#include <stdint.h>

#include "plas.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One sort of a batch. features/layout/dtype/d/side/n as for plas_sort. */
typedef struct {
    const void* features;      /* device, read only */
    int64_t n;                 /* side * side */
    int32_t d;                 /* 1 .. PLAS_MAX_CHANNELS */
    int32_t side;
    int32_t layout;            /* PLAS_LAYOUT_CN or PLAS_LAYOUT_NC */
    int32_t dtype;             /* PLAS_DTYPE_F32 or PLAS_DTYPE_BF16 */
    int32_t storage;           /* PLAS_STORAGE_F32 or PLAS_STORAGE_BF16 */
    int32_t reserved;          /* 0 */
    uint64_t seed;             /* this sort's seed (plas_sort_params.seed) */
    const int32_t* init_perm;  /* device int32[n] start arrangement, or NULL */
    int32_t* perm_out;         /* device int32[n], written in gather form */
    plas_sort_stats* stats;    /* host or NULL (struct_size set by the caller). total_ms is the time
                                  from the start of the call until the host saw this sort finish;
                                  blur/assign times are not filled per sort. */
} plas_batch_item;

/* Launch shape for the sorts whose side lies in [side_lo, side_hi]. */
typedef struct {
    int32_t side_lo;
    int32_t side_hi;
    int32_t blur_waves_per_block; /* staged blur (cells of 16 bytes or more): waves per block, each
                                     walking 64/dp lines; 1, 2 or 4; 0: 2 */
    int32_t assign_blocks;        /* blocks per sort for the assignment; 0: the plas_sort default */
} plas_tune_entry;

typedef struct {
    uint32_t struct_size;          /* sizeof(plas_batch_config); set by plas_batch_config_init */
    int32_t graph;                 /* nonzero: each chunk of reorders is captured once as a HIP graph
                                      and replayed until the set of running sorts changes */
    int32_t reorders_per_sync;     /* reorders between status checks; 0: 32. Rounded up to even with graph. */
    int32_t profile;               /* nonzero: time each launch kind with HIP events (direct launches) */
    int32_t tune_count;            /* entries in tune */
    int32_t reserved;
    const plas_tune_entry* tune;   /* host array; the first entry whose range holds a sort's side
                                      applies; sorts in no range get the defaults. May be NULL. */
} plas_batch_config;

typedef struct {
    uint32_t struct_size;   /* sizeof(plas_batch_stats); the caller sets it */
    int32_t sorts;
    int64_t chunks;         /* status checks */
    int64_t reorder_slots;  /* reorder launch sequences queued */
    int64_t graph_builds;   /* graphs captured and instantiated */
    int64_t launches;       /* kernel launches queued in the reorder loop (graph nodes included) */
    double prepare_ms;      /* ingest, ranges and start arrangements of all sorts */
    double loop_ms;         /* the reorder loop */
    double total_ms;        /* the whole call */
    double step_ms;         /* with config->profile: summed device times per launch kind; the
                               controller step runs at the end of the assignment, so step_ms
                               stays 0 and assign_ms includes it */
    double blur_ms;
    double assign_ms;
} plas_batch_stats;

/* Defaults: direct launches, 32 reorders per check, no tuning table. */
int32_t plas_batch_config_init(plas_batch_config* c);

/*
 * Sort every item (Sec. 3.1). params holds what all sorts share: radius
 * decay, threshold, min_block, start_radius, max_reorders (its seed,
 * init_perm, storage, profile and reorders_per_sync fields are ignored: seed,
 * start arrangement and storage come from each item, the rest from config).
 * params->filter applies to every sort of the batch. Batched sorts start
 * from their items: a params resume returns PLAS_ERR_INVALID_ARGUMENT (here,
 * in plas_autotune_batch and in plas_server_create). A stopped sort's
 * stats->checkpoint is filled as in plas_sort. params and config may be NULL for the defaults; stats may be
 * NULL.
 * Items must not share perm_out buffers. The device memory of a sort
 * (3 grids plus about 8 bytes per cell) is held from its start until it
 * finishes. On a failure no further item is guaranteed to be written.
 */
int32_t plas_sort_batch(plas_handle h, const plas_batch_item* items, int32_t count,
                        const plas_sort_params* params, const plas_batch_config* config,
                        plas_batch_stats* stats);

/*
 * Measure launch shapes for these items and write a tuning table: the items
 * are grouped into side buckets [ceil(2^(b/2)), ceil(2^((b+1)/2)) - 1]; for
 * each bucket, truncated batch sorts of its items (6 reorders at the first,
 * coarsest level and 6 at radius 15) are timed under each candidate blur
 * shape (1, 2, 4 waves per block, grids with cells of 16 bytes or more) and then each
 * candidate assignment block count (default, 256, 1024, 16384), keeping the
 * fastest. graph: as in plas_batch_config. table: host array of cap entries;
 * *entries receives the number written. The items' perm_out contents are
 * overwritten with those of the truncated runs.
 */
int32_t plas_autotune_batch(plas_handle h, const plas_batch_item* items, int32_t count,
                            const plas_sort_params* params, int32_t graph, plas_tune_entry* table,
                            int32_t cap, int32_t* entries);

/* ------------------------------------------------------------------ serving
 *
 * A server is a batch that never closes: jobs are submitted at any time,
 * wait in a first-come queue, and are admitted into the running batch at a
 * reorder boundary as soon as their device memory fits in the server's
 * budget (continuous batching). Each plas_server_step admits what fits, runs
 * one chunk of reorders of every running job, and collects the jobs that
 * finished; their results equal plas_sort's for the same inputs, however
 * the jobs overlapped. A server belongs to one handle and, like it, to one
 * host thread; other calls on that handle are allowed between steps.
 */
typedef struct plas_server* plas_server_handle;

/* Device bytes a job holds while it runs (its grids, permutation, grouping
 * table and small tables), or a negative status for bad arguments. */
int64_t plas_job_footprint(int32_t side, int32_t d, int32_t storage, const plas_sort_params* params);

/* params and config as for plas_sort_batch (NULL: defaults).
 * memory_budget: device bytes that running jobs may hold together (> 0); a
 * job larger than the budget is still admitted when nothing else runs. */
int32_t plas_server_create(plas_handle h, const plas_sort_params* params, const plas_batch_config* config,
                           int64_t memory_budget, plas_server_handle* out);

/* Queue one job. The item's buffers must stay valid until the job is
 * reported finished (features are read when the job is admitted; perm_out
 * and stats are written when it finishes). stats->total_ms becomes the time
 * from submission until the host saw the job finish. job_id receives an
 * increasing identifier. Argument errors are reported here; errors found on
 * admission (e.g. non-finite features) are reported by plas_server_poll. */
int32_t plas_server_submit(plas_server_handle s, const plas_batch_item* item, int64_t* job_id);

/* Admit waiting jobs that fit, run one chunk of reorders of the running
 * jobs (if any) and collect finished ones. running/waiting (may be NULL)
 * receive the counts after the step. An error here (a HIP failure) leaves
 * the server unusable. */
int32_t plas_server_step(plas_server_handle s, int32_t* running, int32_t* waiting);

/* Jobs finished or failed since the last poll: up to cap (id, status) pairs;
 * *count receives how many were written. */
int32_t plas_server_poll(plas_server_handle s, int64_t* job_ids, int32_t* statuses, int32_t cap,
                         int32_t* count);

/* Release the server. Jobs still waiting or running are abandoned (their
 * outputs are not written). NULL is allowed. */
int32_t plas_server_destroy(plas_server_handle s);

#ifdef __cplusplus
}
#endif
#endif
