/*
 * libclue: CLUE per-layer clustering on AMD Instinct MI355X (gfx950).
 *
 * CLUE (Rovere et al., "CLUE: A Fast Parallel Clustering Algorithm for High
 * Granularity Calorimeters in High Energy Physics", arXiv:2001.09761) clusters
 * the hits of each calorimeter layer in five steps:
 *   1. a fixed grid of square tiles per layer (Sec. 2.1, Eq. 1-2);
 *   2. the local density rho_i = sum of w_j over hits within dc (Eq. 3,
 *      Algorithm 1, flat kernel);
 *   3. the nearest-higher nh_i and separation delta_i within
 *      d_m = max(delta_o, delta_c) (Eq. 4, Algorithm 2);
 *   4. seed promotion (rho > rho_c, delta > delta_c), outlier demotion
 *      (rho < rho_c, delta > delta_o) and follower registration (Sec. 2.2,
 *      Eq. 5, Algorithm 3);
 *   5. cluster-index propagation from the seeds down the follower chains
 *      (Sec. 2.2, Algorithm 3); outliers and their descendants are noise.
 *
 * Results are exact functions of the input: densities are float32 sums taken
 * in ascending hit index, "higher" is the strict order on (rho, index),
 * equal distances pick the smaller index, cluster ids count seeds in ascending
 * hit index per event (0..k-1), noise is -1. All hit indices reported (nh,
 * follower lists) are event-local positions in the caller's order.
 *
 * Threading and streams: a context is not thread-safe; use one context per
 * stream (or per serving slot). Every run is enqueued on the caller's HIP
 * stream and returns without waiting; outputs are valid once that stream has
 * reached the end of the run. No host<->device copy happens inside a run.
 *
 * Memory: the caller owns every input and output buffer (device memory, for
 * instance torch tensors); the library never frees them. The context owns a
 * scratch arena sized at creation (the paper allocates once for all events,
 * Sec. 4.2) and grown only by clue_reserve.
 *
 * Errors: every call returns CLUE_OK (0) or a negative code; host-detectable
 * errors are reported synchronously; clue_last_error gives the message.
 */
#ifndef CLUE_H
#define CLUE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CLUE_OK = 0,
  CLUE_ERR_ARG = -1,      /* null pointer, n out of range, invalid parameter */
  CLUE_ERR_CAPACITY = -2, /* run larger than the context's reserved capacity */
  CLUE_ERR_NOMEM = -3,    /* device or host allocation failed */
  CLUE_ERR_HIP = -4,      /* a HIP runtime call failed */
  CLUE_ERR_INPUT = -5,    /* invalid hit data (only detected with CLUE_VALIDATE) */
  CLUE_ERR_BUDGET = -6,   /* arena would exceed the context's HBM budget */
  CLUE_ERR_STATE = -7,    /* call not valid in the context's current state */
  CLUE_ERR_DEVICE = -8    /* the device reported an internal inconsistency */
};

enum {
  /* Check hits on the device before clustering (finite x, y, energy; layer in
   * range; event ids in range and non-decreasing) and synchronise the stream to
   * report CLUE_ERR_INPUT. Without it, invalid hits are clamped into range:
   * memory-safe, result unspecified. */
  CLUE_VALIDATE = 1u,
  /* Keep rho, nh, delta^2 of the last run for clue_get_intermediates. */
  CLUE_KEEP_INTERMEDIATES = 2u,
  /* Eq. 4 literally: j is higher than i only when rho_j > rho_i (ties never
   * higher). Default is the (rho, index) order. For comparison runs only. */
  CLUE_TIE_PAPER_STRICT = 4u,
  /* Skip the explicit follower lists F_i (Eq. 5). The follower relation is
   * still used for labels through the nearest-higher links. */
  CLUE_NO_FOLLOWERS = 8u
};

typedef struct {
  float dc;        /* density cut-off distance (cm), > 0 */
  float rho_c;     /* density threshold for seeds (>) and outliers (<) */
  float delta_c;   /* separation threshold for seeds (>), >= 0 */
  float delta_o;   /* separation threshold for outliers (>), >= 0 */
  float x_min, y_min, x_max, y_max; /* extent of the fixed grid; hits outside
                                       are binned into the edge tiles */
  int32_t n_layers;          /* layer ids in [0, n_layers) */
  float tile_size;           /* grid tile side (cm); <= 0: default */
  int32_t threads_per_query; /* lanes per nearest-higher query (1, 2, 4); <= 0: default */
  uint32_t flags;            /* CLUE_* flags above */
  int32_t kernel;            /* chi of Eq. 3 (Sec. 2.2): CLUE_KERNEL_FLAT (chi = 1),
                                CLUE_KERNEL_GAUSSIAN exp(-d^2 / (2 s^2)) or
                                CLUE_KERNEL_EXPONENTIAL exp(-d / s); rho_i sums
                                fl(chi(d_ij) * energy_j) in ascending j. exp is one
                                fixed binary32 evaluation (Cody-Waite reduction,
                                degree-7 Taylor polynomial; 0 below 2^-125) */
  float kernel_scale;        /* s (cm), > 0 for the Gaussian and exponential kernels */
} clue_params;

enum { CLUE_KERNEL_FLAT = 0, CLUE_KERNEL_GAUSSIAN = 1, CLUE_KERNEL_EXPONENTIAL = 2 };

typedef struct clue_ctx clue_ctx;

/*
 * Create a context on HIP device `hip_device` with scratch for up to
 * `max_hits` hits in up to `max_events` events per run. hbm_budget_bytes > 0
 * caps the arena size (CLUE_ERR_BUDGET if the capacity does not fit); 0 means
 * no cap. Allocates device memory synchronously, once, outside the runs: the
 * paper allocates its device buffers once for all events and leaves that
 * allocation out of its timings (Sec. 4.2). *out is NULL on failure.
 */
int clue_create(clue_ctx **out, const clue_params *p, int hip_device, int64_t max_hits,
                int32_t max_events, uint64_t hbm_budget_bytes);

/* Grow the arena to at least (max_hits, max_events): the one-time
 * allocation of Sec. 4.2 redone for a larger capacity. Synchronous: call it
 * outside timed regions. Invalidates captured graphs (re-captured lazily).
 * CLUE_ERR_ARG for a capacity out of range; CLUE_ERR_BUDGET if the larger
 * arena exceeds the HBM budget (the old arena is kept); CLUE_ERR_NOMEM if its
 * allocation fails (the old arena is already freed: runs are then refused
 * with CLUE_ERR_CAPACITY until a clue_reserve succeeds). */
int clue_reserve(clue_ctx *c, int64_t max_hits, int32_t max_events);

/* Bytes of device memory a context with this capacity allocates (arena plus
 * per-context bookkeeping); for admission control by HBM budget. */
int clue_footprint_bytes(const clue_params *p, int64_t max_hits, int32_t max_events,
                         uint64_t *bytes_out);

/*
 * Cluster one event of n hits (all layers in one structure-of-arrays, Sec. 3):
 * x, y, energy float32[n]; layer int32[n]; outputs cluster_id int32[n] and
 * is_seed uint8[n]. All are DEVICE pointers owned by the caller. `stream` is a
 * hipStream_t (NULL: the default stream). n == 0 is a no-op. Launches one
 * kernel per stage sized to the event ("plain" form).
 */
int clue_run(clue_ctx *c, int64_t n, const float *x, const float *y, const int32_t *layer,
             const float *energy, int32_t *cluster_id, uint8_t *is_seed, void *stream);

/*
 * Cluster a batch of n hits from n_events events in one pass ("batched"
 * form): event int32[n] holds each hit's event id, non-decreasing, in
 * [0, n_events); the other arrays are as in clue_run. Indices and cluster ids
 * are event-local, identical to running each event alone. Sec. 3 processes
 * all layers of one event in each kernel launch; this extends that to many
 * events: one persistent kernel per stage over a device work queue of
 * (event, layer, tile block) items, replayed from a captured HIP graph.
 * Errors as clue_run, plus CLUE_ERR_ARG for a null `event` with n_events > 1;
 * ids out of range or decreasing are caught only with CLUE_VALIDATE (without
 * it the run stays within its buffers, with unspecified results).
 */
int clue_run_batch(clue_ctx *c, int64_t n, int32_t n_events, const int32_t *event, const float *x,
                   const float *y, const int32_t *layer, const float *energy, int32_t *cluster_id,
                   uint8_t *is_seed, void *stream);

/*
 * As clue_run_batch for a contiguous run of events taken from a larger
 * device pool: event ids lie in [first_event, first_event + n_events) and are
 * non-decreasing; results equal clue_run_batch with ids - first_event. Lets
 * a serving loop cluster consecutive pool events with no copy.
 */
int clue_run_batch_range(clue_ctx *c, int64_t n, int32_t first_event, int32_t n_events,
                         const int32_t *event, const float *x, const float *y, const int32_t *layer,
                         const float *energy, int32_t *cluster_id, uint8_t *is_seed, void *stream);

/*
 * Host-resident batched form: the same clustering as clue_run_batch, with
 * every data pointer in HOST memory (the paper's timings include the copies,
 * Sec. 4.2). The events are streamed through the context in chunks of whole
 * events that fit its capacity (max_hits, max_events), so n may exceed
 * max_hits: while chunk k is clustered, chunk k + 1 is copied in and chunk
 * k - 1's results are copied out, on the context's own streams. Pinned host
 * memory (hipHostMalloc) lets the copies overlap the kernels; pageable memory
 * gives the same results with the copies serialised. `event` may be NULL when
 * n_events == 1. Synchronous: returns once cluster_id and is_seed hold every
 * result. The device staging (25 bytes per hit of capacity, two chunks) is
 * allocated on the first call and counted against the HBM budget. Errors: an
 * event larger than max_hits -> CLUE_ERR_CAPACITY; a device-side error of any
 * chunk is returned as clue_status would. Intermediates and follower lists
 * afterwards describe the last chunk.
 */
int clue_run_batch_host(clue_ctx *c, int64_t n, int32_t n_events, const int32_t *event, const float *x,
                        const float *y, const int32_t *layer, const float *energy, int32_t *cluster_id,
                        uint8_t *is_seed);

/*
 * Copy the last run's per-hit intermediates into caller DEVICE buffers, in the
 * caller's hit order: rho float32[n] (Eq. 3), nh int32[n] (event-local, -1 if
 * none), delta2 float32[n] (squared separation, +inf if none). Any pointer may
 * be NULL. Needs CLUE_KEEP_INTERMEDIATES; stream-ordered after the run.
 */
int clue_get_intermediates(clue_ctx *c, float *rho, int32_t *nh, float *delta2, void *stream);

/*
 * Copy the last run's follower lists F_i (Eq. 5) into caller DEVICE buffers:
 * fstart int32[n+1] (CSR offsets over hits in caller order) and flist
 * int32[n] (capacity n; the first fstart[n] entries are the event-local
 * follower indices, ascending within each list).
 * Not available with CLUE_NO_FOLLOWERS. *n_followers_out (host) receives
 * fstart[n] after a stream synchronisation; pass NULL to skip the sync.
 */
int clue_get_followers(clue_ctx *c, int32_t *fstart, int32_t *flist, int64_t *n_followers_out,
                       void *stream);

/* Synchronise `stream`, then return and clear the context's deferred device
 * error (CLUE_ERR_INPUT or CLUE_ERR_DEVICE), or CLUE_OK. */
int clue_status(clue_ctx *c, void *stream);

/* Kernel tuning. Results never depend on it (every candidate the autotuner
 * may pick gives bit-identical outputs); only speed does. */
typedef struct {
  float tile_size;          /* grid tile side (cm); must exceed ~1.002 dc */
  int32_t threads_per_query; /* lanes per full-window nearest-higher query: 1, 2, 4, 8 */
  int32_t block_x, block_y; /* tiles per work item (1..16 each) */
  int32_t lds_cap;          /* hits staged in LDS per work item (64..2048, default
                               960); denser items are split into quarter blocks,
                               then single tiles; a tile still too dense is
                               searched in global memory by a follow-up kernel
                               that spreads its queries over the whole GPU */
  float nh_first_radius;    /* radius (cm) of the first nearest-higher pass; a hit
                               whose nearest-higher lies strictly inside it skips
                               the full d_m search. 0 or >= d_m: single pass */
  int32_t density_quads;    /* 1: merge each 2x2-tile quad once per work item
                               (element ranks by binary search) and scan it per
                               hit; 2: each hit merges its own window lists;
                               3: as 1, one lane merging each quad in order;
                               <= 0 keep */
  int32_t plain_lds_cap;    /* LDS cap of the plain form (clue_run, one event per
                               launch, fewer work items in flight); <= 0 keep
                               (initially the same as lds_cap) */
  int32_t expansion;        /* cluster-id propagation (Sec. 2.2, Algorithm 3):
                               1: every hit follows nearest-higher links to its
                               root (pointer jumping, n-way); 2: one thread per
                               seed walks its follower tree depth first (k-way,
                               as in the paper; builds the follower lists even
                               with CLUE_NO_FOLLOWERS, and may grow the arena);
                               <= 0 keep */
} clue_tuning;

/* Replace the tuning. Fields <= 0 keep their current value, except
 * nh_first_radius where only a negative value keeps it. Synchronous; may
 * grow the arena; invalidates the captured graph. CLUE_ERR_ARG for a tile
 * size the density window cannot use or a block plus halo that is too large
 * (the context keeps its previous tuning). */
int clue_set_tuning(clue_ctx *c, const clue_tuning *t);

/* Current tuning, and the staged halo width in tiles it implies. */
int clue_get_tuning(const clue_ctx *c, clue_tuning *t, int32_t *halo);

/* Bytes of device scratch the no-allocation form holds per device. */
#define CLUE_NOALLOC_SCRATCH_BYTES (64ull << 20)

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. Clusters one
 * event exactly as clue_run does (same kernels, plain launches, identical
 * results for the same parameters and tuning) with no context: its scratch
 * arena is a fixed array of CLUE_NOALLOC_SCRATCH_BYTES in device memory that
 * each device holds from the first call there until the process ends. The
 * call allocates nothing, never synchronises and uses no memset node, so it
 * may be captured into a graph.
 *   p       parameters as for clue_create; CLUE_VALIDATE and
 *           CLUE_KEEP_INTERMEDIATES are refused (they need a context).
 *   t       tuning, or NULL for a fresh context's; fields <= 0 (and a
 *           negative nh_first_radius) keep that default; plain_lds_cap,
 *           when set, is the LDS cap used.
 *   n, x, y, layer, energy, cluster_id, is_seed, stream: as for clue_run
 *           (DEVICE pointers owned by the caller, on the calling thread's
 *           current HIP device; n == 0 is a no-op).
 * Limit: the arena for n hits (53 bytes per hit plus 4 bytes per grid tile,
 * with the follower lists; about 1.2M hits on a 200 x 200 cm, 100-layer grid
 * of 4 cm tiles) must fit the array, else CLUE_ERR_CAPACITY with no launch.
 * Every call on one device shares that array and leaves its contents behind;
 * each run clears what it reads first. Calls that overlap on one device (two
 * streams, two threads) race on it and give undefined results: order them.
 * Errors are returned synchronously (CLUE_ERR_ARG, CLUE_ERR_CAPACITY,
 * CLUE_ERR_HIP); clue_last_error(NULL) gives the message of the calling
 * thread's last failure.
 */
int clue_run_noalloc(const clue_params *p, const clue_tuning *t, int64_t n, const float *x, const float *y,
                     const int32_t *layer, const float *energy, int32_t *cluster_id, uint8_t *is_seed,
                     void *stream);

/* Per-stage timing: when enabled, runs record HIP events between stages on
 * the run's stream (batched runs then launch the stage kernels directly
 * instead of through the graph, with identical kernels and launch shapes).
 * clue_stage_times synchronises on the last run and writes up to `cap`
 * stage durations (ms) and their names; returns the stage count. */
int clue_enable_stage_timing(clue_ctx *c, int enable);
int clue_stage_times(clue_ctx *c, float *ms, const char **names, int cap);

/* Message for the last error on this context (or of the last failed create). */
const char *clue_last_error(const clue_ctx *c);

/* Free the context and its arena. Synchronises the device first. */
void clue_destroy(clue_ctx *c);

#ifdef __cplusplus
}
#endif
#endif /* CLUE_H */
