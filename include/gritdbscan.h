/*
 * gritdbscan.h -- exact grid DBSCAN on one AMD MI355X (gfx950).
 *
 * The library implements the hot path of GriT-DBSCAN (Huang, Ma, Liu, Liu:
 * "GriT-DBSCAN: A Spatial Clustering Algorithm for Very Large Databases"):
 *
 *   1. grids of side eps/sqrt(d) and their identifiers   (Section 4.1, Eq. (1))
 *   2. radix sort of the points by identifier, runs of   (Section 4.1, Algorithm 1)
 *      equal identifiers = the non-empty grids Gs
 *   3. the grid tree over Gs and, per grid, the query    (Section 4.2, Algorithms 2-3,
 *      for its non-empty neighbouring grids Nei(g)        Eq. (2))
 *   4. core points: a grid with at least MinPts points   (Section 3.2 and Section 4.4,
 *      is all core; other points count eps-neighbours     step 2)
 *      over Nei(g) with early exit at MinPts
 *   5. merging core grids: the pruned minimum-distance   (Section 4.3, Algorithms 4-5,
 *      test FastMerging, union-find over core grids       Theorems 1-2; the union-find
 *      visited in ascending core-count order              "LDF" variant of Section 5.2)
 *   6. border / noise assignment                         (Section 3.2, Section 4.4 step 4)
 *
 * The result equals DBSCAN as Definitions 1-5 (Section 3.1) define it
 * (Theorem 4), with canonical labels:
 *   - a cluster's id is the smallest input index among its core points;
 *   - a non-core point within eps of some core point joins the cluster of
 *     its lowest-index core neighbour; every other point is noise (-1).
 * Core flags and labels are therefore unique and bit-exact.
 *
 * Input rules: coordinates are float32 holding integers with |x| <= 2^24;
 * eps is a positive integer (so eps^2 is exact); eps <= GD_EPS_MAX takes
 * 32-bit squared distances, a larger eps 64-bit ones (any eps above 2^27
 * clusters as 2^27 does: valid points are never further apart);
 * 1 <= d <= GD_D_MAX; the packed grid identifier (sum over dimensions of
 * the bit length of the largest identifier) must fit 128 bits (identifiers
 * of up to 64 bits are one word, wider ones two).
 *
 * Every entry point returns a gd_status.  On failure the outputs are
 * unspecified and gd_last_error() describes the failure; the context stays
 * usable.  One context per host thread; calls on one context are serial.
 */
#ifndef GRITDBSCAN_H
#define GRITDBSCAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GD_D_MAX 8
#define GD_EPS_MAX 21845 /* largest eps of the 32-bit distance path: 9 eps^2 <
                            2^32, so squared distances between points of
                            neighbouring grids fit 32 bits exactly */

typedef enum {
    GD_OK = 0,
    GD_EINVAL = -1,       /* bad argument: NULL pointer, n < 0, d out of range,
                             eps not a positive integer, minpts < 1          */
    GD_ERANGE = -2,       /* a coordinate is not an integer of magnitude <= 2^24,
                             or identifiers need > 128 bits                  */
    GD_ENOMEM = -3,       /* device workspace could not be allocated (or the
                             context's workspace limit would be exceeded)     */
    GD_EDEVICE = -4,      /* a HIP runtime call failed                        */
    GD_EUNSUPPORTED = -5  /* valid input outside what the library handles    */
} gd_status;

typedef struct gd_ctx gd_ctx;

/* Counters of the last dbscan() call (filled when stats are enabled, see
 * gd_set_option(GD_OPT_STATS)); sizes are always filled. */
typedef struct {
    int64_t n;                 /* points */
    int32_t d;
    int32_t key_bits;          /* bits of the packed grid identifier */
    int64_t grids;             /* |Gs|: non-empty grids */
    int64_t neighbor_entries;  /* sum over grids of |Nei(g)| */
    int64_t core_points;
    int64_t core_grids;
    int64_t dense_grids;       /* grids with >= MinPts points (all core) */
    int64_t max_grid_points;
    int64_t merge_pairs;       /* core-grid pairs considered by the merge step */
    int64_t merge_skipped;     /* pairs skipped: already in the same set */
    int64_t merge_tests;       /* FastMerging calls */
    int64_t merge_yes;         /* FastMerging calls that answered yes */
    int64_t merge_iterations;  /* sum of FastMerging iterations (kappa) */
    int64_t merge_max_iterations;
    int64_t merge_distances;   /* point-to-point distances evaluated by FastMerging */
    int64_t core_distances;    /* distances evaluated while marking core points */
    int64_t border_points;
    int64_t noise_points;
    int64_t clusters;
    int64_t merge_set_points;  /* sum over FastMerging calls of |s_i| + |s_j| */
    int64_t graph_replays;     /* 1 if the call replayed a captured HIP graph
                                  (then only the size fields are filled) */
    int64_t core_candidates;   /* candidate points streamed while marking core
                                  points (once per batch of 64 queries) */
    int64_t core_neighbor_grids; /* neighbour grids opened while marking */
    int64_t neighbor_walk;     /* 1 if the consumers walked the grid tree themselves
                                  (GD_OPT_NEIGHBOR_MODE): neighbor_entries then
                                  counts only the lists of grids with more than 8
                                  core points */
} gd_stats;

/* Create a context bound to HIP device `device` (the caller's current device
 * is not changed permanently).  The caller owns *ctx and frees it with
 * gd_destroy.  Returns GD_EINVAL for a NULL ctx or a bad device index. */
int gd_create(gd_ctx **ctx, int device);

/* Release the context and all device memory it holds.  NULL is a no-op. */
void gd_destroy(gd_ctx *ctx);

/*
 * dbscan: cluster n points of dimension d (Algorithm 6 with the LDF merge
 * order of Section 5.2).
 *
 *   points      DEVICE pointer, n*d float32, row-major (point i at
 *               points[i*d .. i*d+d-1]); integer-valued, |x| <= 2^24.
 *   n           number of points, 0 <= n < 2^31 (n == 0 returns GD_OK).
 *   d           dimension, 1 <= d <= GD_D_MAX.
 *   eps         radius; a positive integer.
 *   minpts      density threshold, >= 1 (|N(p)| counts p itself).
 *   labels      DEVICE pointer, n int32 out: cluster id (smallest input index
 *               of the cluster's core points) or -1 for noise.
 *   core_flags  DEVICE pointer, n uint8 out: 1 core, 0 not core.
 *   stream      hipStream_t to run on (NULL: the default stream).
 *
 * The call is synchronous: it returns after the results are written.  The
 * caller owns points, labels and core_flags; the context owns its
 * workspace, which grows on demand and is kept for later calls.
 *
 * Errors (outputs unspecified, message in gd_last_error): GD_EINVAL for
 * bad sizes, a non-integer or non-positive eps, minpts < 1 or NULL
 * pointers; GD_ERANGE for a coordinate that is not a finite integer of
 * magnitude <= 2^24, or for grid identifiers that would need more than 128
 * bits (eps too small for the data's extent); GD_ENOMEM if the workspace
 * cannot be allocated or exceeds GD_OPT_WORKSPACE_LIMIT; GD_EDEVICE for a
 * failed HIP call.
 *
 * Core sets of more than 262144 points (beyond the merge kernels' LDS
 * bitmaps) are merged by a second pass with bitmaps in device memory; such
 * calls run eagerly (no graph replay).
 */
int dbscan(gd_ctx *ctx, const float *points, int64_t n, int32_t d, double eps,
           int32_t minpts, int32_t *labels, uint8_t *core_flags, void *stream);

/*
 * dbscan_noalloc: dbscan() for callers that cannot allocate device memory
 * (tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * result and errors as dbscan(); the call itself allocates and frees
 * nothing: every workspace buffer is carved from one fixed array of
 * GD_NOALLOC_SCRATCH_BYTES bytes per device, part of the library's device
 * code and held until the process ends (its device address is looked up by
 * gd_create).  The context must exist already.  Like dbscan() the call
 * reads counts back to the host between phases, so it cannot itself be
 * recorded into a HIP graph.
 *
 * Limits: the workspace of one call must fit the array (about 230 bytes per
 * point at d = 3 plus 4 bytes per neighbour-list entry and the output hash
 * table: roughly a million points of clustered 3-D data); a larger input
 * returns GD_ENOMEM with the sizes in gd_last_error(), before any kernel
 * runs, or once the neighbour-list total is known.  Every call on one
 * device shares that device's array, and it keeps the last call's contents:
 * calls that overlap on one device (several host threads, or several
 * streams without ordering between them) race and must not be made.  The
 * call never captures or replays a graph.
 */
#define GD_NOALLOC_SCRATCH_BYTES (256ull << 20)
int dbscan_noalloc(gd_ctx *ctx, const float *points, int64_t n, int32_t d, double eps, int32_t minpts,
                   int32_t *labels, uint8_t *core_flags, void *stream);

/* One instance of a batch (dbscan_batched).  Pointers are DEVICE pointers
 * with the same meaning as dbscan()'s arguments. */
typedef struct {
    const float *points;   /* n*d float32 row-major, integer-valued, |x| <= 2^24 */
    int64_t n;
    int32_t d;             /* 1 <= d <= GD_D_MAX; instances may differ */
    int32_t minpts;        /* >= 1 */
    double eps;            /* positive integer */
    int32_t *labels;       /* n int32 out: smallest core index of the cluster
                              (an index into this instance's points) or -1 */
    uint8_t *core_flags;   /* n uint8 out */
} gd_instance;

#define GD_BATCH_MAX 65536

/*
 * dbscan_batched: cluster `count` independent instances (HOST array of
 * descriptors) in one pass of the pipeline: every phase is launched once for
 * the whole batch.  Each instance gets exactly the result dbscan() would
 * give it.  The instances' points, labels and flags are DEVICE memory owned
 * by the caller; the sum of n must stay below 2^31.  Synchronous on
 * `stream`.  On error no output is valid; gd_last_error() names the first
 * offending instance.
 *
 * Graph replay (GD_OPT_GRAPH, on by default for this call): the first call
 * for a batch shape (instance count, each n and d) runs with host
 * synchronisation between phases, then captures a synchronisation-free run,
 * sized from that call's grid, neighbour and core-set counts plus headroom,
 * into a HIP graph on a stream of the context.  Later calls with the same
 * shape replay the graph (any coordinates, eps, MinPts and pointers) after
 * the caller's stream's prior work; a replay whose data outgrow the captured
 * sizes is detected on the device and the call reruns without the graph, so
 * the result is always exact.  Graph replays need no per-call allocation.
 */
int dbscan_batched(gd_ctx *ctx, const gd_instance *inst, int32_t count, void *stream);

/* Options (gd_set_option). */
typedef enum {
    GD_OPT_STATS = 1,         /* 1: count merge/core work into gd_stats (slower) */
    GD_OPT_LDF_ORDER = 2,     /* 1 (default): visit core grids in ascending
                                 core-count order; 0: grid (identifier) order */
    GD_OPT_WORKSPACE_LIMIT = 3,/* bytes of device workspace the context may hold;
                                 0 = unlimited (default)                      */
    GD_OPT_TIMING = 4,        /* 1: record HIP events around every phase on the
                                 call's stream (see gd_get_phase_times)       */
    GD_OPT_GRAPH = 5,         /* graph replay (see dbscan_batched): 0 never,
                                 1 (default) dbscan_batched only, 2 also
                                 dbscan(); calls with GD_OPT_STATS or
                                 GD_OPT_TIMING on always run without it      */
    GD_OPT_TILE_POINTS = 6,   /* points per workgroup of the point-indexed
                                 kernels: a multiple of 256 in [256, 65536]
                                 (default 4096)                               */
    GD_OPT_MERGE_WAVES = 7,   /* waves per workgroup of the FastMerging
                                 kernel: 1, 2 or 4 (default 4)                */
    GD_OPT_NEIGHBOR_MODE = 8, /* how the consumers get Nei(g) (Algorithm 3):
                                 1 lists written out for every grid first;
                                 2 core marking, the merging of core sets of at
                                 most 8 points and border assignment each walk
                                 the grid tree for their own grid (lists only
                                 for grids with more core points: far less
                                 memory, slower); 0 (default) lists, or walks
                                 when the lists would not fit the workspace
                                 (GD_OPT_WORKSPACE_LIMIT, or the fixed array
                                 of dbscan_noalloc).  The result is the same in
                                 every mode.                                   */
    GD_OPT_MERGE_ORDER = 9,   /* order in which core grids are merged: 0 grid
                                 (identifier) order with union-find; 1 (default)
                                 ascending core count with union-find (the LDF
                                 variant, Section 5.2); 2 the breadth-first
                                 searches of Algorithm 6 (Section 4.4), run level
                                 by level from many seeds, on the full lists and
                                 without graph replay or the learned proposal.
                                 GD_OPT_LDF_ORDER sets 1 or 0.  The result is
                                 the same in every order (Theorem 4).         */
    GD_OPT_APPROX_DELTA = 10, /* approximate FastMerging (Section 4.3.3, the
                                 remark on numerical error): an integer delta
                                 in [0, 65535 - GD_EPS_MAX]; 0 (default) is
                                 exact.  With delta > 0 FastMerging answers yes
                                 as soon as it meets a pair within eps + delta
                                 (Pruning keeps eps), so its iterations are
                                 bounded independently of eps and d.  Core
                                 flags and border rules are unchanged; core
                                 grids whose core points come within eps are
                                 always joined, and grids are only joined when
                                 some pair of their core points is within
                                 eps + delta: each cluster is a union of exact
                                 clusters and lies inside one component of the
                                 core points' (eps + delta)-graph.  Labels are
                                 then NOT those of dbscan(): an opt-in mode.  */
    GD_OPT_NEIGHBOR_QUERY = 11, /* how the lists Nei(g) are found: 0 (default)
                                 the grid tree of Algorithm 3, lists ordered by
                                 offset (Eq. (2)) where core marking's early
                                 exit pays for the ordering (at most 2^19 grids
                                 of at least 8 points on average) and in walk
                                 order otherwise; 1 the grid tree, lists in
                                 walk order always; 2 direct hashing of every
                                 candidate identifier with offset < d in a
                                 table of the non-empty grids, lists ordered
                                 by offset (the query the grid tree avoids;
                                 candidates grow as (2 ceil(sqrt(d)) + 1)^d);
                                 3 the grid tree, lists ordered by offset for
                                 at most 2^20 grids whatever their size.
                                 The result is the same for every query.      */
    GD_OPT_GRID_LANES = 12,   /* lanes per grid in the kernels that serve
                                 small grids (the merging of tiny core sets,
                                 border assignment):
                                 0 (default) chooses from the mean list length
                                 and grid size (16 when they are at most 40
                                 entries and 32 points, else 64), 16 (four
                                 grids per wave) or 64 (one).  Same result.   */
    GD_OPT_PACKED_ROWS = 13   /* 1 (default): the radix sort of Algorithm 1
                                 carries each point's low coordinate bits
                                 (beside its index, or inside a two-word
                                 identifier's sort word when both fit 64
                                 bits) and the sorted coordinate rows are
                                 rebuilt in order from them and the grid (for
                                 a single instance with 32-bit identifiers by
                                 the sort's last pass itself); 2: the same,
                                 always with a separate rebuilding pass; 0:
                                 the rows are gathered from the input in
                                 sorted order.  Same result.                   */
} gd_option;

int gd_set_option(gd_ctx *ctx, int option, int64_t value);

/* One configuration tried by gd_autotune. */
typedef struct {
    int32_t tile_points;   /* GD_OPT_TILE_POINTS */
    int32_t merge_waves;   /* GD_OPT_MERGE_WAVES */
    int32_t grid_lanes;    /* GD_OPT_GRID_LANES */
    double ms;             /* best wall time of the call, milliseconds */
} gd_tuning;

/*
 * gd_autotune: time dbscan_batched() on the caller's batch (HOST descriptor
 * array, as for dbscan_batched) under every tunable configuration (tile
 * points 1024/4096 x merge waves 1/2/4 x lanes per small grid 16/64; the
 * median of three calls each, after one untimed call, without graph replay)
 * and keep the fastest in the context.  Every configuration gives the same
 * result; the outputs hold the last run's.  `results` (HOST, up to
 * max_results entries, may be NULL) receives the timings and *n_results
 * their number.
 *
 * With a tuning file (gd_set_tuning_file) the batch's shape key (instance
 * count, total points and largest n rounded to powers of two, the range of
 * d) is looked up first: a stored configuration is applied without timing
 * anything (*n_results = 0); otherwise the search runs and its winner is
 * added to the file.
 */
int gd_autotune(gd_ctx *ctx, const gd_instance *inst, int32_t count, void *stream, gd_tuning *results,
                int32_t max_results, int32_t *n_results);

/*
 * gd_set_tuning_file: the JSON file of tuned configurations gd_autotune
 * reads and extends, an object mapping shape keys to
 * {"tile_points": .., "merge_waves": .., "grid_lanes": .., "ms": ..}
 * (HOST string, copied; NULL or "" switches the file off).  A missing file
 * is created on the first search; an unreadable entry is ignored.
 */
int gd_set_tuning_file(gd_ctx *ctx, const char *path);

/* Copy the counters of the last successful dbscan() call. */
int gd_get_stats(gd_ctx *ctx, gd_stats *out);

/* Phases of dbscan() timed with GD_OPT_TIMING. */
#define GD_PHASE_COUNT 14

/* Device time in milliseconds of each phase of the last dbscan() call made
 * with GD_OPT_TIMING on (HOST array of up to `count` doubles; phases that
 * did not run read 0).  Each phase is bracketed by HIP events on the call's
 * stream, so the figure is the GPU time of its kernels. */
int gd_get_phase_times(gd_ctx *ctx, double *ms, int32_t count);

/* Name of phase i (0 <= i < GD_PHASE_COUNT), or NULL. */
const char *gd_phase_name(int32_t i);

/*
 * Intermediate results of the last successful dbscan() call on this
 * context, for checking each step on its own.  HOST output pointers; any may
 * be NULL.  They stay valid until the next dbscan() call.
 *
 * gd_debug_grids (Section 4.1, Algorithm 1):
 *   *n_grids        number of non-empty grids |Gs|
 *   sorted_index    n: input index of the i-th point in sorted order (points
 *                   sorted by grid identifier, ascending input index within a
 *                   grid: the radix sort is stable)
 *   grid_start      |Gs|+1: first sorted position of each grid
 *   grid_ids        |Gs| x d row-major: identifiers of Eq. (1), grids in
 *                   lexicographic order
 * gd_debug_neighbors (Section 4.2.2, Algorithm 3):
 *   offsets         |Gs|+1 (uint64): Nei(g) of grid g is
 *   neighbors       neighbors[offsets[g] .. offsets[g+1]) (grid indices),
 *                   g itself excluded, ordered by the offset of Eq. (2) when
 *                   the lists were written in that order (see
 *                   GD_OPT_NEIGHBOR_QUERY), else in walk order (first-level
 *                   keys g_1, g_1 + 1, .., g_1 + 3, g_1 - 1, .., g_1 - 3,
 *                   each subtree ascending).
 *                   Needs the lists of every grid (GD_EUNSUPPORTED after a
 *                   call that walked instead, see GD_OPT_NEIGHBOR_MODE).
 * gd_debug_core: core_flags_sorted (n, sorted order), grid_label (|Gs|:
 *   cluster id of a core grid, -1 otherwise).
 */
int gd_debug_grids(gd_ctx *ctx, int64_t *n_grids, uint32_t *sorted_index, uint32_t *grid_start,
                   int32_t *grid_ids);
int gd_debug_neighbors(gd_ctx *ctx, uint64_t *offsets, uint32_t *neighbors);
int gd_debug_core(gd_ctx *ctx, uint8_t *core_flags_sorted, int32_t *grid_label);

/*
 * gd_merge_test: FastMerging (Algorithm 5 with Pruning, Algorithm 4) on
 * caller-given point sets, one answer per pair: 1 iff MinDist(A, B) <= eps
 * (Theorem 2).
 *   points      DEVICE, d x m int32 structure-of-arrays (coordinate k of point
 *               i at points[k*m + i]).
 *   pairs       DEVICE, npairs x 4 uint32: a_begin, a_count, b_begin, b_count
 *               (two runs of points; counts >= 1).
 *   answers     DEVICE out, npairs uint8.
 *   iterations  DEVICE out, npairs uint32 (FastMerging iterations), or NULL.
 * The caller guarantees what holds for core sets of neighbouring grids:
 * every coordinate difference between the two sets, and within a set, is
 * below 2^24 in magnitude and every squared distance is below 2^32 (for
 * eps <= GD_EPS_MAX; above it, differences below 2^25, distances in 64
 * bits).  eps <= 2^27, else GD_ERANGE.
 * Counts must not exceed 262144.  Synchronous on `stream`.
 */
int gd_merge_test(gd_ctx *ctx, const int32_t *points, int64_t m, int32_t d, double eps, const uint32_t *pairs,
                  int64_t npairs, uint8_t *answers, uint32_t *iterations, void *stream);

/*
 * Learned proposal (this project's addition to the method).  A
 * 16 -> 64 -> 64 -> 2 ReLU perceptron scores pairs of neighbouring core
 * grids: output 0 is the logit that they merge, output 1 the logit that
 * FastMerging is cheaper started from the second grid.  With a proposal set,
 * the merge step tests each chunk's remaining pairs in descending merge
 * logit and starts FastMerging on the side and at the point the proposal
 * picks.  FastMerging still decides every pair exactly (Theorem 2): labels
 * and core flags are identical with and without a proposal.
 *
 * Parameter vector (GD_MLP_PARAMS values): W1 [64 x 16] row-major, b1 [64],
 * W2 [64 x 64], b2 [64], W3 [2 x 64], b3 [2]; the blob is these in IEEE
 * binary16, the master copy in float32.
 */
#define GD_MLP_PARAMS 5378
#define GD_MLP_FEATURES 16

/* Use the FP16 blob (HOST, GD_MLP_PARAMS halves) in later dbscan() /
 * dbscan_batched() calls; NULL switches the proposal off. */
int gd_set_proposal(gd_ctx *ctx, const uint16_t *fp16_params);

/*
 * Harvest training pairs from the last successful dbscan() call: core grid
 * pairs (a, b), a < b, each kept when a hash of (a, b, seed) is divisible by
 * keep_mod, at most `cap` of them.  For each pair FastMerging runs from a's
 * first core point (the plain method), from a's and from b's starting
 * candidate.  Outputs (DEVICE): features [cap x 16] FP16, targets [cap x 3]
 * float32 (merged, b-side cheaper, sides differ), costs [cap x 3] float32
 * distance evaluations of the three runs (may be NULL).  *count (HOST)
 * receives the number of pairs written.
 */
int gd_proposal_harvest(gd_ctx *ctx, uint32_t seed, uint32_t keep_mod, int64_t cap, uint16_t *features,
                        float *targets, float *costs, int64_t *count, void *stream);

/*
 * Train the scorer on the GPU: `steps` Adam steps (beta 0.9 / 0.999) over
 * mini-batches of `batch` samples; order (DEVICE, steps*batch indices into
 * the S samples) fixes the batches.  params / adam_m / adam_v (DEVICE,
 * GD_MLP_PARAMS float32 each) are read and updated; adam_t0 is the number of
 * steps they already took.  loss (DEVICE, steps floats) receives each step's
 * mean loss; blob (DEVICE, GD_MLP_PARAMS halves) the final FP16 weights.
 * Either may be NULL.  The forward pass uses the weights rounded to FP16,
 * FP16 inputs and hidden activations, FP32 accumulation.
 */
int gd_mlp_train(gd_ctx *ctx, const uint16_t *features, const float *targets, int64_t S, const uint32_t *order,
                 int32_t steps, int32_t batch, float lr, int32_t adam_t0, float *params, float *adam_m,
                 float *adam_v, float *loss, uint16_t *blob, void *stream);

/* Gradient (DEVICE out, GD_MLP_PARAMS float32) and mean loss (DEVICE out, 1
 * float) of one batch (the samples order[0..batch)), with the training
 * kernel's arithmetic and no update. */
int gd_mlp_grad(gd_ctx *ctx, const uint16_t *features, const float *targets, const uint32_t *order,
                int32_t batch, const float *params, float *grad, float *loss, void *stream);

/* Scorer logits (DEVICE out, B x 2 float32) for features (DEVICE, B x 16
 * FP16) with the FP16 parameter blob (DEVICE). */
int gd_mlp_forward(gd_ctx *ctx, const uint16_t *features, int64_t B, const uint16_t *blob, float *logits,
                   void *stream);

/* Text of the last error on this context ("" if none).  The pointer stays
 * valid until the next call on the context. */
const char *gd_last_error(gd_ctx *ctx);

/* Name of a status code. */
const char *gd_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* GRITDBSCAN_H */
