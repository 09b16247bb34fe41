/*
 * vcm.h -- C-ABI of the MI355X visibility color map (VCM) library.
 *
 * Problem statement (Def. 2.1, target-centric form): given obstacles O and a
 * target T, return a colour c in [0,1] for every viewpoint of a discretised
 * d-dimensional space (d = 2 or 3).  The colour is the visual angle of T
 * (Eq. 1, with the oblique size of Eq. 2) normalised by its largest value,
 * and it is 0 wherever T is not completely visible (obstructed region,
 * Def. 2.3) or outside the field of view (Sec. III-B).  The parameters follow
 * the paper's parameter table (Table 2).
 *
 * Conventions for every entry point:
 *   - Plain C types only.  Each call returns a vcm_status; on failure the
 *     outputs are untouched and vcm_last_error() (thread-local) holds a
 *     message.
 *   - Coordinates are metres.  Every coordinate handed to the library (box
 *     bounds, target centre and sizes, grid origin, and the derived sample
 *     and viewpoint positions) must be a multiple of 2^-8 with magnitude
 *     below 2^14; otherwise VCM_E_INVALID.  This makes float32 hold every
 *     input and every difference exactly, which is what lets the float32 ray
 *     test with its float64 recheck return exact visibility.
 *   - Result buffers are device memory owned by the caller (for example
 *     torch tensors passed by data_ptr()).  The library never frees them.
 *   - `stream` is a hipStream_t cast to void*; NULL means the null stream.
 *     Calls enqueue work on that stream and return without waiting, unless
 *     stated otherwise.
 */
#ifndef VCM_H
#define VCM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VCM_OK = 0,
    VCM_E_INVALID = 1,  /* bad argument; see vcm_last_error()            */
    VCM_E_NOMEM = 2,    /* device or host allocation failed               */
    VCM_E_DEVICE = 3,   /* a HIP call or kernel launch failed             */
    VCM_E_AGAIN = 4,    /* admission refused for now; retry later         */
    VCM_E_NOTFOUND = 5, /* unknown ticket                                 */
    VCM_E_PENDING = 6,  /* request not finished yet                       */
    VCM_E_INTERNAL = 7  /* library bug or request cancelled at shutdown   */
} vcm_status;

/* Message for the calling thread's most recent failure ("" if none). */
const char *vcm_last_error(void);

/* Library version string. */
const char *vcm_version(void);

/* ------------------------------------------------------------ obstacles --- */

/* Obstacles O: closed axis-aligned boxes [lo, hi] (Def. 2.2 treats an
 * obstacle as the set a line of sight must not cut; Def. 3.1 counts touching
 * as blocking).  Host memory, structure of arrays: lo[k][i], hi[k][i] for
 * axis k < dim and box i < n.  For dim == 2 the z arrays are ignored and may
 * be NULL.  The arrays are read during the call only. */
typedef struct {
    int32_t dim;            /* 2 or 3                                        */
    int64_t n;              /* number of boxes, >= 0                         */
    const double *lo[3];
    const double *hi[3];
} vcm_obstacles;

typedef struct {
    double cell_size;       /* column width in metres, a power of two; 0 = automatic */
    int32_t device;         /* HIP device ordinal                            */
    void *stream;           /* stream for the build; NULL = null stream      */
} vcm_index_opts;

typedef struct vcm_index vcm_index;

/* Build the device-resident obstacle index: a uniform grid of vertical
 * columns over the boxes' footprints, each listing the boxes whose footprint,
 * grown by 2^-6 m, overlaps the column, sorted by decreasing top height.
 * It replaces the paper's disk R*-tree (Sec. III-B) and is immutable once
 * built.  Blocks until the index is ready.  *out owns device memory until
 * vcm_free_index. */
vcm_status vcm_build_index(const vcm_obstacles *obstacles, const vcm_index_opts *opts,
                           vcm_index **out);

/* Release an index.  No call that uses it may be in flight. */
vcm_status vcm_free_index(vcm_index *index);

/* Size of the index on the device in bytes, and its column grid. */
typedef struct {
    int64_t n_boxes;
    int64_t n_refs;        /* box references over all columns              */
    int32_t nx, ny;        /* columns                                      */
    double cell_size;
    double origin[2];
    size_t device_bytes;
    double build_ms;       /* wall time of the build                       */
    double kernel_ms;      /* device time of the build kernels             */
    int32_t longest_list;  /* box references in the longest column         */
} vcm_index_info;
vcm_status vcm_index_get_info(const vcm_index *index, vcm_index_info *info);

/* --------------------------------------------------------------- queries --- */
/* (vcm_tune_cell_size, which needs the query type, follows the batches.) */

typedef enum {
    VCM_SEGMENT = 0,   /* 2-D line target (Sec. III uses it for exposition) */
    VCM_BILLBOARD = 1, /* 3-D vertical rectangle                            */
    VCM_CUBE = 2,      /* 3-D axis-aligned cube                             */
    VCM_VIEWER = 3     /* 2-D or 3-D: the viewer of a viewer-centric map    */
} vcm_target_kind;

/* Target T.  Segment: length size[0], lying along the axis orthogonal to
 * normal_axis (0 = x, 1 = y).  Billboard: width size[0] (horizontal, along
 * the other horizontal axis) by height size[1] (z), in the vertical plane
 * orthogonal to normal_axis.  Cube: edge size[0].  T is represented by the
 * centres of a samples_u x samples_v lattice on each facet; a viewpoint sees
 * T only if it sees every live sample (Def. 2.3).  For the cube, a face's
 * samples are live only for viewpoints strictly outside its plane.  The
 * paper's size S in Eq. 1 is the largest of the target's dimensions. */
/* Viewer (Sec. IV-B): the viewer-centric map of a viewer at `center`
 * covers the closed ball of radius d_max = size[0] about it (2^-8 lattice);
 * the size S entering Eq. 1 is the one whose visual angle at d_max is mu,
 * S = 2 d_max tan(mu / 2), and every point is taken to face the viewer (no
 * foreshortening).  One sample, the viewer itself (samples_u = samples_v =
 * 1); a point of the map is seen when the segment to the viewer meets no
 * obstacle (by the symmetry of visibility).  normal_axis / normal_sign
 * orient the field of view (the gaze) and the meridian plane of the MBR and
 * tangent approximations; the pruned methods' cells are the distance rings,
 * one band each.  Points outside the ball get count 0 and colour 0. */
typedef struct {
    int32_t kind;
    int32_t normal_axis;   /* segment, billboard, viewer: 0 or 1            */
    int32_t normal_sign;   /* +1 or -1: orientation of the FOV wedge        */
    int32_t samples_u;     /* 1..64                                         */
    int32_t samples_v;     /* 1..64 (segment: 1)                            */
    double center[3];
    double size[2];
} vcm_target;

/* Viewpoints: cell centres of an n[0] x n[1] x n[2] lattice over the box
 * [origin, origin + extent]; viewpoint (i, j, k) sits at
 * origin + (2i+1, 2j+1, 2k+1) * extent / (2n) and has linear index
 * i + n[0] (j + n[1] k).  For dim == 2, n[2] must be 1 and z is ignored. */
typedef struct {
    double origin[3];
    double extent[3];
    int32_t n[3];
} vcm_grid;

typedef enum { VCM_BRUTE = 0, VCM_PRUNED_E = 1, VCM_PRUNED_M = 2, VCM_PRUNED_T = 3 } vcm_method;
typedef enum { VCM_FULL = 0, VCM_FRACTION = 1 } vcm_mode;
typedef enum { VCM_BIN_LINEAR = 0, VCM_BIN_LOG = 1 } vcm_bin_scale;

/* Parameters (Table 2 names and defaults where the paper gives them). */
typedef struct {
    double mu_arcmin;      /* angular resolution mu, arcminutes (4)          */
    double near_d0;        /* near-point distance d0, metres (0.25)          */
    double fov_deg;        /* field of view, (0, 360]; below 360, cube
                              targets need a gaze                           */
    int32_t n_bins;        /* colour bins B, 2..256                          */
    int32_t bin_scale;     /* vcm_bin_scale                                  */
    int32_t method;        /* vcm_method                                     */
    int32_t mode;          /* VCM_FULL: the paper's complete-visibility rule;
                              VCM_FRACTION: colour scaled by the visible
                              fraction of live samples                      */
    int32_t theta_blocks;  /* minimum block size, in viewpoints (1)          */
    double recheck_eps;    /* float32 slab-test margin in units of the ray
                              parameter (2^-20); +inf rechecks every test.
                              At least 2^-21: the float32 slab gap carries
                              up to 3.5 * 2^-23 of rounding error, and a
                              smaller margin would let float32 decide rays
                              it cannot decide exactly (VCM_E_INVALID)     */
    int32_t precision;     /* VCM_FP32_RECHECK: float32 ray tests, exact
                              float64 recheck near the boundary, float32
                              measure; VCM_FP64: every ray test exact in
                              float64 and the measure in float64           */
    int32_t gaze;          /* axis of the field-of-view wedge: 0 = the
                              target's normal (normal_axis, normal_sign);
                              +-(1 + k) = the +-k axis (k < dim), which lets
                              the gaze turn without moving the target
                              (Sec. IV-C) and gives cubes a wedge           */
} vcm_params;

typedef enum { VCM_FP32_RECHECK = 0, VCM_FP64 = 1 } vcm_precision;

typedef struct {
    vcm_target target;
    vcm_grid grid;
    vcm_params params;
} vcm_query;

/* Optional counters for one call (collected only when requested). */
typedef struct {
    uint64_t viewpoints;     /* viewpoints in the grid                       */
    uint64_t rays;           /* live samples summed over in-FOV viewpoints   */
    uint64_t box_tests;      /* float32 ray/box slab tests                   */
    uint64_t rechecks;       /* tests sent to the exact float64 predicate    */
    uint64_t fp32_disagree;  /* with recheck_eps = +inf: float32 decisions,
                                taken with the default margin, that differ
                                from the exact predicate (must be 0)        */
    uint64_t columns;        /* grid columns visited                         */
    uint64_t slot_tests;     /* wavefront-level slab tests (64 lanes each)   */
    uint64_t inside_box;     /* viewpoints found inside an obstacle          */
    uint64_t t_fallbacks;    /* VCM_PRUNED_T: viewpoints no tangent trapezoid
                                contained (coloured by their exact cell)    */
    uint64_t records;        /* box records the column scans examined        */
    uint64_t narrow_tests;   /* candidate records checked against the
                                corridor over their own extent along the
                                walk                                        */
    double kernel_ms;        /* device time of the call's kernels            */
    /* Pruned methods only (0 otherwise): */
    double err_signed;       /* Sec. V-A error, sum(c_ref - c) / sum(c_ref),
                                c_ref the brute-force colour (VCM_PRUNED_E)
                                or the VCM_PRUNED_E colour (_M, _T) under
                                the same visibility gate                    */
    double err_abs;          /* the same with |c_ref - c|                    */
    double bound;            /* VCM_PRUNED_M / _T: E_MBR / E_Tangent of
                                Sec. IV-A over the whole space (the printed
                                sum over one meridian quadrant times 4 in
                                2-D, over one half-space times 2 in 3-D)     */
    double bound_measured;   /* the error that bound covers, over this grid:
                                sum over viewpoints within d_max of
                                |V_approx - V_E| (radians, no visibility
                                gate) times the area (2-D) or volume (3-D)
                                of one lattice cell                         */
    uint64_t blocks;         /* visible-region blocks classified (Sec.
                                III-C-1): those of edge 8 and more; below
                                that, tracing replaces classifying (the map
                                is the same)                                */
    uint64_t blocks_decided; /* of which decided as a whole                  */
    uint64_t leaves;         /* theta > 1: smallest blocks (edge theta,
                                rounded down to a power of two) of the
                                undecided classified blocks, traced at their
                                representative viewpoint; theta = 1:
                                viewpoints the blocks left undecided, traced
                                one by one                                  */
} vcm_stats;

/* Results: caller-owned buffers of grid.n[0]*n[1]*n[2] entries.
 *   bin   : colour bin, min(B-1, floor(c' B)) with c' the colour in the
 *           chosen scale (required);
 *   c     : colour in [0, 1] (optional, may be NULL);
 *   count : FRACTION mode: visible live samples; FULL mode: N(q) where
 *           every live sample is visible, else 0 (the walk stops at the
 *           first blocked ray, so a partial count is not known); 0 outside
 *           the FOV (optional, may be NULL).
 *   host  : 0: the buffers are device memory (every entry point);
 *           1: host memory (vcm_compute only): the call computes into
 *           device buffers of its own, copies the maps back and waits for
 *           `stream` before returning. */
typedef struct {
    uint8_t *bin;
    float *c;
    uint16_t *count;
    int32_t host;
} vcm_result;

/* Compute one VCM.  Enqueues on `stream` and returns; the results are ready
 * when the stream reaches this point.  If stats is non-NULL the call also
 * gathers counters, which makes it wait for the stream before returning. */
vcm_status vcm_compute(const vcm_index *index, const vcm_query *query,
                       const vcm_result *result, void *stream, vcm_stats *stats);

/* vcm_compute without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same results as vcm_compute; no statistics.  Its scratch
 * memory (the work-item counters and the pruned methods' block gates) is a
 * static device array of 64 MiB, one per device, held from the first call
 * on that device until the process ends.  A query that needs more scratch
 * than that fails with VCM_E_INVALID before any device work: a brute-force
 * map needs 2 KiB, a pruned map about 4 bytes per viewpoint more (a gate
 * word per viewpoint and the lists of classified and smallest blocks),
 * so grids of up to about 16 million viewpoints.  Every call on
 * one device shares the array, so calls that overlap on a device (other
 * streams, other threads) race; the caller must order them.  Enqueues on
 * `stream` and returns; results as for vcm_compute. */
vcm_status vcm_compute_noalloc(const vcm_index *index, const vcm_query *query,
                               const vcm_result *result, void *stream);

/* ---------------------------------------------------------------- batches --- */

/* Many queries on one index (each query is a Def. 2.1 problem of its own;
 * batching changes how they are scheduled, never their results).  The
 * queries' work is one persistent launch per group of queries that share a
 * precision and a mode, so that maps of very different sizes fill the device
 * together.  queries[i] writes results[i]; every result is bit-identical to
 * what vcm_compute gives for that query alone.  Result buffers must not
 * overlap.  Enqueues on `stream` and returns; with stats non-NULL it waits
 * and reports counters summed over the batch. */
vcm_status vcm_compute_batch(const vcm_index *index, const vcm_query *queries, int32_t nq,
                             const vcm_result *results, void *stream, vcm_stats *stats);

/* A prepared batch: validated queries, their device records and (optionally)
 * the launch sequence captured as a HIP graph, replayed by vcm_batch_run.
 * The queries and result pointers are fixed at creation. */
typedef struct vcm_batch vcm_batch;

typedef struct {
    int32_t chunk;          /* viewpoints per work item, 1..64; 0 = by mode
                               (FULL 64, FRACTION 8)                         */
    int32_t blocks_per_cu;  /* persistent workgroups per CU, 1..16; 0 = default 8 */
    int32_t autotune;       /* 1: at creation, time the candidate shapes
                               (chunk 4/8/16/32/64 x 4/8 workgroups per CU) on a
                               sample of the queries and keep the fastest;
                               an explicit chunk or blocks_per_cu wins.  This
                               runs the kernels and writes result buffers.  */
    int32_t use_graph;      /* 1: capture the launches in a HIP graph         */
} vcm_batch_opts;

typedef struct {
    int32_t chunk;          /* 0: by mode                                    */
    int32_t blocks_per_cu;
    int32_t launches;       /* persistent ray launches per run              */
    int32_t graph;          /* 1 if runs replay a captured graph            */
    uint64_t viewpoints;
    uint64_t work_items;
    size_t device_bytes;    /* records, counters and block gates            */
    double tune_ms;         /* host time spent autotuning                   */
} vcm_batch_info;

/* Create a batch (blocking; allocates its device buffer).  opts may be NULL. */
vcm_status vcm_batch_create(const vcm_index *index, const vcm_query *queries, int32_t nq,
                            const vcm_result *results, const vcm_batch_opts *opts,
                            vcm_batch **out);
/* Enqueue one run of the batch on `stream`.  Runs of one batch must not
 * overlap (they share counters and outputs); order them on one stream. */
vcm_status vcm_batch_run(vcm_batch *batch, void *stream);
vcm_status vcm_batch_get_info(const vcm_batch *batch, vcm_batch_info *info);
/* Wait for the device, then release the batch. */
vcm_status vcm_batch_destroy(vcm_batch *batch);

/* -------------------------------------------------------------- autotuning --- */

/* The column width of the index is a trade-off: narrow columns list fewer
 * boxes that a corridor only grazes, wide columns cost fewer column visits
 * and list each box fewer times.  vcm_tune_cell_size builds the index of
 * `obstacles` at every power of two from cell_min to cell_max, times the
 * given queries on it (one warm-up and `reps` timed runs of the batch, the
 * fastest kept), and returns the fastest width, for vcm_index_opts.cell_size.
 * Blocking; allocates result buffers for the queries for the duration of the
 * call. */
typedef struct {
    double cell_min;    /* smallest candidate width (power of two); 0 = 16   */
    double cell_max;    /* largest; 0 = 128                                 */
    int32_t device;
    int32_t reps;       /* timed runs per width, 1..100; 0 = 2              */
} vcm_tune_opts;

typedef struct {
    double best_cell;
    int32_t n;          /* widths tried (at most 16)                         */
    double cell[16];    /* widths the index used (a grid too fine is coarsened) */
    double ms[16];      /* fastest time of the queries at that width         */
} vcm_tune_result;

vcm_status vcm_tune_cell_size(const vcm_obstacles *obstacles, const vcm_query *queries, int32_t nq,
                              const vcm_tune_opts *opts, vcm_tune_result *out);

/* ---------------------------------------------------------------- serving --- */

/* A server keeps an index resident and serves VCM queries submitted from any
 * thread.  Admission is by device memory: a request's footprint is its result
 * buffers (1 B bin + 4 B colour + 2 B count per viewpoint, for the buffers
 * given), its work record and, for the pruned methods, the workspace of the
 * block hierarchy (4 B per viewpoint and 4 B per listed block);
 * a request is admitted while the footprints of all unfinished requests fit
 * in mem_budget_bytes.  One engine thread batches the admitted requests as
 * they arrive: whenever one of max_inflight launch slots (streams) is free it
 * takes every waiting request, up to max_batch, into one batched launch
 * (vcm_compute_batch), so launches overlap on the device.  Each result is
 * bit-identical to vcm_compute of the same query alone.  The index must
 * outlive the server; result buffers must stay valid until the request is
 * finished (vcm_poll / vcm_wait returns other than VCM_E_PENDING). */
typedef struct vcm_server vcm_server;

typedef struct {
    size_t mem_budget_bytes;  /* 0 = half of the device memory free at creation */
    int32_t max_inflight;     /* launch slots, 1..8; 0 = 2                      */
    int32_t max_batch;        /* requests per launch, 1..4096; 0 = 64           */
    int32_t chunk;            /* launch shape as in vcm_batch_opts; 0 = default */
    int32_t blocks_per_cu;
} vcm_server_opts;

typedef struct {
    double latency_ms;        /* submit to completion seen by the engine      */
    double queue_ms;          /* submit to launch                             */
    uint64_t viewpoints;
} vcm_request_info;

typedef struct {
    uint64_t completed, failed;
    uint64_t rejected;        /* submits refused with VCM_E_AGAIN             */
    uint64_t launches;
    uint64_t viewpoints;      /* of completed requests                        */
    double p50_ms, p99_ms, max_ms;   /* latency of completed requests (nearest rank) */
    double requests_per_s;    /* completed / (last completion - first submit) */
    double viewpoints_per_s;
    size_t mem_in_use, mem_peak, mem_budget;
} vcm_server_stats;

vcm_status vcm_server_create(const vcm_index *index, const vcm_server_opts *opts,
                             vcm_server **out);
/* Validate and admit a query.  VCM_E_AGAIN: the budget is in use now, retry
 * later (nothing was queued); VCM_E_INVALID: the query is invalid or larger
 * than the whole budget.  On VCM_OK, *ticket names the request. */
vcm_status vcm_submit(vcm_server *server, const vcm_query *query, const vcm_result *result,
                      uint64_t *ticket);
/* VCM_E_PENDING while the request runs.  Once it is finished, returns its
 * status (VCM_OK, or the error that ended it) once, fills info if non-NULL,
 * and forgets the ticket (later polls give VCM_E_NOTFOUND). */
vcm_status vcm_poll(vcm_server *server, uint64_t ticket, vcm_request_info *info);
/* vcm_poll after waiting up to timeout_ms (< 0: no limit) for the request. */
vcm_status vcm_wait(vcm_server *server, uint64_t ticket, int32_t timeout_ms,
                    vcm_request_info *info);
/* Wait until every admitted request has finished (while launches are held,
 * until every launch in flight has finished). */
vcm_status vcm_server_drain(vcm_server *server);
/* hold != 0: admitted requests queue but no launch starts; hold == 0:
 * release, and every free launch slot takes up to max_batch of the queued
 * requests at once.  For callers that gather a burst into as few launches as
 * possible, and for tests of batching that must not depend on timing. */
vcm_status vcm_server_hold(vcm_server *server, int32_t hold);
vcm_status vcm_server_get_stats(vcm_server *server, vcm_server_stats *stats);
vcm_status vcm_server_reset_stats(vcm_server *server);
/* Stop the engine: requests not yet launched finish with VCM_E_INTERNAL
 * (their buffers untouched), launches in flight are waited for; then the
 * server is released and its tickets with it. */
vcm_status vcm_server_destroy(vcm_server *server);

/* ------------------------------------------------------ incremental views --- */

/* Incremental processing (Sec. IV-C).  vcm_view_create computes, once, the
 * visibility of every viewpoint of `query` with the field of view at 360
 * degrees (the query's fov_deg and gaze are ignored) and keeps it on the
 * device (4 bytes per viewpoint, 8 for the pruned methods); it blocks until
 * that is done.  vcm_view_render then colours the query's map for a field of
 * view of fov_deg about the given gaze (as in vcm_params) into `result`
 * (device buffers), without tracing a ray: a brute-force map, or a pruned
 * map with theta_blocks = 1, equals vcm_compute of the query with that field
 * of view bit for bit.  A pruned map with larger blocks masks every
 * viewpoint by its own position (vcm_compute would give a smallest block
 * across the wedge its representative's gate).  Enqueues on `stream`.
 * Renders of one view may run one after another on one stream; the index
 * must outlive the view. */
typedef struct vcm_view vcm_view;
typedef struct {
    uint64_t viewpoints;
    size_t device_bytes;
    double create_ms;       /* wall time of vcm_view_create                  */
} vcm_view_info;
vcm_status vcm_view_create(const vcm_index *index, const vcm_query *query, void *stream,
                           vcm_view **out);
vcm_status vcm_view_render(vcm_view *view, double fov_deg, int32_t gaze, const vcm_result *result,
                           void *stream);
vcm_status vcm_view_get_info(const vcm_view *view, vcm_view_info *info);
/* Wait for the device, then release the view. */
vcm_status vcm_view_destroy(vcm_view *view);

/* Approximation error of Sec. V-A between two colour maps of n viewpoints
 * (caller-owned device buffers, one float each), every viewpoint standing
 * for the same area:  out[0] = sum(c_exact - c_approx) / sum(c_exact)
 * (signed), out[1] = sum|c_exact - c_approx| / sum(c_exact).  Both are 0
 * when sum(c_exact) is 0.  Waits for `stream`. */
vcm_status vcm_map_error(const float *c_exact, const float *c_approx, int64_t n, int32_t device,
                         void *stream, double out[2]);

/* Error bounds of the MBR (out[0]) and tangential (out[1]) approximations
 * (Sec. IV-A, the sums E_MBR and E_Tangent) for the query's target size, mu
 * and near point, evaluated as printed: per ring, the number of rings that
 * can be mis-coloured times the number of bands below the stated angle times
 * mu, weighted by the size of each cell of the ring (area in the meridian
 * quadrant for dim 2, volume of revolution about the normal for dim 3).
 * Host computation. */
vcm_status vcm_error_bounds(const vcm_query *query, int32_t dim, double out[2]);

#ifdef __cplusplus
}
#endif

#endif /* VCM_H */
