/*
 * pcms_mls.h -- C interface of the MI355X (gfx950) point-cloud field-transfer
 * library: moving-least-squares ("local weighted polynomial fitting") mapping
 * of fields from a source point cloud to a target point cloud.
 *
 * The operation is the one of the PCMS paper (Merson et al., "PCMS: Parallel
 * Coupler For Multimodel Simulations"), Section 3.2.1, Eq. 1: for every
 * target t_i, the sources selected by a radial cut-off (Section 3.2.1's
 * selection function) are fitted by the weighted, Tikhonov-regularised
 * least-squares polynomial of total degree <= p, and the fit is evaluated at
 * t_i.  Sources are located with a uniform-grid search or a linear
 * bounding volume hierarchy (the two structures Section 3.3 compares); both
 * give the same neighbour lists.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array argument is a DEVICE pointer owned by the caller (for
 *    example torch.Tensor.data_ptr()).  It must stay valid until the work
 *    enqueued on `stream` has completed.  The library never frees caller
 *    memory and keeps no caller pointer past the call.
 *  - Opaque handles (pcms_grid) are owned by the library and released with
 *    their *_free function.
 *  - Points are [n][dim] float64 row-major, dim in 1..5.  Fields are
 *    [n_fields][n] float64 (field-major).  Indices and per-target counts are
 *    int32 (n_src < 2^31).  Coordinates must be finite.
 *  - Every call enqueues on `stream` (NULL = the null stream).  Unless
 *    PCMS_ASYNC is set, the call then waits for the stream and turns the
 *    per-target statuses into its return code.  The transfers without
 *    PCMS_PROFILE (pcms_mls_transfer, pcms_mls_transfer_grid) also run the
 *    target ordering on a library-owned side stream of the calling thread
 *    (one per device, default priority), forked from `stream` with an event
 *    and joined back before the work that reads it, so everything the call
 *    enqueues stays ordered after earlier work on `stream` and before later
 *    work.  For HIP graph capture use pcms_mls_transfer_grid_noalloc (no
 *    allocation, no side stream, no host-to-device copy) or a batch plan,
 *    which captures itself.
 *  - Argument errors are detected on the host before any HIP call and
 *    return PCMS_ERR_ARG.  No C++ exception crosses this interface.  The
 *    last error message of the calling thread is pcms_last_error().
 *
 * Per-target status (uint8): 0 OK; 1 UNDERDETERMINED (fewer than m kept
 * sources: the paper's error condition); 2 SINGULAR (a Cholesky pivot at or
 * below 1e-13 * max diag of the moment matrix -- 4e-6 * max diag in MIXED,
 * whose FP32-accumulated moments resolve nothing finer -- or, in
 * MIXED_REFINE, a refinement correction that stops shrinking); 3
 * RADIUS_EXHAUSTED (growing radius ran out of doublings before reaching the
 * minimum count); bit 0x10 CAPPED (more than k_cap sources were inside the
 * radius; the k_cap nearest by (distance, source index) were kept).  Targets
 * with status 1-3 get NaN outputs.
 */
#ifndef PCMS_MLS_H
#define PCMS_MLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *pcms_stream_t; /* a hipStream_t */

typedef int32_t pcms_status;
#define PCMS_OK 0
#define PCMS_ERR_ARG 1              /* invalid argument, nothing was enqueued */
#define PCMS_ERR_HIP 2              /* a HIP runtime call failed */
#define PCMS_ERR_NOMEM 3            /* device allocation failed */
#define PCMS_ERR_UNDERDETERMINED 4  /* at least one target was underdetermined */
#define PCMS_ERR_SINGULAR 5         /* at least one target had a singular moment matrix */
#define PCMS_ERR_RADIUS_EXHAUSTED 6 /* at least one growing radius ran out of doublings */

#define PCMS_TGT_OK 0
#define PCMS_TGT_UNDERDETERMINED 1
#define PCMS_TGT_SINGULAR 2
#define PCMS_TGT_RADIUS_EXHAUSTED 3
#define PCMS_TGT_CAPPED 0x10

#define PCMS_MAX_DIM 5
#define PCMS_MAX_KCAP 256

/* Radius selection (Section 3.2.1).  The distance is the metric
 * D = sum_k ((t_k - s_k) * g_k)^2 evaluated in FP64 as a fused multiply-add
 * chain in dimension order; a source is selected when D < r^2 (strictly).
 *   FIXED: r is given.
 *   GROW:  r starts at `r`; per target, r^2 doubles until at least `n_min`
 *          sources are inside or `max_iter` doublings are spent (the paper's
 *          "minimum number of source points and an initial radius").
 *   KNN:   r^2 is the k-th smallest D over all sources, so k-1 sources lie
 *          strictly inside (ties aside) and the k-th sits where the weight
 *          vanishes. */
#define PCMS_RADIUS_FIXED 0
#define PCMS_RADIUS_KNN 1
#define PCMS_RADIUS_GROW 2
typedef struct {
    int32_t mode;     /* PCMS_RADIUS_* */
    int32_t k;        /* KNN order, 1 <= k <= n_src */
    int32_t n_min;    /* GROW minimum count, >= 1 */
    int32_t max_iter; /* GROW doublings, >= 0 (40 is a good default) */
    double r;         /* FIXED radius / GROW initial radius, finite, > 0 */
} pcms_radius;

/* Radial weights phi(q), q = sqrt(D) / r (Table 1 of the paper, shape
 * parameter a = 2, plus Wendland C2 (1-q)^4 (4q+1), the default).  Table 1's
 * No_Op (identity, phi = 1 everywhere) weighs the selected sources exactly as
 * Const (phi = 1 inside the radius): only sources strictly inside the radius
 * enter the fit, so the two give the same results.  Multiquadric, thin plate
 * spline and cubic spline are not positive and decreasing on [0, 1) and are
 * not offered as least-squares weights. */
#define PCMS_WEIGHT_WENDLAND_C2 0
#define PCMS_WEIGHT_C4 1
#define PCMS_WEIGHT_GAUSSIAN 2
#define PCMS_WEIGHT_CONST 3
#define PCMS_WEIGHT_IMQ 4
#define PCMS_WEIGHT_NO_OP 5

/* Arithmetic of the moment assembly.
 *   FP64:         everything in FP64.
 *   MIXED:        weights and the moment matrix G = P^T W P in FP32 with FP32
 *                 accumulation; Cholesky, solve and evaluation in FP64.  No
 *                 refinement: the error grows with the conditioning of G.
 *   MIXED_REFINE: FP32 moment matrix and an FP32 Cholesky factor of it as
 *                 the preconditioner of FP64 iterative refinement of the
 *                 shape functional y = G^{-1} e_0, the residual e_0 - G y
 *                 formed in FP64 from FP64 weights and monomials; converges
 *                 to the FP64 result (one or two steps, up to four for
 *                 ill-conditioned targets; a correction that stops
 *                 shrinking marks the target SINGULAR). */
#define PCMS_FP64 0
#define PCMS_MIXED 1
#define PCMS_MIXED_REFINE 2

#define PCMS_ASYNC 0x1u   /* return after enqueue; statuses land in opts.summary */
#define PCMS_PROFILE 0x2u /* time the phases with HIP events (see pcms_last_phase_ms) */
#define PCMS_LBVH 0x4u    /* pcms_mls_transfer, pcms_operator_build: locate sources with
                             an LBVH (pcms_lbvh_build) instead of the uniform grid; calls
                             on a prebuilt handle use the handle's structure */

typedef struct {
    int32_t weight;           /* PCMS_WEIGHT_* */
    int32_t precision;        /* PCMS_FP64 / PCMS_MIXED / PCMS_MIXED_REFINE */
    double lambda;            /* Tikhonov parameter of Eq. 1, >= 0, in the radius-scaled basis */
    uint32_t flags;           /* PCMS_ASYNC | PCMS_PROFILE | PCMS_LBVH (other bits: PCMS_ERR_ARG) */
    int32_t block;            /* threads per workgroup (one per target): 0 = library choice, else 64/128/256 */
    int32_t *summary;         /* device int32[4] or NULL: counts of statuses 1, 2, 3 and CAPPED */
} pcms_mls_opts;

/* Set opts to the defaults (Wendland C2, FP64, lambda 0, synchronous). */
void pcms_mls_opts_default(pcms_mls_opts *opts);

/* ---------------------------------------------------------------------- */
/* Uniform grid (Section 3.3): sources sorted by bucket.                   */
/* ---------------------------------------------------------------------- */
typedef struct pcms_grid pcms_grid;

/* Build a uniform grid over the sources.  The grid keeps its own sorted copy
 * of the coordinates, so `src` may be freed once the stream has passed this
 * call.  inv_scale: HOST float64[dim] metric factors g (NULL = all 1).
 * cell_width: bucket width in metric units (> 0), or 0 to size buckets for
 * about `pts_per_cell` sources each (pts_per_cell <= 0 picks 2^dim).  In
 * two or more dimensions, dimension 0 (along which a row of buckets is
 * contiguous in sorted order) is then cut into 4 slices per bucket width,
 * or into 1, 2, 8 or 16 if the environment variable PCMS_ROW_SLICES says
 * so (fewer if the bucket count would exceed 2 n_src + 64; then the width
 * grows): a search pays per row of buckets, and the slices let each row's
 * range follow the ball's chord.  Every grid the library builds (one-shot
 * calls, operators, batches) is sliced the same way.
 * Reusable across transfers of changing fields (the paper's case of a static
 * discretisation queried many times). */
pcms_status pcms_grid_build(const double *src, int64_t n_src, int32_t dim, const double *inv_scale,
                            double cell_width, double pts_per_cell, pcms_stream_t stream,
                            pcms_grid **out);
pcms_status pcms_grid_free(pcms_grid *grid);

/* Build a linear bounding volume hierarchy over the sources (Section 3.3's
 * alternative to the uniform grid) and return it as a pcms_grid handle that
 * every call taking a grid accepts (pcms_neighbors, pcms_mls_transfer_grid,
 * pcms_mls_transfer_grid_noalloc) and pcms_grid_free releases.  The sources
 * are sorted by the 32-bit Morton code of their position in the bounding box
 * (32 / dim bits per coordinate); the leaves are the largest subtrees of the
 * radix tree over the sorted codes that hold at most max_leaf sources
 * (aligned Morton cells: compact boxes at any density), and a binary radix
 * tree over the leaves' codes joins them, with FP32 boxes rounded outward.
 * max_leaf: 1..64, or 0 for the default (4; the one-shot PCMS_LBVH calls
 * use the default unless the environment variable PCMS_LBVH_LEAF sets
 * another).  A search visits the leaves within reach of its
 * ball and applies the grid's selection to their sources, so neighbour lists
 * and statuses are bitwise those of the uniform grid; fitted values agree to
 * rounding (the moment sums run in Morton order instead of bucket order).
 * inv_scale: HOST float64[dim] metric factors (NULL = all 1).  The handle
 * holds its own sorted coordinates. */
pcms_status pcms_lbvh_build(const double *src, int64_t n_src, int32_t dim, const double *inv_scale,
                            int32_t max_leaf, pcms_stream_t stream, pcms_grid **out);

/* 1 if the handle was built by pcms_lbvh_build, 0 otherwise (or NULL). */
int32_t pcms_grid_is_lbvh(const pcms_grid *grid);

/* Neighbour lists (Section 3.2.1 selection set, capped).  For target i:
 * nbr[i*k_cap + e], e < n_kept[i], are the kept original source indices in
 * ascending order (entries past n_kept are unspecified); n_found[i] is the
 * count strictly inside the radius before the cap; r2[i] the squared radius;
 * status[i] as above (UNDERDETERMINED is not judged here).  n_found, r2 and
 * status may be NULL.  1 <= k_cap <= 256. */
pcms_status pcms_neighbors(const pcms_grid *grid, const double *tgt, int64_t n_tgt,
                           const pcms_radius *radius, int32_t k_cap, pcms_stream_t stream,
                           int32_t *nbr, int32_t *n_kept, int32_t *n_found, double *r2,
                           uint8_t *status);

/* Field transfer (Section 3.2.1, Eq. 1), one shot: builds the grid, searches,
 * fits and evaluates.  src_vals [n_fields][n_src]; tgt_vals [n_fields][n_tgt]
 * receives the fitted values (NaN for failed targets); status [n_tgt] may be
 * NULL.  basis_degree 0..2 (m = C(dim+degree, degree) monomials in
 * target-centred, radius-scaled coordinates); m <= k_cap <= 256.
 * inv_scale: HOST float64[dim] or NULL. */
pcms_status pcms_mls_transfer(const double *src, int64_t n_src, int32_t dim, const double *src_vals,
                              int32_t n_fields, const double *tgt, int64_t n_tgt,
                              int32_t basis_degree, const pcms_radius *radius, int32_t k_cap,
                              const double *inv_scale, const pcms_mls_opts *opts,
                              pcms_stream_t stream, double *tgt_vals, uint8_t *status);

/* Same on a prebuilt grid (its metric and sorted sources are reused). */
pcms_status pcms_mls_transfer_grid(const pcms_grid *grid, const double *src_vals, int32_t n_fields,
                                   const double *tgt, int64_t n_tgt, int32_t basis_degree,
                                   const pcms_radius *radius, int32_t k_cap,
                                   const pcms_mls_opts *opts, pcms_stream_t stream,
                                   double *tgt_vals, uint8_t *status);

/* ---------------------------------------------------------------------- */
/* Precomputed transfer operator: with the source and target clouds fixed, */
/* the fit of Section 3.2.1, Eq. 1 is linear in the field values,          */
/* fhat_i = sum_j N_ij f_j with the shape functions                        */
/* N_ij = w_j p(xi_j)^T (P^T W P + lambda I)^{-1} p(0) of target i's kept  */
/* sources.  Building N once and applying it to each new set of fields is  */
/* the coupling pattern of a static discretisation exchanged every step.   */
/* ---------------------------------------------------------------------- */
typedef struct pcms_operator pcms_operator;

/* Build the operator of the sources [n_src][dim] and targets [n_tgt][dim]
 * (same arguments and checks as pcms_mls_transfer, without field values):
 * the search, the moment assembly and solve of opts.precision, and the
 * shape functions of every kept source (in FP64).  The operator is library
 * owned (pcms_operator_free) and holds, per target, at most
 * pcms_operator_width(op) <= k_cap weights and source indices (the width is
 * k_cap, or k + 8 for a KNN radius with k + 8 < k_cap); the coordinates are
 * not kept.  status [n_tgt] (may be NULL) and the return code are as for
 * pcms_mls_transfer; on such a status code *out is still set (failed targets
 * give NaN when applied).  With PCMS_LBVH the search runs on an LBVH (same
 * kept sources; weights equal to rounding). */
pcms_status pcms_operator_build(const double *src, int64_t n_src, int32_t dim, const double *tgt,
                                int64_t n_tgt, int32_t basis_degree, const pcms_radius *radius,
                                int32_t k_cap, const double *inv_scale, const pcms_mls_opts *opts,
                                pcms_stream_t stream, uint8_t *status, pcms_operator **out);

/* tgt_vals[l][i] = sum over target i's kept sources j of N_ij src_vals[l][j]
 * for l < n_fields (layouts of pcms_mls_transfer; src_vals of the n_src
 * sources of the build), NaN for failed targets.  Enqueues one kernel on
 * `stream` and returns. */
pcms_status pcms_operator_apply(const pcms_operator *op, const double *src_vals, int32_t n_fields,
                                pcms_stream_t stream, double *tgt_vals);

/* Copy the operator to DEVICE arrays in original target order: n_kept[i]
 * (-1 for a failed target) and, for e < n_kept[i], cols[i*stride + e] (source
 * index) and weights[i*stride + e] (N); every other entry of the stride-long
 * row is written as -1 and 0.  stride >= pcms_operator_width(op), else
 * PCMS_ERR_ARG.  cols and weights may be NULL.  Entries come in search order,
 * not sorted by source index. */
pcms_status pcms_operator_export(const pcms_operator *op, int32_t stride, pcms_stream_t stream,
                                 int32_t *n_kept, int32_t *cols, double *weights);

/* Slots per target of the operator (0 for NULL). */
int32_t pcms_operator_width(const pcms_operator *op);

/* Release the operator (waits for the device first). */
pcms_status pcms_operator_free(pcms_operator *op);

/* ---------------------------------------------------------------------- */
/* Batched transfer: many independent problems of uneven size, dimension,  */
/* degree and field count (each one the operation of pcms_mls_transfer)    */
/* executed as work items grouped by class, largest first, with every      */
/* stage captured once into a HIP graph and replayed.                      */
/* ---------------------------------------------------------------------- */

/* One problem of a batch.  Every pointer is a DEVICE pointer except
 * inv_scale (HOST float64[dim] or NULL), and must stay valid, at the same
 * address, for the life of the plan: a plan replays against these buffers,
 * so new source values written into src_vals between executions are picked
 * up.  Constraints as for pcms_mls_transfer; status may be NULL. */
typedef struct {
    const double *src;        /* [n_src][dim] */
    int64_t n_src;
    int32_t dim;              /* 1..5 */
    int32_t basis_degree;     /* 0..2 */
    const double *src_vals;   /* [n_fields][n_src] */
    int32_t n_fields;         /* >= 1 */
    int32_t k_cap;            /* m..256 */
    const double *tgt;        /* [n_tgt][dim] */
    int64_t n_tgt;            /* >= 0 */
    pcms_radius radius;
    const double *inv_scale;  /* HOST [dim] or NULL */
    double *tgt_vals;         /* [n_fields][n_tgt] */
    uint8_t *status;          /* [n_tgt] or NULL */
} pcms_problem;

/* Batch options.  block (targets per workgroup) and cell_factor (bucket
 * width as a fraction of the radius: of the fixed or initial radius, or of
 * the expected kNN radius) are tuning knobs that change speed, not results;
 * 0 takes the value stored in tune_cache (a file written by pcms_autotune)
 * if given and readable, else the library default. */
typedef struct {
    int32_t weight;           /* PCMS_WEIGHT_* (all problems) */
    int32_t precision;        /* PCMS_FP64 / PCMS_MIXED / PCMS_MIXED_REFINE */
    double lambda;            /* >= 0 */
    int32_t block;            /* 0, 64, 128 or 256 */
    double cell_factor;       /* 0 or in (0, 4] */
    const char *tune_cache;   /* HOST path or NULL */
} pcms_batch_opts;

/* Set opts to the defaults (Wendland C2, MIXED_REFINE, lambda 0, library
 * tuning). */
void pcms_batch_opts_default(pcms_batch_opts *opts);

typedef struct pcms_batch_plan pcms_batch_plan;

/* Plan a batch of n >= 1 problems: validates every problem (an invalid one
 * fails the call with its index in the message), allocates the device
 * workspace of all grids, sorted copies and the work queue (library owned,
 * released by pcms_batch_plan_free), and orders the work items (problem,
 * tile of targets) by estimated cost, largest first.  Nothing is enqueued;
 * the work is captured on the first pcms_batch_plan_exec. */
pcms_status pcms_batch_plan_create(const pcms_problem *problems, int32_t n,
                                   const pcms_batch_opts *opts, pcms_batch_plan **out);

/* Execute the plan on `stream`: every grid build, target ordering and
 * value scatter, then the work queue of (problem, tile of targets) items:
 * one launch per class of problems present (dimension 1-3, degree, metric),
 * each compiled for its class, with one block per item in decreasing order
 * of estimated cost (problems of dimension 4 or 5 run through the
 * one-problem kernel after them).  The first
 * call on a plan with a non-null stream captures the sequence into a HIP
 * graph and later calls replay it (the legacy null stream cannot be
 * captured: there every call enqueues the kernels directly).  summary:
 * DEVICE int32[4] or NULL.  With summary NULL the call waits and returns
 * the batch's status code as pcms_mls_transfer does; with a
 * summary it returns after enqueue and the counts of statuses 1, 2, 3 and
 * CAPPED over all problems land there.  Calls on one plan must not overlap. */
pcms_status pcms_batch_plan_exec(pcms_batch_plan *plan, pcms_stream_t stream, int32_t *summary);

/* Release the plan's workspace and graph (waits for the device first). */
pcms_status pcms_batch_plan_free(pcms_batch_plan *plan);

/* Tuning knobs chosen by pcms_autotune. */
typedef struct {
    int32_t block;
    double cell_factor;
    float ms;                 /* measured time of one execution */
} pcms_tune_result;

/* Time executions of the batch `sample` for each (block, cell_factor) in
 * {64, 128, 256} x {0.6, 0.7, 0.85, 1.0} (weight, precision and lambda from
 * opts) and return the fastest in *out; when cache_path is not NULL it is
 * also written there as a small JSON object that pcms_batch_plan_create
 * reads through pcms_batch_opts.tune_cache.  Runs on `stream` and
 * synchronises it. */
pcms_status pcms_autotune(const pcms_problem *sample, int32_t n, const pcms_batch_opts *opts,
                          const char *cache_path, pcms_stream_t stream, pcms_tune_result *out);

/* ---------------------------------------------------------------------- */
/* Allocation-free transfer on a prebuilt grid.                            */
/* ---------------------------------------------------------------------- */

/* Bytes of the fixed device workspace of pcms_mls_transfer_grid_noalloc. */
#define PCMS_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, checks, results and return codes as pcms_mls_transfer_grid,
 * but the call allocates nothing (no hipMalloc, hipMallocAsync, hipFree or
 * event creation): its workspace -- status counts, target order, sort
 * buffers, bucket-ordered field records and staged outputs, about
 * 8 * (n_src + n_tgt) * (n_fields rounded up to even) + 28 * n_tgt bytes --
 * is a fixed
 * device array of PCMS_NOALLOC_SCRATCH_BYTES per GPU, which the library holds
 * from the moment it is loaded on that GPU until the process ends.  A call
 * needing more returns PCMS_ERR_ARG before any HIP call.  PCMS_PROFILE is
 * rejected (PCMS_ERR_ARG).  Every call on one GPU uses that GPU's one array:
 * calls that overlap on the same GPU (other streams, other threads) race and
 * give wrong results; serialise them.  The grid must be built beforehand
 * (pcms_grid_build allocates). */
pcms_status pcms_mls_transfer_grid_noalloc(const pcms_grid *grid, const double *src_vals,
                                           int32_t n_fields, const double *tgt, int64_t n_tgt,
                                           int32_t basis_degree, const pcms_radius *radius,
                                           int32_t k_cap, const pcms_mls_opts *opts,
                                           pcms_stream_t stream, double *tgt_vals,
                                           uint8_t *status);

/* PCMS_NOALLOC_SCRATCH_BYTES as built into the library. */
size_t pcms_noalloc_scratch_bytes(void);

/* ---------------------------------------------------------------------- */
/* Work-space sizes.                                                       */
/* ---------------------------------------------------------------------- */

/* Device memory of a problem of n_src sources of dimension dim, n_fields
 * fields and n_tgt targets, in bytes.  The library's temporary buffers come
 * from the HIP stream-ordered pool of the current device (hipMallocAsync,
 * which keeps freed blocks cached); callers that reserve that pool, or
 * choose between the allocating and the allocation-free calls, size it from
 * these figures. */
typedef struct {
    size_t grid_bytes;           /* a pcms_grid (held until pcms_grid_free) */
    size_t grid_build_bytes;     /* temporary, during pcms_grid_build */
    size_t transfer_bytes;       /* peak temporary of pcms_mls_transfer (either structure) */
    size_t transfer_grid_bytes;  /* temporary of pcms_mls_transfer_grid (the
                                    work space pcms_mls_transfer_grid_noalloc
                                    needs, <= noalloc_limit to be accepted) */
    size_t operator_apply_bytes; /* temporary of pcms_operator_apply */
    size_t noalloc_limit;        /* PCMS_NOALLOC_SCRATCH_BYTES */
    size_t lbvh_bytes;           /* a pcms_lbvh_build handle */
    size_t lbvh_build_bytes;     /* temporary, during pcms_lbvh_build */
} pcms_workspace;

/* Fills *out (host) for the given sizes; host-only arithmetic, no HIP call.
 * PCMS_ERR_ARG for dim outside 1..5, n_src outside [1, 2^30), n_tgt outside
 * [0, 2^30) or n_fields < 1. */
pcms_status pcms_workspace_query(int64_t n_src, int32_t dim, int32_t n_fields, int64_t n_tgt,
                                 pcms_workspace *out);

/* Phase times in milliseconds of the calling thread's last call made with
 * PCMS_PROFILE, measured with HIP events on that call's stream: [0] grid
 * build, [1] target ordering, [2] field gather into bucket order, [3] the
 * search-and-fit kernel, [4] the transpose of the outputs into field-major
 * order.  Writes min(n, 5) entries to the host array `ms` and returns that
 * count (0 if no profiled call was made).  A profiled call does not wait for
 * its events: they are read when a later profiled call has been enqueued,
 * or here (which waits for them). */
int32_t pcms_last_phase_ms(float *ms, int32_t n);

/* Sums of the phase times (as above) over every profiled call of the
 * calling thread since the last reset, into the host array sum_ms[min(n,
 * 5)] (may be NULL); returns the number of calls summed (-1 on a HIP
 * error).  Waits for the pending events.  reset != 0 clears the sums after
 * reading them. */
int32_t pcms_phase_ms_sum(double *sum_ms, int32_t n, int32_t reset);

/* Library version (major*10000 + minor*100 + patch) and the calling
 * thread's last error message ("" if none). */
int32_t pcms_version(void);
const char *pcms_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PCMS_MLS_H */
