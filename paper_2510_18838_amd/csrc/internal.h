// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

#include "device_common.h"
#include "pcms_mls.h"

namespace pcms {

// Library-owned grid handle.
struct Grid {
    int dim;
    int64_t n_src;
    int n_cells_cap;
    double g[kMaxDim];
    GridParams *params;   // device
    int *cell_start;      // device [n_cells_cap + 1]
    int *perm;            // device [n_src]: sorted position -> source index
    int *iperm;           // device [n_src]: source index -> sorted position
    double *spts;         // device [n_src * padded_dim(dim)]: sorted coordinates
    float *spts32;        // device [n_src * dim]: fl32(coordinate - lo), packed, followed
                          // by the fixed-point records sq (one allocation)
    uint32_t *sq;         // device [n_src * dim]: quantize(coordinate), packed
    int device;
    // LBVH (lbvh != 0): one bucket holding the sources in Morton order, and
    // the tree's records (bvh.h; room for the worst case of one leaf per
    // source, the leaf count itself stays on the device)
    int lbvh;
    float *bvh_nodes;     // device [2 n_src - 1][bvh_stride(dim)]
};

// error plumbing ------------------------------------------------------------
void set_error(const std::string &msg);
pcms_status hip_fail(hipError_t e, const char *what);

#define PCMS_HIP(call)                                              \
    do {                                                            \
        hipError_t e_ = (call);                                     \
        if (e_ != hipSuccess) return ::pcms::hip_fail(e_, #call);   \
    } while (0)

// stream-ordered scratch allocation ------------------------------------------
pcms_status scratch_alloc(void **p, size_t bytes, hipStream_t s);
void scratch_free(void *p, hipStream_t s);

// grid construction (sort.hip) ----------------------------------------------
int cells_cap_for(int64_t n_src);
// Slices of dimension 0 per bucket width (kRowSlices; the environment
// variable PCMS_ROW_SLICES = 1, 2, 4, 8 or 16 overrides it).
int row_slices();
// Builds `grid` (allocated by the caller with the right capacity) from src.
// cell_width > 0: metric bucket width; else buckets sized for pts_per_cell.
// after_params (may be NULL) is called once grid->params is enqueued, before
// the sort: work that needs only the parameters can fork off there.
pcms_status build_grid_device(Grid *grid, const double *src, double cell_width,
                              double pts_per_cell, hipStream_t s,
                              const std::function<pcms_status()> *after_params = nullptr);
// Stream-ordered scratch that build_grid_device takes while it runs.
size_t grid_build_scratch_bytes(int64_t n_src);
// The two stages build_grid_device shares with the LBVH build: the bounding
// box and the GridParams of the sources (gdev: a device copy of the metric,
// bb: the box keys, both scratch), and the sorted coordinate records and
// inverse permutation from grid->perm.
pcms_status source_bbox_params(Grid *grid, const double *src, double *gdev, long long *bb,
                               double cell_width, double pts_per_cell, hipStream_t s);
pcms_status gather_records(Grid *grid, const double *src, hipStream_t s);
// LBVH over the sources (lbvh.hip): `grid` allocated with n_cells_cap = 1
// and bvh_node_bytes() of records; leaves of at most max_leaf sources.
pcms_status build_lbvh_device(Grid *grid, const double *src, int max_leaf, hipStream_t s,
                              const std::function<pcms_status()> *after_params = nullptr);
size_t bvh_node_bytes(int64_t n_src, int dim);
size_t bvh_link_ints(int64_t n_src);   // build scratch of the tree passes
// Exclusive scan of n ints in place; scratch holds exclusive_scan_ints(n).
pcms_status exclusive_scan(int *data, int n, int *scratch, hipStream_t s);
size_t exclusive_scan_ints(int n);
// 32-bit Morton codes of points in the box of gp (keys) with their indices.
pcms_status morton_keys(int dim, const GridParams *gp, const double *pts, int64_t n,
                        unsigned *keys, int *vals, hipStream_t s);
// Bits of the target ordering key that the sort uses (the top ones): 24, or
// PCMS_TARGET_KEY_BITS (8..32) from the environment.  Fewer bits save sort
// passes but cost more in the search kernel than they save (16 bits: the
// 4M-target kNN step's kernel takes 13 % longer).
constexpr int kTargetKeyBits = 24;
int target_key_bits();
// Target ordering: tperm[i] = index of the target at sorted position i.  Its
// sort buffers are `ws` (sort_targets_bytes(n_tgt) bytes, 256-byte aligned)
// when given, else stream-ordered scratch.
size_t sort_targets_bytes(int64_t n_tgt);
pcms_status sort_targets(const Grid *grid, const double *tgt, int64_t n_tgt, int *tperm,
                         hipStream_t s, void *ws = nullptr);
// out[l][t] = stage[t * padded_dim(n_fields) + l] for l < n_fields.
pcms_status unstage_fields(const double *stage, int64_t n_tgt, int n_fields, double *out,
                           hipStream_t s);
// Sorted field copy: svals[p * n_fields + l] = vals[l * n_src + perm[p]].
pcms_status gather_values(const Grid *grid, const double *vals, int n_fields, double *svals,
                          hipStream_t s);

// Stable LSD radix sort of (key, value) pairs by the low `bits` key bits; the
// result ends in (k0, v0).  hist and scan_scratch hold sort_hist_ints(n) and
// sort_scan_ints(n) ints.  Enqueues kernels and device copies only.
pcms_status sort_pairs(unsigned *k0, int *v0, unsigned *k1, int *v1, int n, int bits, int *hist,
                       int *scan_scratch, hipStream_t s);
size_t sort_hist_ints(int n);
size_t sort_scan_ints(int n);
// Smallest b <= 32 with 2^b >= bound.
int bits_for(double bound);

// transfer on a built grid (abi.hip) -------------------------------------------
// Bytes of the workspace of transfer_on_grid: status counts, target order,
// its sort buffers and the bucket-ordered field records.
size_t transfer_ws_bytes(int64_t n_src, int n_fields, int64_t n_tgt);
// The target order's part of that workspace: tperm and its sort buffers.
void transfer_ws_order(void *ws, int64_t n_src, int n_fields, int64_t n_tgt, int **tperm,
                       void **sort_ws);
// Marks the point of s after which the calling thread's side stream
// (default priority, created once per device) may run: records its fork
// event on s.
pcms_status side_fork(hipStream_t s);
// Target ordering of grid g on the calling thread's side stream, after the
// work enqueued so far on s (record_fork) or after the point side_fork last
// marked on s (!record_fork: the host can enqueue more work on s first);
// *join is recorded there when tperm is complete, for s to wait on.
pcms_status order_targets_aside(const Grid *g, const double *tgt, int64_t n_tgt, int *tperm,
                                void *sort_ws, hipStream_t s, hipEvent_t *join,
                                bool record_fork = true);
// Target ordering, field gather, search-and-fit and the status plumbing of
// a transfer on grid g (arguments already validated).  ws: a device
// workspace of transfer_ws_bytes(...) bytes, 256-byte aligned, or NULL for
// stream-ordered scratch.  overlap: order the targets on the side stream
// while the fields are gathered on s.  ordered: the target order is already
// being computed into ws (order_targets_aside), complete at this event.
pcms_status transfer_on_grid(const Grid *g, const double *src_vals, int32_t n_fields,
                             const double *tgt, int64_t n_tgt, int32_t degree,
                             const pcms_radius *radius, int32_t k_cap, const pcms_mls_opts *opts,
                             hipStream_t s, double *tgt_vals, uint8_t *status, void *ws,
                             bool overlap = false, hipEvent_t ordered = nullptr);
// Turns off the calling thread's phase timing for the next transfer.
void profile_off();
// Host-side validation of a transfer's arguments (PCMS_ERR_ARG with a message).
pcms_status check_transfer_args(int64_t n_src, int32_t dim, const double *src_vals,
                                int32_t n_fields, const double *tgt, int64_t n_tgt, int32_t degree,
                                const pcms_radius *radius, int32_t k_cap,
                                const pcms_mls_opts *opts, double *tgt_vals);

// search and fit (mls.hip) ----------------------------------------------------
struct LaunchSpec {
    const Grid *grid;
    const double *tgt;
    const int *tperm;
    int64_t n_tgt;
    pcms_radius radius;
    int k_cap;
    int block;
    int32_t *summary;   // device [4]
};

pcms_status launch_neighbors(const LaunchSpec &ls, int32_t *nbr, int32_t *n_kept,
                             int32_t *n_found, double *r2, uint8_t *status, hipStream_t s);

// stage: NULL, or [n_tgt][padded_dim(n_fields)] records for unstage_fields.
pcms_status launch_transfer(const LaunchSpec &ls, const double *svals, int n_fields, int degree,
                            int weight, int precision, double lambda, double *out,
                            double *stage, uint8_t *status, hipStream_t s);

pcms_status zero_ints(int32_t *p, int n, hipStream_t s);

// precomputed transfer operator (mls.hip, op.hip) ----------------------------
// Library-owned operator: for sorted target i and slot e < op_n[i], weight
// op_w[e * n_tgt + i] of the source at sorted position op_c[e * n_tgt + i];
// op_n[i] = -1 for a failed target; tperm[i] = original index of target i;
// perm / iperm map sorted source positions to original indices and back.
struct Operator {
    int64_t n_src = 0, n_tgt = 0;
    int width = 0;
    void *mem = nullptr;      // one allocation holding the arrays below
    int *tperm = nullptr;
    int *perm = nullptr;
    int *iperm = nullptr;
    int32_t *op_n = nullptr;
    int32_t *op_c = nullptr;
    double *op_w = nullptr;
};
// Emits the operator of the targets of ls (sorted by ls.tperm).
pcms_status launch_operator(const LaunchSpec &ls, int degree, int weight, int precision,
                            double lambda, double *op_w, int32_t *op_c, int32_t *op_n,
                            uint8_t *status, hipStream_t s);
// Slots per target the operator needs (>= every kept count).
int operator_width(const LaunchSpec &ls);
// tgt_vals[l][t] = sum_e w f_l[c] over the target's slots, NaN where failed:
// the fields are first copied into bucket order (records of padded_dim(nf)
// doubles in stream-ordered scratch), then gathered by sorted position.
pcms_status operator_apply(const Operator &op, const double *vals, int n_fields, double *out,
                           hipStream_t s);
// Copies the operator to caller arrays in original target order:
// n_kept[t], cols[t * stride + e], weights[t * stride + e] (e < n_kept[t]).
pcms_status operator_export(const Operator &op, int stride, int32_t *n_kept, int32_t *cols,
                            double *weights, hipStream_t s);

// batched transfer (batch.hip) -------------------------------------------------
// Device descriptor of one problem of a batch; its grid, sorted copies and
// target order are slices of the batch's global arrays at the given offsets.
struct BatchProb {
    const double *src;
    const double *vals;
    const double *tgt;
    double *out;
    uint8_t *status;
    int64_t src_off;      // into the global source order (perm, iperm, keys)
    int64_t tgt_off;      // into the global target order (tperm)
    int64_t cs_off;       // into the global cell_start array
    int64_t spts_off;     // doubles, into the sorted coordinates
    int64_t s32_off;      // words, into the sorted FP32 and fixed-point records
    int64_t sval_off;     // doubles, into the sorted field records
    unsigned key_off;     // source sort keys: key_off + bucket id
    unsigned tkey_off;    // target sort keys: tkey_off + processing-order key
    int n_src, n_tgt, dim, degree, nf, nfs, k_cap, words, stride;
    int mode, k, n_min, max_iter, unit, tiled, cells_cap;
    double r, cell_width, pts_per_cell;
    double g[kMaxDim];
};

// A planned batch: host descriptors and the device workspace (one
// allocation) of every stage.
struct BatchPlan {
    int n = 0;
    std::vector<BatchProb> hp;
    int weight = 0, precision = 0, block = 256;
    double lambda = 0.0, cell_factor = 0.0;
    int64_t n_src_tot = 0, n_tgt_tot = 0, cs_tot = 0;
    int key_bits = 0, tkey_bits = 0, max_stride = 1;
    void *ws = nullptr;
    BatchProb *probs_d = nullptr;
    GridParams *params = nullptr;
    long long *bb = nullptr;          // [n][2][kMaxDim] ordered min/max keys
    int64_t *src_pref = nullptr, *tgt_pref = nullptr, *cs_pref = nullptr;   // [n + 1]
    unsigned *k0 = nullptr, *k1 = nullptr;
    int *v0 = nullptr, *v1 = nullptr, *hist = nullptr, *scan = nullptr;
    int *cs = nullptr, *perm = nullptr, *iperm = nullptr, *tperm = nullptr;
    double *spts = nullptr, *svals = nullptr;
    float *spts32 = nullptr;
    uint32_t *sq = nullptr;
    int4 *items = nullptr;
    int n_items = 0;
    // per class of problems: its slice [cls_begin, cls_end) of the queue
    std::vector<int> cls_begin, cls_end;
    int32_t *summary = nullptr;       // device [4]

    std::vector<int> outer;           // problems of dimension > 3: one-problem kernel
    std::vector<Grid> views;          // host views of every problem's grid slices
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// Lays out the workspace of a plan whose hp[] sizes are filled in (sets the
// offsets, the work items and the device pointers); allocates it.
pcms_status batch_setup(BatchPlan &p);
// Enqueues every stage of the plan on s (no allocation, no host sync).
pcms_status batch_enqueue(BatchPlan &p, hipStream_t s);
// Copies the 4 status counts (device to device, enqueued on s).
pcms_status batch_copy_summary(const int32_t *from, int32_t *to, hipStream_t s);

}  // namespace pcms
