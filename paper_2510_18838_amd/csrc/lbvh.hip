// Construction of the linear bounding volume hierarchy over the sources (the
// alternative localisation structure of the PCMS paper, Section 3.3).
//
//  1. The sources' bounding box and a single-bucket GridParams over it (so the
//     sorted source arrays, the records and every per-target code path built
//     for the uniform grid apply unchanged, with one bucket holding all
//     sources in Morton order).
//  2. 32-bit Morton codes (32 / dim bits per coordinate of the box) and one
//     stable radix sort of the sources by code.
//  3. The sorted coordinate records (the grid's gather kernel).
//  4. Leaves: every internal node of the radix tree over the sorted sources
//     marks its split as a leaf boundary when it holds more than max_leaf
//     sources; a scan of the marks numbers the leaves and gives their
//     starts and the leaf count (kept on the device).
//  5. The radix tree over the leaves (keyed by their first source's code,
//     ties by leaf index), all nodes in parallel; then every record's rope
//     and source range from the splits and leaf starts.
//  6. Boxes bottom up, level by level: the leaves' boxes from their
//     sources, every internal node's depth (its climb to the root), the
//     nodes bucketed by depth, then one launch per depth from the deepest
//     up, each node uniting its children's boxes.  The kernel boundaries
//     order the levels, so no thread waits on another or fences memory
//     (a device-scope fence writes back a whole L2 on this chip, which made
//     the usual arrival-counter climb several times slower).
// Every launch is sized for the worst case of one leaf per source and reads
// the leaf count from the device, so the build never waits for the host.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "bvh.h"
#include "internal.h"

namespace pcms {

namespace {

// One thread per item (n < 2^30 items, so the count fits the grid's x range).
int blocks_for(int64_t n, int tpb)
{
    return (int)std::max<int64_t>((n + tpb - 1) / tpb, 1);
}

template <int D>
__global__ void k_morton(const GridParams *__restrict__ gpp, const double *__restrict__ pts,
                         int64_t n, unsigned *__restrict__ keys, int *__restrict__ vals)
{
    const GridParams gp = *gpp;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        keys[i] = bvh_morton<D>(gp, pts + i * D);
        vals[i] = (int)i;
    }
}

__global__ void k_single_cell(int n, int *cell_start)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        cell_start[0] = 0;
        cell_start[1] = n;
    }
}

// Leaf boundaries from the internal nodes of the tree over the sources.
__global__ void k_point_cuts(const unsigned *__restrict__ codes, int n, int max_leaf,
                             int *__restrict__ cut)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n - 1) bvh_point_cut(codes, n, i, max_leaf, cut);
}

__global__ void k_leaf_flags(const int *__restrict__ cut, int n, int *__restrict__ lid)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) lid[i] = i == 0 || cut[i - 1];
}

// After the exclusive scan of the flags: leaf starts, and the leaf count.
__global__ void k_leaf_starts(const int *__restrict__ cut, const int *__restrict__ lid, int n,
                              int *__restrict__ leaf_start, int *__restrict__ nl_dev)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int flag = i == 0 || cut[i - 1];
    if (flag) leaf_start[lid[i]] = i;
    if (i == n - 1) {
        const int nl = lid[i] + flag;
        *nl_dev = nl;
        leaf_start[nl] = n;
    }
}

// Internal node i of the tree over the leaves (bvh_radix_node).
template <int D>
__global__ void k_radix_tree(const unsigned *__restrict__ codes, const int *__restrict__ leaf_start,
                             const int *__restrict__ nl_dev, float *__restrict__ nodes,
                             int *__restrict__ parent, int *__restrict__ child1,
                             int *__restrict__ split_right)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nl = *nl_dev;
    if (i < nl - 1) bvh_radix_node<D>(codes, leaf_start, nl, i, nodes, parent, child1, split_right);
}

template <int D>
__global__ void k_ropes(const int *__restrict__ nl_dev, float *__restrict__ nodes,
                        const int *__restrict__ leaf_start, const int *__restrict__ split_right)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int nl = *nl_dev;
    if (r < 2 * nl - 1) bvh_rope<D>(nl, r, nodes, leaf_start, split_right);
}

constexpr int kLevels = 64;   // internal-node depths (0..63: the keys have 64 bits)

template <int D>
__device__ __forceinline__ void store_box(float *nd, const float (&lo)[D], const float (&hi)[D])
{
#pragma unroll
    for (int k = 0; k < D; ++k) {
        nd[k] = lo[k];
        nd[D + k] = hi[k];
    }
}

template <int D>
__global__ void k_leaf_boxes(const double *__restrict__ spts, const int *__restrict__ leaf_start,
                             const int *__restrict__ nl_dev, float *__restrict__ nodes)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    const int nl = *nl_dev;
    if (l >= nl) return;
    float lo[D], hi[D];
    bvh_leaf_box<D>(spts, leaf_start[l], leaf_start[l + 1], lo, hi);
    store_box<D>(nodes + (size_t)(nl - 1 + l) * bvh_stride(D), lo, hi);
}

// Depth of every internal node (parent hops to the root) and the per-depth
// counts (aggregated per block in LDS, then one atomic per block and depth).
__global__ void k_node_depth(const int *__restrict__ parent, const int *__restrict__ nl_dev,
                             int *__restrict__ depth, int *__restrict__ count)
{
    __shared__ int c[kLevels];
    for (int j = threadIdx.x; j < kLevels; j += blockDim.x) c[j] = 0;
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n_int = *nl_dev - 1;
    if (i < n_int) {
        int d = 0;
        for (int r = i; r != 0 && d < kLevels - 1; r = parent[r]) ++d;
        depth[i] = d;
        atomicAdd(&c[d], 1);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < kLevels; j += blockDim.x)
        if (c[j]) atomicAdd(&count[j], c[j]);
}

// start[d] = nodes of depth < d (exclusive scan of the kLevels counts); the
// fill cursors start there.
__global__ void k_depth_starts(const int *__restrict__ count, int *__restrict__ start,
                               int *__restrict__ fill)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int run = 0;
    for (int d = 0; d < kLevels; ++d) {
        start[d] = run;
        fill[d] = run;
        run += count[d];
    }
    start[kLevels] = run;
}

// order[start[depth]..] = the nodes of each depth (block-aggregated slots).
__global__ void k_depth_scatter(const int *__restrict__ depth, const int *__restrict__ nl_dev,
                                int *__restrict__ fill, int *__restrict__ order)
{
    __shared__ int c[kLevels], base[kLevels];
    for (int j = threadIdx.x; j < kLevels; j += blockDim.x) c[j] = 0;
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool on = i < *nl_dev - 1;
    const int d = on ? depth[i] : 0;
    const int rank = on ? atomicAdd(&c[d], 1) : 0;
    __syncthreads();
    for (int j = threadIdx.x; j < kLevels; j += blockDim.x)
        base[j] = c[j] ? atomicAdd(&fill[j], c[j]) : 0;
    __syncthreads();
    if (on) order[base[d] + rank] = i;
}

// One level: every node of depth d unites its children's boxes (written by
// earlier launches: the leaves, or the deeper levels).
template <int D>
__global__ void k_level_boxes(int d, const int *__restrict__ start, const int *__restrict__ order,
                              const int *__restrict__ child1, float *__restrict__ nodes)
{
    constexpr int S = bvh_stride(D);
    const int beg = start[d], end = start[d + 1];
    for (int idx = beg + blockIdx.x * blockDim.x + threadIdx.x; idx < end;
         idx += gridDim.x * blockDim.x) {
        const int i = order[idx];
        float *nd = nodes + (size_t)i * S;
        const float *a = nodes + (size_t)bvh_int(nd, 2 * D) * S;
        const float *b = nodes + (size_t)child1[i] * S;
        float lo[D], hi[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            lo[k] = fminf(a[k], b[k]);
            hi[k] = fmaxf(a[D + k], b[D + k]);
        }
        store_box<D>(nd, lo, hi);
    }
}

__global__ void k_zero(int *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Scratch of the tree passes over n sources (ints).
struct TreeScratch {
    int *leaf_start, *nl, *parent, *child1, *split_right, *depth, *order, *count, *start, *fill,
        *scan;
    explicit TreeScratch(int *base, int n)
    {
        leaf_start = base;              // [n + 1]
        nl = leaf_start + n + 1;        // [1]
        parent = nl + 1;                // [2n - 1] (record -> internal node)
        child1 = parent + 2 * n;        // [n]
        split_right = child1 + n;       // [n]
        depth = split_right + n;        // [n]
        order = depth + n;              // [n]
        count = order + n;              // [kLevels]
        start = count + kLevels;        // [kLevels + 1]
        fill = start + kLevels + 1;     // [kLevels]
        scan = fill + kLevels;          // exclusive_scan_ints(n)
    }
    static size_t ints(int n) { return (size_t)7 * n + 2 + 3 * kLevels + 1 + exclusive_scan_ints(n); }
};

// Steps 4-6 over the n sorted sources (codes sorted; cut and lid are n-int
// work arrays).
template <int D>
pcms_status build_tree(Grid *g, const unsigned *codes, int n, int max_leaf, int *cut, int *lid,
                       const TreeScratch &w, hipStream_t s)
{
    const int b1 = blocks_for(n, 256);
    if (n > 1) {
        k_point_cuts<<<blocks_for(n - 1, 256), 256, 0, s>>>(codes, n, max_leaf, cut);
        PCMS_HIP(hipGetLastError());
    }
    k_leaf_flags<<<b1, 256, 0, s>>>(cut, n, lid);
    PCMS_HIP(hipGetLastError());
    pcms_status st = exclusive_scan(lid, n, w.scan, s);
    if (st != PCMS_OK) return st;
    k_leaf_starts<<<b1, 256, 0, s>>>(cut, lid, n, w.leaf_start, w.nl);
    PCMS_HIP(hipGetLastError());
    k_zero<<<1, kLevels, 0, s>>>(w.count, kLevels);
    PCMS_HIP(hipGetLastError());
    if (n > 1) {
        k_radix_tree<D><<<blocks_for(n - 1, 256), 256, 0, s>>>(codes, w.leaf_start, w.nl,
                                                               g->bvh_nodes, w.parent, w.child1,
                                                               w.split_right);
        PCMS_HIP(hipGetLastError());
    }
    k_ropes<D><<<blocks_for(2 * (int64_t)n - 1, 256), 256, 0, s>>>(w.nl, g->bvh_nodes,
                                                                  w.leaf_start, w.split_right);
    PCMS_HIP(hipGetLastError());
    k_leaf_boxes<D><<<b1, 256, 0, s>>>(g->spts, w.leaf_start, w.nl, g->bvh_nodes);
    PCMS_HIP(hipGetLastError());
    if (n > 1) {
        k_node_depth<<<b1, 256, 0, s>>>(w.parent, w.nl, w.depth, w.count);
        PCMS_HIP(hipGetLastError());
        k_depth_starts<<<1, 64, 0, s>>>(w.count, w.start, w.fill);
        PCMS_HIP(hipGetLastError());
        k_depth_scatter<<<b1, 256, 0, s>>>(w.depth, w.nl, w.fill, w.order);
        PCMS_HIP(hipGetLastError());
        // deepest level first; an empty level is one short launch
        const int lb = std::min(blocks_for(n, 256), 1024);
        for (int d = kLevels - 1; d >= 0; --d) {
            k_level_boxes<D><<<lb, 256, 0, s>>>(d, w.start, w.order, w.child1, g->bvh_nodes);
            PCMS_HIP(hipGetLastError());
        }
    }
    return PCMS_OK;
}

}  // namespace

// Records: at most one leaf per source, so at most 2 n_src - 1.
size_t bvh_node_bytes(int64_t n_src, int dim)
{
    return sizeof(float) * (size_t)bvh_stride(dim) * (size_t)(2 * n_src - 1);
}

size_t bvh_link_ints(int64_t n_src) { return TreeScratch::ints((int)n_src); }

pcms_status morton_keys(int dim, const GridParams *gp, const double *pts, int64_t n,
                        unsigned *keys, int *vals, hipStream_t s)
{
    const int blocks = blocks_for(n, 256);
    switch (dim) {
    case 1: k_morton<1><<<blocks, 256, 0, s>>>(gp, pts, n, keys, vals); break;
    case 2: k_morton<2><<<blocks, 256, 0, s>>>(gp, pts, n, keys, vals); break;
    case 3: k_morton<3><<<blocks, 256, 0, s>>>(gp, pts, n, keys, vals); break;
    case 4: k_morton<4><<<blocks, 256, 0, s>>>(gp, pts, n, keys, vals); break;
    default: k_morton<5><<<blocks, 256, 0, s>>>(gp, pts, n, keys, vals); break;
    }
    PCMS_HIP(hipGetLastError());
    return PCMS_OK;
}

pcms_status build_lbvh_device(Grid *g, const double *src, int max_leaf, hipStream_t s,
                              const std::function<pcms_status()> *after_params)
{
    const int dim = g->dim;
    const int n = (int)g->n_src;
    // scratch: bbox keys, metric copy, sort buffers, tree links and counters
    const size_t sort_bytes = grid_build_scratch_bytes(n);
    void *raw = nullptr;
    pcms_status st = scratch_alloc(&raw, sort_bytes + sizeof(int) * bvh_link_ints(n) + 256, s);
    if (st != PCMS_OK) return st;
    char *cur = (char *)raw;
    long long *bb = (long long *)cur;
    cur += 128;
    double *gdev = (double *)cur;
    cur += 128;
    unsigned *k0 = (unsigned *)cur;
    cur += sizeof(unsigned) * (size_t)n;
    unsigned *k1 = (unsigned *)cur;
    cur += sizeof(unsigned) * (size_t)n;
    int *v1 = (int *)cur;
    cur += sizeof(int) * (size_t)n;
    int *hist = (int *)cur;
    cur += sizeof(int) * sort_hist_ints(n);
    int *scan_scratch = (int *)cur;
    cur += sizeof(int) * sort_scan_ints(n);
    cur = (char *)(((uintptr_t)cur + 255) & ~(uintptr_t)255);
    const TreeScratch w((int *)cur, n);
    g->lbvh = 1;   // before after_params: work forked there orders targets by Morton code

    if ((st = source_bbox_params(g, src, gdev, bb, 0.0, (double)n, s)) != PCMS_OK) return st;
    if (after_params && (st = (*after_params)()) != PCMS_OK) return st;
    if ((st = morton_keys(dim, g->params, src, n, k0, g->perm, s)) != PCMS_OK) return st;
    if ((st = sort_pairs(k0, g->perm, k1, v1, n, 32, hist, scan_scratch, s)) != PCMS_OK) return st;
    k_single_cell<<<1, 64, 0, s>>>(n, g->cell_start);
    PCMS_HIP(hipGetLastError());
    if ((st = gather_records(g, src, s)) != PCMS_OK) return st;
    // the sort's second buffers (free once sorted) hold the leaf marks
    int *cut = (int *)k1, *lid = v1;
    switch (dim) {
    case 1: st = build_tree<1>(g, k0, n, max_leaf, cut, lid, w, s); break;
    case 2: st = build_tree<2>(g, k0, n, max_leaf, cut, lid, w, s); break;
    case 3: st = build_tree<3>(g, k0, n, max_leaf, cut, lid, w, s); break;
    case 4: st = build_tree<4>(g, k0, n, max_leaf, cut, lid, w, s); break;
    default: st = build_tree<5>(g, k0, n, max_leaf, cut, lid, w, s); break;
    }
    if (st != PCMS_OK) return st;
    scratch_free(raw, s);
    return PCMS_OK;
}

}  // namespace pcms
