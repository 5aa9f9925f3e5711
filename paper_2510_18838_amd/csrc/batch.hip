// Batched field transfer: many independent problems (each the operation of
// the PCMS paper, Section 3.2.1, Eq. 1, on its own uniform grid, Section
// 3.3) executed together.
//
// All grids are built by one pass of segmented kernels.  Every source gets
// the sort key (problem key offset + bucket id), and a single stable radix
// sort orders the sources of all problems by (problem, bucket).  Each
// problem's sorted sources, bucket offsets, coordinates and field records
// are then contiguous slices of global arrays, laid out exactly as the
// one-problem path lays out its own grid, so the per-target code (search,
// moment assembly, solve, evaluation) runs unchanged on every slice.
// Targets are ordered the same way.  The (problem, tile of targets) work
// items are grouped by the problems' class (dimension, degree, metric) and,
// within a class, ordered by estimated cost, largest first.  One kernel per
// class present, each compiled for its class alone (its own register
// allocation), runs one block per item of its class; blocks are dispatched
// in queue order, which schedules the largest items first.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <climits>

#include "batch_kernel.h"

namespace pcms {

namespace {

constexpr int kChunk = 4096;   // sources per block of the bounding-box pass

// The q with pref[q] <= j < pref[q + 1], for 0 <= j < pref[n] (pref is the
// non-decreasing prefix sum of the segment sizes, so empty segments are
// skipped).
__device__ __forceinline__ int segment_of(const int64_t *__restrict__ pref, int n, int64_t j)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pref[mid] <= j) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ inline long long ordered_key(double x)
{
    long long b = __double_as_longlong(x);
    return b >= 0 ? b : (b ^ 0x7fffffffffffffffLL);
}

__device__ inline double ordered_val(long long k)
{
    long long b = k >= 0 ? k : (k ^ 0x7fffffffffffffffLL);
    return __longlong_as_double(b);
}

int grid_for(int64_t n, int tpb)
{
    const int64_t b = (n + tpb - 1) / tpb;
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 65536);
}

// Running min/max keys of every problem and the summary.
__global__ void k_batch_init(long long *bb, int n, int32_t *summary)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n * kMaxDim) {
        const int q = i / kMaxDim, k = i % kMaxDim;
        bb[(size_t)q * 2 * kMaxDim + k] = LLONG_MAX;
        bb[(size_t)q * 2 * kMaxDim + kMaxDim + k] = LLONG_MIN;
    }
    if (i == 0)
        for (int k = 0; k < 4; ++k) summary[k] = 0;
}

// Per-problem bounding boxes: a block reduces a chunk of the global source
// index space, problem by problem (chunks rarely span more than one), with
// one atomic per problem, dimension and block.
__global__ void __launch_bounds__(256) k_batch_bbox(const BatchProb *__restrict__ probs,
                                                    const int64_t *__restrict__ pref, int n,
                                                    long long *bb)
{
    __shared__ double smn[4][kMaxDim], smx[4][kMaxDim];
    const int64_t total = pref[n];
    for (int64_t c0 = (int64_t)blockIdx.x * kChunk; c0 < total; c0 += (int64_t)gridDim.x * kChunk) {
        const int64_t c1 = min(c0 + (int64_t)kChunk, total);
        for (int q = segment_of(pref, n, c0); q < n && pref[q] < c1; ++q) {
            const BatchProb &P = probs[q];
            const int dim = P.dim;
            const int64_t a = max(c0, pref[q]), b = min(c1, pref[q + 1]);
            double mn[kMaxDim], mx[kMaxDim];
#pragma unroll
            for (int k = 0; k < kMaxDim; ++k) {
                mn[k] = INFINITY;
                mx[k] = -INFINITY;
            }
            for (int64_t j = a + threadIdx.x; j < b; j += blockDim.x) {
                const double *x = P.src + (j - pref[q]) * dim;
#pragma unroll
                for (int k = 0; k < kMaxDim; ++k) {
                    if (k < dim) {
                        mn[k] = fmin(mn[k], x[k]);
                        mx[k] = fmax(mx[k], x[k]);
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < kMaxDim; ++k) {
                for (int off = 32; off > 0; off >>= 1) {
                    mn[k] = fmin(mn[k], __shfl_xor(mn[k], off));
                    mx[k] = fmax(mx[k], __shfl_xor(mx[k], off));
                }
            }
            const int w = threadIdx.x >> 6;
            if ((threadIdx.x & 63) == 0) {
#pragma unroll
                for (int k = 0; k < kMaxDim; ++k) {
                    smn[w][k] = mn[k];
                    smx[w][k] = mx[k];
                }
            }
            __syncthreads();
            if (threadIdx.x == 0 && a < b) {
                for (int k = 0; k < dim; ++k) {
                    double lo = smn[0][k], hi = smx[0][k];
                    for (int v = 1; v < (int)(blockDim.x >> 6); ++v) {
                        lo = fmin(lo, smn[v][k]);
                        hi = fmax(hi, smx[v][k]);
                    }
                    atomicMin(&bb[(size_t)q * 2 * kMaxDim + k], ordered_key(lo));
                    atomicMax(&bb[(size_t)q * 2 * kMaxDim + kMaxDim + k], ordered_key(hi));
                }
            }
            __syncthreads();
        }
    }
}

// Bucket sizing of every problem (one thread each).
__global__ void k_batch_params(const BatchProb *__restrict__ probs, int n,
                               const long long *__restrict__ bb, int sub, GridParams *params)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const BatchProb &P = probs[q];
    double lo[kMaxDim], hi[kMaxDim];
    for (int k = 0; k < kMaxDim; ++k) {
        lo[k] = k < P.dim ? ordered_val(bb[(size_t)q * 2 * kMaxDim + k]) : 0.0;
        hi[k] = k < P.dim ? ordered_val(bb[(size_t)q * 2 * kMaxDim + kMaxDim + k]) : 0.0;
    }
    grid_params_compute(lo, hi, P.dim, P.n_src, P.g, P.cell_width, P.pts_per_cell, P.cells_cap,
                        sub, &params[q]);
}

// Sort keys of all sources: problem key offset + bucket id; value = global
// source index.
__global__ void k_batch_src_keys(const BatchProb *__restrict__ probs,
                                 const GridParams *__restrict__ params,
                                 const int64_t *__restrict__ pref, int n, unsigned *keys, int *vals)
{
    const int64_t total = pref[n];
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int q = segment_of(pref, n, j);
        const BatchProb &P = probs[q];
        const double *x = P.src + (j - P.src_off) * P.dim;
        keys[j] = P.key_off + bucket_key(params[q], x);
        vals[j] = (int)j;
    }
}

// Bucket offsets of every problem (local sorted positions), from the sorted
// keys: cs[c] = #(the problem's keys below key_off + c), for c <= n_cells;
// entries past n_cells (never read) are set to n_src.
__global__ void k_batch_cell_start(const BatchProb *__restrict__ probs,
                                   const GridParams *__restrict__ params,
                                   const int64_t *__restrict__ cs_pref, int n,
                                   const unsigned *__restrict__ keys, int *cs)
{
    const int64_t total = cs_pref[n];
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < total;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int q = segment_of(cs_pref, n, c);
        const BatchProb &P = probs[q];
        const int cl = (int)(c - cs_pref[q]);
        if (cl > params[q].n_cells) {
            cs[c] = P.n_src;
            continue;
        }
        const unsigned key = P.key_off + (unsigned)cl;
        int64_t lo = P.src_off, hi = P.src_off + P.n_src;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (keys[mid] < key) lo = mid + 1;
            else hi = mid;
        }
        cs[c] = (int)(lo - P.src_off);
    }
}

// Sorted (padded) coordinates and their FP32 records, and the local
// permutation and its inverse.
__global__ void k_batch_gather_pts(const BatchProb *__restrict__ probs,
                                   const GridParams *__restrict__ params,
                                   const int64_t *__restrict__ pref, int n,
                                   const int *__restrict__ sorted_vals, double *spts, float *spts32,
                                   uint32_t *sq, int *perm, int *iperm)
{
    const int64_t total = pref[n];
    for (int64_t P0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; P0 < total;
         P0 += (int64_t)gridDim.x * blockDim.x) {
        const int q = segment_of(pref, n, P0);
        const BatchProb &B = probs[q];
        const int p = (int)(P0 - B.src_off);
        const int jl = (int)(sorted_vals[P0] - B.src_off);
        write_records_dim(B.src + (int64_t)jl * B.dim, B.dim, params[q],
                          spts + B.spts_off + (int64_t)p * padded_dim(B.dim),
                          spts32 + B.s32_off + (int64_t)p * B.dim, sq + B.s32_off + (int64_t)p * B.dim);
        perm[P0] = jl;
        iperm[B.src_off + jl] = p;
    }
}

// Field records in sorted order (padded_dim(nf) doubles, padding zero).
__global__ void k_batch_scatter_vals(const BatchProb *__restrict__ probs,
                                     const int64_t *__restrict__ pref, int n,
                                     const int *__restrict__ iperm, double *svals)
{
    const int64_t total = pref[n];
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int q = segment_of(pref, n, j);
        const BatchProb &B = probs[q];
        const int64_t jl = j - B.src_off;
        double *row = svals + B.sval_off + (int64_t)iperm[j] * B.nfs;
        // whole 16-byte words (the records are 16-byte aligned)
        for (int l = 0; l < B.nfs; l += 2) {
            const double a = B.vals[(int64_t)l * B.n_src + jl];
            const double b = l + 1 < B.nf ? B.vals[(int64_t)(l + 1) * B.n_src + jl] : 0.0;
            *reinterpret_cast<double2 *>(row + l) = make_double2(a, b);
        }
    }
}

// Processing-order keys of all targets (problem offset + tiled Morton key,
// or bucket id when the batch's tiled keys would not fit 32 bits).
__global__ void k_batch_tgt_keys(const BatchProb *__restrict__ probs,
                                 const GridParams *__restrict__ params,
                                 const int64_t *__restrict__ pref, int n, unsigned *keys, int *vals)
{
    const int64_t total = pref[n];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int q = segment_of(pref, n, i);
        const BatchProb &P = probs[q];
        const double *x = P.tgt + (i - P.tgt_off) * P.dim;
        keys[i] = P.tkey_off + (P.tiled ? target_key(params[q], x) : bucket_key(params[q], x));
        vals[i] = (int)i;
    }
}

// Local target order of every problem from the sorted global indices.
__global__ void k_batch_tperm(const int64_t *__restrict__ pref, int n,
                              const int *__restrict__ sorted_vals, int *tperm)
{
    const int64_t total = pref[n];
    for (int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; I < total;
         I += (int64_t)gridDim.x * blockDim.x) {
        const int q = segment_of(pref, n, I);
        tperm[I] = (int)(sorted_vals[I] - pref[q]);
    }
}

__global__ void k_copy_summary(const int32_t *from, int32_t *to)
{
    if (threadIdx.x < 4) to[threadIdx.x] = from[threadIdx.x];
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

pcms_status batch_setup(BatchPlan &p)
{
    const int n = p.n;
    // offsets of every problem's slices
    int64_t src = 0, tgt = 0, cs = 0, sp = 0, sv = 0, s32 = 0;
    double keys = 0.0, tkeys = 0.0;
    for (int q = 0; q < n; ++q) {
        BatchProb &B = p.hp[q];
        B.src_off = src;
        B.tgt_off = tgt;
        B.cs_off = cs;
        B.spts_off = sp;
        B.s32_off = s32;
        B.sval_off = sv;
        B.key_off = (unsigned)keys;
        src += B.n_src;
        tgt += B.n_tgt;
        cs += (int64_t)B.cells_cap + 1;
        sp += (int64_t)B.n_src * padded_dim(B.dim);
        s32 += (int64_t)B.n_src * B.dim;
        sv += (int64_t)B.n_src * B.nfs;
        keys += (double)B.cells_cap;
        tkeys += tile_key_bound((double)B.cells_cap, B.dim);
        p.max_stride = std::max(p.max_stride, B.stride);
    }
    if (src >= ((int64_t)1 << 31) || tgt >= ((int64_t)1 << 31) || keys >= 4294967295.0) {
        set_error("batch too large: total sources and targets must stay below 2^31");
        return PCMS_ERR_ARG;
    }
    const bool tiled = tkeys < 4294967295.0;
    double t = 0.0;
    for (int q = 0; q < n; ++q) {
        BatchProb &B = p.hp[q];
        B.tiled = tiled;
        B.tkey_off = (unsigned)t;
        t += tiled ? tile_key_bound((double)B.cells_cap, B.dim) : (double)B.cells_cap;
    }
    p.n_src_tot = src;
    p.n_tgt_tot = tgt;
    p.cs_tot = cs;
    p.key_bits = bits_for(keys);
    p.tkey_bits = bits_for(t);
    // work items: tiles of `block` targets of the problems of dimension <= 3,
    // grouped by class, largest estimated cost first within a class
    std::vector<int4> items;
    std::vector<double> cost;
    std::vector<int> cls;
    p.outer.clear();
    for (int q = 0; q < n; ++q) {
        const BatchProb &B = p.hp[q];
        if (B.n_tgt == 0) continue;
        if (B.dim > 3) {
            p.outer.push_back(q);
            continue;
        }
        const int m = B.degree == 0 ? 1 : B.degree == 1 ? 1 + B.dim : 1 + B.dim + B.dim * (B.dim + 1) / 2;
        for (int t0 = 0; t0 < B.n_tgt; t0 += p.block) {
            const int c = std::min(p.block, B.n_tgt - t0);
            items.push_back(make_int4(q, t0, c, 0));
            cost.push_back((double)c * (B.k_cap + 16) * (m + 4) * (m + 4));
            cls.push_back(batch_class(B.dim, B.degree, B.unit));
        }
    }
    std::vector<int> order(items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return cls[x] != cls[y] ? cls[x] < cls[y] : cost[x] > cost[y];
    });
    std::vector<int4> sorted(items.size());
    for (size_t i = 0; i < order.size(); ++i) sorted[i] = items[order[i]];
    p.n_items = (int)sorted.size();
    p.cls_begin.assign(kBatchClasses, 0);
    p.cls_end.assign(kBatchClasses, 0);
    for (size_t i = order.size(); i-- > 0;) p.cls_begin[cls[order[i]]] = (int)i;
    for (size_t i = 0; i < order.size(); ++i) p.cls_end[cls[order[i]]] = (int)i + 1;
    // workspace
    const int64_t nmax = std::max<int64_t>(std::max(src, tgt), 1);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + std::max<size_t>(bytes, 4));
        return o;
    };
    const size_t o_probs = take(sizeof(BatchProb) * n);
    const size_t o_params = take(sizeof(GridParams) * n);
    const size_t o_bb = take(sizeof(long long) * 2 * kMaxDim * n);
    const size_t o_sp = take(sizeof(int64_t) * (n + 1));
    const size_t o_tp = take(sizeof(int64_t) * (n + 1));
    const size_t o_cp = take(sizeof(int64_t) * (n + 1));
    const size_t o_k0 = take(sizeof(unsigned) * nmax);
    const size_t o_k1 = take(sizeof(unsigned) * nmax);
    const size_t o_v0 = take(sizeof(int) * nmax);
    const size_t o_v1 = take(sizeof(int) * nmax);
    const size_t o_hist = take(sizeof(int) * sort_hist_ints((int)nmax));
    const size_t o_scan = take(sizeof(int) * sort_scan_ints((int)nmax));
    const size_t o_cs = take(sizeof(int) * cs);
    const size_t o_perm = take(sizeof(int) * src);
    const size_t o_iperm = take(sizeof(int) * src);
    const size_t o_tperm = take(sizeof(int) * tgt);
    const size_t o_spts = take(sizeof(double) * sp);
    const size_t o_svals = take(sizeof(double) * sv);
    const size_t o_s32 = take(sizeof(float) * 2 * s32);   // FP32 records, then fixed-point ones
    const size_t o_items = take(sizeof(int4) * std::max<size_t>(sorted.size(), 1));
    const size_t o_sum = take(sizeof(int32_t) * 4);
    hipError_t e = hipMalloc(&p.ws, off);
    if (e != hipSuccess) {
        p.ws = nullptr;
        return hip_fail(e, "hipMalloc(batch workspace)");
    }
    char *w = (char *)p.ws;
    p.probs_d = (BatchProb *)(w + o_probs);
    p.params = (GridParams *)(w + o_params);
    p.bb = (long long *)(w + o_bb);
    p.src_pref = (int64_t *)(w + o_sp);
    p.tgt_pref = (int64_t *)(w + o_tp);
    p.cs_pref = (int64_t *)(w + o_cp);
    p.k0 = (unsigned *)(w + o_k0);
    p.k1 = (unsigned *)(w + o_k1);
    p.v0 = (int *)(w + o_v0);
    p.v1 = (int *)(w + o_v1);
    p.hist = (int *)(w + o_hist);
    p.scan = (int *)(w + o_scan);
    p.cs = (int *)(w + o_cs);
    p.perm = (int *)(w + o_perm);
    p.iperm = (int *)(w + o_iperm);
    p.tperm = (int *)(w + o_tperm);
    p.spts = (double *)(w + o_spts);
    p.svals = (double *)(w + o_svals);
    p.spts32 = (float *)(w + o_s32);
    p.sq = reinterpret_cast<uint32_t *>(p.spts32 + s32);
    p.items = (int4 *)(w + o_items);
    p.summary = (int32_t *)(w + o_sum);
    std::vector<int64_t> sp_h(n + 1), tp_h(n + 1), cp_h(n + 1);
    for (int q = 0; q < n; ++q) {
        sp_h[q] = p.hp[q].src_off;
        tp_h[q] = p.hp[q].tgt_off;
        cp_h[q] = p.hp[q].cs_off;
    }
    sp_h[n] = src;
    tp_h[n] = tgt;
    cp_h[n] = cs;
    PCMS_HIP(hipMemcpy(p.probs_d, p.hp.data(), sizeof(BatchProb) * n, hipMemcpyHostToDevice));
    PCMS_HIP(hipMemcpy(p.src_pref, sp_h.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice));
    PCMS_HIP(hipMemcpy(p.tgt_pref, tp_h.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice));
    PCMS_HIP(hipMemcpy(p.cs_pref, cp_h.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice));
    if (!sorted.empty())
        PCMS_HIP(hipMemcpy(p.items, sorted.data(), sizeof(int4) * sorted.size(), hipMemcpyHostToDevice));
    int dev = 0;
    PCMS_HIP(hipGetDevice(&dev));
    // host views of every problem's grid (for the problems of dimension > 3)
    p.views.assign(n, Grid{});
    for (int q = 0; q < n; ++q) {
        const BatchProb &B = p.hp[q];
        Grid &G = p.views[q];
        G.dim = B.dim;
        G.n_src = B.n_src;
        G.n_cells_cap = B.cells_cap;
        for (int k = 0; k < kMaxDim; ++k) G.g[k] = B.g[k];
        G.params = p.params + q;
        G.cell_start = p.cs + B.cs_off;
        G.perm = p.perm + B.src_off;
        G.iperm = p.iperm + B.src_off;
        G.spts = p.spts + B.spts_off;
        G.spts32 = p.spts32 + B.s32_off;
        G.sq = p.sq + B.s32_off;
        G.device = dev;
    }
    return PCMS_OK;
}

pcms_status batch_enqueue(BatchPlan &p, hipStream_t s)
{
    const int n = p.n;
    const int tpb = 256;
    k_batch_init<<<grid_for((int64_t)n * kMaxDim, tpb), tpb, 0, s>>>(p.bb, n, p.summary);
    PCMS_HIP(hipGetLastError());
    k_batch_bbox<<<grid_for((p.n_src_tot + kChunk - 1) / kChunk, 1), 256, 0, s>>>(p.probs_d, p.src_pref, n,
                                                                                 p.bb);
    PCMS_HIP(hipGetLastError());
    k_batch_params<<<grid_for(n, 64), 64, 0, s>>>(p.probs_d, n, p.bb, row_slices(), p.params);
    PCMS_HIP(hipGetLastError());
    k_batch_src_keys<<<grid_for(p.n_src_tot, tpb), tpb, 0, s>>>(p.probs_d, p.params, p.src_pref, n,
                                                               p.k0, p.v0);
    PCMS_HIP(hipGetLastError());
    pcms_status st = sort_pairs(p.k0, p.v0, p.k1, p.v1, (int)p.n_src_tot, p.key_bits, p.hist,
                                p.scan, s);
    if (st != PCMS_OK) return st;
    k_batch_cell_start<<<grid_for(p.cs_tot, tpb), tpb, 0, s>>>(p.probs_d, p.params, p.cs_pref, n,
                                                              p.k0, p.cs);
    PCMS_HIP(hipGetLastError());
    k_batch_gather_pts<<<grid_for(p.n_src_tot, tpb), tpb, 0, s>>>(p.probs_d, p.params, p.src_pref,
                                                                 n, p.v0, p.spts, p.spts32, p.sq,
                                                                 p.perm, p.iperm);
    PCMS_HIP(hipGetLastError());
    k_batch_scatter_vals<<<grid_for(p.n_src_tot, tpb), tpb, 0, s>>>(p.probs_d, p.src_pref, n,
                                                                   p.iperm, p.svals);
    PCMS_HIP(hipGetLastError());
    if (p.n_tgt_tot > 0) {
        k_batch_tgt_keys<<<grid_for(p.n_tgt_tot, tpb), tpb, 0, s>>>(p.probs_d, p.params, p.tgt_pref,
                                                                   n, p.k0, p.v0);
        PCMS_HIP(hipGetLastError());
        st = sort_pairs(p.k0, p.v0, p.k1, p.v1, (int)p.n_tgt_tot, p.tkey_bits, p.hist, p.scan, s);
        if (st != PCMS_OK) return st;
        k_batch_tperm<<<grid_for(p.n_tgt_tot, tpb), tpb, 0, s>>>(p.tgt_pref, n, p.v0, p.tperm);
        PCMS_HIP(hipGetLastError());
    }
    if (p.n_items > 0) {
        BArgs b{};
        b.probs = p.probs_d;
        b.params = p.params;
        b.cs = p.cs;
        b.spts = p.spts;
        b.spts32 = p.spts32;
        b.sq = p.sq;
        b.perm = p.perm;
        b.tperm = p.tperm;
        b.svals = p.svals;
        b.items = p.items;
        b.summary = p.summary;
        b.weight = p.weight;
        b.lambda = p.lambda;
        const size_t shm = (size_t)p.block * p.max_stride * sizeof(int);
        // one launch per class present, in class order
        for (int c = 0; c < kBatchClasses; ++c) {
            if (p.cls_end[c] <= p.cls_begin[c]) continue;
            b.item_begin = p.cls_begin[c];
            b.item_end = p.cls_end[c];
            st = p.precision == PCMS_FP64  ? batch_launch<PCMS_FP64>(c, b, p.block, shm, s)
               : p.precision == PCMS_MIXED ? batch_launch<PCMS_MIXED>(c, b, p.block, shm, s)
                                           : batch_launch<PCMS_MIXED_REFINE>(c, b, p.block, shm, s);
            if (st != PCMS_OK) return st;
        }
    }
    for (int q : p.outer) {
        const BatchProb &B = p.hp[q];
        pcms_radius r{B.mode, B.k, B.n_min, B.max_iter, B.r};
        LaunchSpec ls{&p.views[q], B.tgt, p.tperm + B.tgt_off, B.n_tgt, r, B.k_cap, p.block, p.summary};
        st = launch_transfer(ls, p.svals + B.sval_off, B.nf, B.degree, p.weight, p.precision, p.lambda,
                             B.out, nullptr, B.status, s);
        if (st != PCMS_OK) return st;
    }
    return PCMS_OK;
}

pcms_status batch_copy_summary(const int32_t *from, int32_t *to, hipStream_t s)
{
    k_copy_summary<<<1, 64, 0, s>>>(from, to);
    PCMS_HIP(hipGetLastError());
    return PCMS_OK;
}

}  // namespace pcms
