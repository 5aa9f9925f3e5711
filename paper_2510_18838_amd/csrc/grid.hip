// Uniform-grid spatial hash (PCMS paper, Section 3.3: a single-level uniform
// grid as the point-localisation structure), built on the GPU:
//   bounding box -> bucket sizing -> bucket id per point -> stable LSD radix
//   sort of the bucket ids (8-bit digits, LDS histograms and LDS wave
//   multisplit ranking) -> per-bucket start offsets -> sorted coordinates.
// The sort is stable, so within a bucket sources keep ascending index order
// and the whole layout is deterministic.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>

#include <algorithm>

#include "internal.h"
#include "launch_common.h"

namespace pcms {

namespace {

constexpr int kSortThreads = 256;          // 4 waves of 64
constexpr int kSortRounds = 16;            // items per thread per block
constexpr int kSortItems = kSortThreads * kSortRounds;
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4 * kScanThreads;

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

__global__ void k_bbox_init(long long *bb, int dim)
{
    int k = threadIdx.x;
    if (k < dim) {
        bb[k] = 0x7fffffffffffffffLL;              // running min
        bb[dim + k] = (long long)0x8000000000000000ULL;  // running max
    }
}

// Per-dimension min/max of the points: wave reductions, then one atomic per
// block and dimension.  Each lane takes kBboxUnroll points per step with
// their loads issued together (the grid is capped at 1024 blocks to bound
// the atomics, so a lane has several points and one at a time left the loop
// bound by load latency).
constexpr int kBboxUnroll = 4;
template <int D>
__global__ void __launch_bounds__(256) k_bbox(const double *__restrict__ pts, int64_t n, long long *bb)
{
    __shared__ double smn[4][D], smx[4][D];
    double mn[D], mx[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        mn[k] = INFINITY;
        mx[k] = -INFINITY;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i0 < n;
         i0 += kBboxUnroll * stride) {
        double x[kBboxUnroll][D];
#pragma unroll
        for (int u = 0; u < kBboxUnroll; ++u) {
            const int64_t i = i0 + u * stride;
            const int64_t j = i < n ? i : i0;   // i0 < n: a repeat leaves min and max unchanged
#pragma unroll
            for (int k = 0; k < D; ++k) x[u][k] = pts[j * D + k];
        }
#pragma unroll
        for (int u = 0; u < kBboxUnroll; ++u)
#pragma unroll
            for (int k = 0; k < D; ++k) {
                mn[k] = fmin(mn[k], x[u][k]);
                mx[k] = fmax(mx[k], x[u][k]);
            }
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        for (int off = 32; off > 0; off >>= 1) {
            mn[k] = fmin(mn[k], __shfl_xor(mn[k], off));
            mx[k] = fmax(mx[k], __shfl_xor(mx[k], off));
        }
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            smn[w][k] = mn[k];
            smx[w][k] = mx[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < D) {
        const int k = threadIdx.x;
        double a = smn[0][k], b = smx[0][k];
        for (int v = 1; v < (int)(blockDim.x >> 6); ++v) {
            a = fmin(a, smn[v][k]);
            b = fmax(b, smx[v][k]);
        }
        if (a <= b) {
            atomicMin(&bb[k], ordered_key(a));
            atomicMax(&bb[D + k], ordered_key(b));
        }
    }
}

// Chooses the bucket widths (one thread).
__global__ void k_grid_params(const long long *bb, int dim, int64_t n, const double *g,
                              double cell_width, double pts_per_cell, int cap, int sub,
                              GridParams *gp)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double lo[kMaxDim], hi[kMaxDim];
    for (int k = 0; k < dim; ++k) {
        lo[k] = ordered_val(bb[k]);
        hi[k] = ordered_val(bb[dim + k]);
    }
    grid_params_compute(lo, hi, dim, n, g, cell_width, pts_per_cell, cap, sub, gp);
}

template <int D>
__global__ void k_bucket_keys(const GridParams *__restrict__ gp, const double *__restrict__ pts,
                              int64_t n, unsigned *__restrict__ keys, int *__restrict__ vals)
{
    const GridParams &p = *gp;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int id = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) id += bucket_of(p, k, pts[i * D + k]) * p.stride[k];
        keys[i] = (unsigned)id;
        vals[i] = (int)i;
    }
}

// Processing-order keys of the targets (tiled Morton order, target_key).
template <int D>
__global__ void k_target_keys(const GridParams *__restrict__ gp, const double *__restrict__ pts,
                              int64_t n, unsigned *__restrict__ keys, int *__restrict__ vals)
{
    GridParams p = *gp;
    p.dim = D;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double x[D];
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = pts[i * D + k];
        keys[i] = target_key(p, x);
        vals[i] = (int)i;
    }
}

template <int D>
void launch_bucket_keys(const GridParams *gp, const double *pts, int64_t n, unsigned *keys,
                        int *vals, int blocks, hipStream_t s)
{
    k_bucket_keys<D><<<blocks, 256, 0, s>>>(gp, pts, n, keys, vals);
}

pcms_status bucket_keys(int dim, const GridParams *gp, const double *pts, int64_t n,
                        unsigned *keys, int *vals, int blocks, hipStream_t s)
{
    switch (dim) {
    case 1: launch_bucket_keys<1>(gp, pts, n, keys, vals, blocks, s); break;
    case 2: launch_bucket_keys<2>(gp, pts, n, keys, vals, blocks, s); break;
    case 3: launch_bucket_keys<3>(gp, pts, n, keys, vals, blocks, s); break;
    case 4: launch_bucket_keys<4>(gp, pts, n, keys, vals, blocks, s); break;
    default: launch_bucket_keys<5>(gp, pts, n, keys, vals, blocks, s); break;
    }
    PCMS_HIP(hipGetLastError());
    return PCMS_OK;
}

pcms_status bbox(int dim, const double *pts, int64_t n, long long *bb, hipStream_t s)
{
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
    switch (dim) {
    case 1: k_bbox<1><<<blocks, 256, 0, s>>>(pts, n, bb); break;
    case 2: k_bbox<2><<<blocks, 256, 0, s>>>(pts, n, bb); break;
    case 3: k_bbox<3><<<blocks, 256, 0, s>>>(pts, n, bb); break;
    case 4: k_bbox<4><<<blocks, 256, 0, s>>>(pts, n, bb); break;
    default: k_bbox<5><<<blocks, 256, 0, s>>>(pts, n, bb); break;
    }
    PCMS_HIP(hipGetLastError());
    return PCMS_OK;
}

// --- stable LSD radix sort, 8-bit digits --------------------------------------

__global__ void __launch_bounds__(kSortThreads)
k_digit_hist(const unsigned *__restrict__ keys, int n, int shift, int *__restrict__ hist, int nb)
{
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int base = blockIdx.x * kSortItems;
    for (int r = 0; r < kSortRounds; ++r) {
        int i = base + r * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];   // digit-major
}

// One block's kSortItems keys: each is ranked within its digit in block
// order (the wave multisplit of every round against the block's running
// digit counts), placed digit-sorted in LDS, and then written out so that
// consecutive threads store consecutive slots of one digit's run (the run
// starts at the block's global offset for the digit).  Writing straight
// from the rounds stored every key to an isolated slot; the reorder makes
// the stores whole segments.  Stable: a digit's keys keep their block order,
// and the blocks their order through the digit-major offsets.
__global__ void __launch_bounds__(kSortThreads)
k_digit_scatter(const unsigned *__restrict__ kin, const int *__restrict__ vin, int n, int shift,
                const int *__restrict__ offs, int nb, unsigned *__restrict__ kout,
                int *__restrict__ vout)
{
    __shared__ int running[256];
    __shared__ int wave_cnt[4][256];
    __shared__ int lstart[257];
    __shared__ unsigned skey[kSortItems];
    __shared__ int sval[kSortItems];
    const int t = threadIdx.x;
    const int w = t >> 6;
    const int lane = t & 63;
    running[t] = 0;
    const int base = blockIdx.x * kSortItems;
    unsigned key_r[kSortRounds];
    int val_r[kSortRounds], lpos_r[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        lpos_r[r] = -1;
        key_r[r] = 0u;
        val_r[r] = 0;
        if (base + r * kSortThreads >= n) continue;      // uniform across the block
        const int i = base + r * kSortThreads + t;
        const bool valid = i < n;
        const unsigned key = valid ? kin[i] : 0u;
        const int val = valid ? vin[i] : 0;
        const int digit = (key >> shift) & 255;
        unsigned long long bits[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) bits[b] = __ballot((digit >> b) & 1);
        const unsigned long long mask = digit_match(__ballot(valid), bits, digit);
        wave_cnt[0][t] = 0;
        wave_cnt[1][t] = 0;
        wave_cnt[2][t] = 0;
        wave_cnt[3][t] = 0;
        __syncthreads();
        if (valid && (mask & lanes_below(lane)) == 0) wave_cnt[w][digit] = __popcll(mask);
        __syncthreads();
        if (valid) {
            lpos_r[r] = scatter_slot(running[digit], wave_cnt, w, digit, mask, lane);
            key_r[r] = key;
            val_r[r] = val;
        }
        __syncthreads();
        running[t] += wave_cnt[0][t] + wave_cnt[1][t] + wave_cnt[2][t] + wave_cnt[3][t];
        __syncthreads();
    }
    // lstart = exclusive scan of the block's digit counts (Hillis-Steele)
    int c = running[t];
    lstart[t + 1] = c;
    if (t == 0) lstart[0] = 0;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int x = t >= off ? lstart[t + 1 - off] : 0;
        __syncthreads();
        lstart[t + 1] += x;
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        if (lpos_r[r] >= 0) {
            const int p = lstart[(key_r[r] >> shift) & 255] + lpos_r[r];
            skey[p] = key_r[r];
            sval[p] = val_r[r];
        }
    }
    __syncthreads();
    const int nvalid = min(kSortItems, n - base);
    for (int j = t; j < nvalid; j += kSortThreads) {
        const unsigned key = skey[j];
        const int d = (key >> shift) & 255;
        const int pos = offs[d * nb + blockIdx.x] + (j - lstart[d]);
        kout[pos] = key;
        vout[pos] = sval[j];
    }
}

// --- exclusive scan of int32 (3 phases, recursive on the block sums) ----------

__global__ void __launch_bounds__(kScanThreads)
k_scan_blocks(int *__restrict__ data, int n, int *__restrict__ sums)
{
    __shared__ int s[kScanThreads];
    int base = blockIdx.x * kScanItems + threadIdx.x * 4;
    int v[4];
    int local = 0;
    for (int j = 0; j < 4; ++j) {
        v[j] = (base + j < n) ? data[base + j] : 0;
        local += v[j];
    }
    s[threadIdx.x] = local;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int x = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += x;
        __syncthreads();
    }
    int run = s[threadIdx.x] - local;   // exclusive prefix of this thread
    for (int j = 0; j < 4; ++j) {
        if (base + j < n) data[base + j] = run;
        run += v[j];
    }
    if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = s[threadIdx.x];
}

__global__ void k_scan_add(int *__restrict__ data, int n, const int *__restrict__ sums)
{
    int i = blockIdx.x * kScanItems + threadIdx.x;
    int add = sums[blockIdx.x];
    for (int j = 0; j < 4; ++j, i += kScanThreads)
        if (i < n) data[i] += add;
}

pcms_status scan_exclusive(int *data, int n, int *scratch, hipStream_t s)
{
    int nb = (n + kScanItems - 1) / kScanItems;
    if (nb <= 0) return PCMS_OK;
    k_scan_blocks<<<nb, kScanThreads, 0, s>>>(data, n, scratch);
    PCMS_HIP(hipGetLastError());
    if (nb > 1) {
        pcms_status st = scan_exclusive(scratch, nb, scratch + nb, s);
        if (st != PCMS_OK) return st;
        k_scan_add<<<nb, kScanThreads, 0, s>>>(data, n, scratch);
        PCMS_HIP(hipGetLastError());
    }
    return PCMS_OK;
}

int scan_scratch_ints(int n)
{
    int total = 0;
    while (n > 1) {
        n = (n + kScanItems - 1) / kScanItems;
        total += n;
    }
    return total + 1;
}

int key_bits(int n_cells_cap)
{
    int b = 0;
    while (b < 31 && (1u << b) < (unsigned)n_cells_cap) ++b;
    return b;
}

// Sorts (keys, vals) stably by key bits [lo_bit, bits); the result ends up
// in (k0, v0).
pcms_status radix_sort(unsigned *k0, int *v0, unsigned *k1, int *v1, int n, int bits, int *hist,
                       int *scan_scratch, hipStream_t s, int lo_bit = 0)
{
    int nb = (n + kSortItems - 1) / kSortItems;
    if (nb == 0) return PCMS_OK;
    int passes = std::max(1, (bits - lo_bit + 7) / 8);
    unsigned *kin = k0, *kout = k1;
    int *vin = v0, *vout = v1;
    for (int ps = 0; ps < passes; ++ps) {
        int shift = lo_bit + 8 * ps;
        k_digit_hist<<<nb, kSortThreads, 0, s>>>(kin, n, shift, hist, nb);
        PCMS_HIP(hipGetLastError());
        pcms_status st = scan_exclusive(hist, 256 * nb, scan_scratch, s);
        if (st != PCMS_OK) return st;
        k_digit_scatter<<<nb, kSortThreads, 0, s>>>(kin, vin, n, shift, hist, nb, kout, vout);
        PCMS_HIP(hipGetLastError());
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    if (kin != k0) {
        PCMS_HIP(hipMemcpyAsync(k0, kin, sizeof(unsigned) * (size_t)n, hipMemcpyDeviceToDevice, s));
        PCMS_HIP(hipMemcpyAsync(v0, vin, sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, s));
    }
    return PCMS_OK;
}

size_t sort_scratch_bytes(int n)
{
    int nb = (n + kSortItems - 1) / kSortItems;
    size_t ints = (size_t)256 * nb + (size_t)scan_scratch_ints(256 * nb);
    return sizeof(unsigned) * 2 * (size_t)n + sizeof(int) * 2 * (size_t)n + sizeof(int) * ints + 256;
}

// cell_start[c] = first sorted position whose key is >= c, for c in
// [0, n_cells], in one pass over the sorted keys: each position i in 0..n
// writes the buckets it starts (cell_run).  A run of empty buckets
// shorter than kCellRun is written by the lane that ends it; longer runs are
// queued in LDS and written by the whole block, so that a large empty region
// costs a block's coalesced stores instead of one lane's.  One lane per
// position 0..n, no grid-stride (the queue is per block).
constexpr int kCellRun = 32;
constexpr int kCellStartBlock = 256;

__global__ void __launch_bounds__(kCellStartBlock)
k_cell_start(const GridParams *__restrict__ gp, const unsigned *__restrict__ keys, int n,
             int *__restrict__ cell_start)
{
    __shared__ int q_lo[kCellStartBlock], q_hi[kCellStartBlock], q_val[kCellStartBlock];
    __shared__ int q_n;
    const int n_cells = gp->n_cells;
    if (threadIdx.x == 0) q_n = 0;
    __syncthreads();
    const int i = (int)blockIdx.x * kCellStartBlock + (int)threadIdx.x;
    if (i <= n) {
        int lo, hi;
        cell_run(keys, n, n_cells, i, lo, hi);
        if (hi - lo < kCellRun) {
            for (int c = lo; c <= hi; ++c) cell_start[c] = i;
        } else {
            const int e = atomicAdd(&q_n, 1);
            q_lo[e] = lo;
            q_hi[e] = hi;
            q_val[e] = i;
        }
    }
    __syncthreads();
    const int m = q_n;
    for (int e = 0; e < m; ++e)
        for (int c = q_lo[e] + (int)threadIdx.x; c <= q_hi[e]; c += kCellStartBlock)
            cell_start[c] = q_val[e];
}

// Sorted coordinates with the padded stride (padding written as zero), their
// FP32 records fl32(x_k - lo_k) and fixed-point records, and the inverse
// permutation.
template <int D>
__global__ void k_gather_pts(const double *__restrict__ src, const int *__restrict__ perm,
                             const GridParams *__restrict__ gpp, int64_t n,
                             double *__restrict__ spts, float *__restrict__ spts32,
                             uint32_t *__restrict__ sq, int *__restrict__ iperm)
{
    constexpr int DP = padded_dim(D);
    const GridParams gp = *gpp;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = perm[p];
        write_records<D>(src + j * D, gp, spts + p * DP, spts32 + p * D, sq + p * D);
        iperm[j] = (int)p;
    }
}

// Fields into bucket order, [n][nf]: read each field coalesced in source
// order, write the whole row of a source at its sorted slot.
// Field values of source j to its sorted slot as one record of padded_dim(nf)
// doubles (the padding written as zero): each field is read coalesced in
// source order, and the record is written in whole 16-byte words (a scattered
// 8-byte store per field left the record's line to be merged in pieces).
__global__ void k_scatter_vals(const double *__restrict__ vals, const int *__restrict__ iperm,
                               int64_t n, int nf, double *__restrict__ svals)
{
    const int nfs = padded_dim(nf);
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        double *row = svals + (int64_t)iperm[j] * nfs;
        int l = 0;
        for (; l + 8 <= nf; l += 8) {
            double v[8];
#pragma unroll
            for (int h = 0; h < 8; ++h) v[h] = vals[(int64_t)(l + h) * n + j];
#pragma unroll
            for (int h = 0; h < 8; h += 2)
                *reinterpret_cast<double2 *>(row + l + h) = make_double2(v[h], v[h + 1]);
        }
        for (; l < nfs; l += 2) {
            const double a = vals[(int64_t)l * n + j];
            const double b = l + 1 < nf ? vals[(int64_t)(l + 1) * n + j] : 0.0;
            *reinterpret_cast<double2 *>(row + l) = make_double2(a, b);
        }
    }
}

// out[l][t] = stage[t][l] for l < nf: each thread reads its target's record
// in 16-byte words and writes one coalesced element per field.
__global__ void k_unstage(const double *__restrict__ stage, int64_t n, int nf, int nfs,
                          double *__restrict__ out)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const double *rec = stage + t * nfs;
        for (int l = 0; l < nf; l += 2) {
            const double2 v = *reinterpret_cast<const double2 *>(rec + l);
            out[(int64_t)l * n + t] = v.x;
            if (l + 1 < nf) out[(int64_t)(l + 1) * n + t] = v.y;
        }
    }
}

int grid_blocks(int64_t n, int tpb)
{
    int64_t b = (n + tpb - 1) / tpb;
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 65536);
}

}  // namespace

int row_slices()
{
    const char *env = getenv("PCMS_ROW_SLICES");
    const int v = env ? atoi(env) : 0;
    return v == 1 || v == 2 || v == 4 || v == 8 || v == 16 ? v : kRowSlices;
}

int cells_cap_for(int64_t n_src)
{
    int64_t c = 2 * n_src + 64;
    return (int)std::min<int64_t>(c, (int64_t)1 << 30);
}

size_t grid_build_scratch_bytes(int64_t n_src)
{
    // bbox keys + metric copy + sort buffers
    return 256 + sort_scratch_bytes((int)n_src) + 64 * sizeof(double);
}

pcms_status source_bbox_params(Grid *grid, const double *src, double *gdev, long long *bb,
                               double cell_width, double pts_per_cell, hipStream_t s)
{
    const int dim = grid->dim;
    const int n = (int)grid->n_src;
    PCMS_HIP(hipMemcpyAsync(gdev, grid->g, sizeof(double) * dim, hipMemcpyHostToDevice, s));
    k_bbox_init<<<1, 64, 0, s>>>(bb, dim);
    PCMS_HIP(hipGetLastError());
    pcms_status st = bbox(dim, src, n, bb, s);
    if (st != PCMS_OK) return st;
    k_grid_params<<<1, 1, 0, s>>>(bb, dim, n, gdev, cell_width, pts_per_cell, grid->n_cells_cap,
                                  row_slices(), grid->params);
    PCMS_HIP(hipGetLastError());
    return PCMS_OK;
}

pcms_status gather_records(Grid *grid, const double *src, hipStream_t s)
{
    const int n = (int)grid->n_src;
    const int blocks = grid_blocks(n, 256);
    switch (grid->dim) {
#define PCMS_GATHER(DD)                                                                          \
    case DD:                                                                                     \
        k_gather_pts<DD><<<blocks, 256, 0, s>>>(src, grid->perm, grid->params, n, grid->spts,    \
                                                grid->spts32, grid->sq, grid->iperm);            \
        break;
        PCMS_GATHER(1) PCMS_GATHER(2) PCMS_GATHER(3) PCMS_GATHER(4) PCMS_GATHER(5)
#undef PCMS_GATHER
    }
    PCMS_HIP(hipGetLastError());
    return PCMS_OK;
}

pcms_status build_grid_device(Grid *grid, const double *src, double cell_width,
                              double pts_per_cell, hipStream_t s,
                              const std::function<pcms_status()> *after_params)
{
    const int n = (int)grid->n_src;
    size_t bytes = grid_build_scratch_bytes(n);
    void *raw = nullptr;
    pcms_status st = scratch_alloc(&raw, bytes, s);
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
    int nb = (n + kSortItems - 1) / kSortItems;
    int *hist = (int *)cur;
    cur += sizeof(int) * (size_t)256 * nb;
    int *scan_scratch = (int *)cur;

    if ((st = source_bbox_params(grid, src, gdev, bb, cell_width, pts_per_cell, s)) != PCMS_OK)
        return st;
    if (after_params && (st = (*after_params)()) != PCMS_OK) return st;
    if ((st = bucket_keys(grid->dim, grid->params, src, n, k0, grid->perm, grid_blocks(n, 256), s)) != PCMS_OK)
        return st;
    st = radix_sort(k0, grid->perm, k1, v1, n, key_bits(grid->n_cells_cap), hist, scan_scratch, s);
    if (st != PCMS_OK) return st;
    k_cell_start<<<(unsigned)(((int64_t)n + kCellStartBlock) / kCellStartBlock), kCellStartBlock, 0,
                   s>>>(grid->params, k0, n, grid->cell_start);
    PCMS_HIP(hipGetLastError());
    if ((st = gather_records(grid, src, s)) != PCMS_OK) return st;
    scratch_free(raw, s);
    return PCMS_OK;
}

size_t sort_targets_bytes(int64_t n_tgt) { return sort_scratch_bytes((int)n_tgt); }

pcms_status sort_targets(const Grid *grid, const double *tgt, int64_t n_tgt, int *tperm,
                         hipStream_t s, void *ws)
{
    const int n = (int)n_tgt;
    void *raw = nullptr;
    pcms_status st;
    if (!ws) {
        st = scratch_alloc(&raw, sort_scratch_bytes(n), s);
        if (st != PCMS_OK) return st;
    }
    char *cur = (char *)(ws ? ws : raw);
    unsigned *k0 = (unsigned *)cur;
    cur += sizeof(unsigned) * (size_t)n;
    unsigned *k1 = (unsigned *)cur;
    cur += sizeof(unsigned) * (size_t)n;
    int *v1 = (int *)cur;
    cur += sizeof(int) * (size_t)n;
    int nb = (n + kSortItems - 1) / kSortItems;
    int *hist = (int *)cur;
    cur += sizeof(int) * (size_t)256 * nb;
    int *scan_scratch = (int *)cur;
    // tiled Morton order when its keys fit 32 bits, else bucket order; on an
    // LBVH (one bucket) the Morton order of the tree's box
    const double bound = tile_key_bound((double)grid->n_cells_cap, grid->dim);
    int bits;
    if (grid->lbvh) {
        if ((st = morton_keys(grid->dim, grid->params, tgt, n, k0, tperm, s)) != PCMS_OK) return st;
        bits = 32;
    } else if (bound < 4294967295.0) {
        const int blocks = grid_blocks(n, 256);
        switch (grid->dim) {
        case 1: k_target_keys<1><<<blocks, 256, 0, s>>>(grid->params, tgt, n, k0, tperm); break;
        case 2: k_target_keys<2><<<blocks, 256, 0, s>>>(grid->params, tgt, n, k0, tperm); break;
        case 3: k_target_keys<3><<<blocks, 256, 0, s>>>(grid->params, tgt, n, k0, tperm); break;
        case 4: k_target_keys<4><<<blocks, 256, 0, s>>>(grid->params, tgt, n, k0, tperm); break;
        default: k_target_keys<5><<<blocks, 256, 0, s>>>(grid->params, tgt, n, k0, tperm); break;
        }
        PCMS_HIP(hipGetLastError());
        bits = 0;
        while (bits < 32 && (double)(1ull << bits) < bound) ++bits;
    } else {
        if ((st = bucket_keys(grid->dim, grid->params, tgt, n, k0, tperm, grid_blocks(n, 256), s)) != PCMS_OK)
            return st;
        bits = key_bits(grid->n_cells_cap);
    }
    // only the key's top target_key_bits() bits are sorted on: the order is
    // for locality (a wave's targets close together), and the lowest bits
    // of the finest keys buy no measurable locality for their extra pass
    st = radix_sort(k0, tperm, k1, v1, n, bits, hist, scan_scratch, s,
                    std::max(bits - target_key_bits(), 0));
    if (st != PCMS_OK) return st;
    if (raw) scratch_free(raw, s);
    return PCMS_OK;
}

int target_key_bits()
{
    const char *env = getenv("PCMS_TARGET_KEY_BITS");
    const int v = env ? atoi(env) : 0;
    return v >= 8 && v <= 32 ? v : kTargetKeyBits;
}

pcms_status sort_pairs(unsigned *k0, int *v0, unsigned *k1, int *v1, int n, int bits, int *hist,
                       int *scan_scratch, hipStream_t s)
{
    return radix_sort(k0, v0, k1, v1, n, bits, hist, scan_scratch, s);
}

pcms_status exclusive_scan(int *data, int n, int *scratch, hipStream_t s)
{
    return scan_exclusive(data, n, scratch, s);
}

size_t exclusive_scan_ints(int n) { return (size_t)scan_scratch_ints(n); }

size_t sort_hist_ints(int n) { return (size_t)256 * ((n + kSortItems - 1) / kSortItems); }

size_t sort_scan_ints(int n) { return (size_t)scan_scratch_ints((int)sort_hist_ints(n)); }

int bits_for(double bound)
{
    int b = 0;
    while (b < 32 && (double)(1ull << b) < bound) ++b;
    return b;
}

pcms_status unstage_fields(const double *stage, int64_t n_tgt, int n_fields, double *out,
                           hipStream_t s)
{
    k_unstage<<<grid_blocks(n_tgt, 256), 256, 0, s>>>(stage, n_tgt, n_fields,
                                                      padded_dim(n_fields), out);
    PCMS_HIP(hipGetLastError());
    return PCMS_OK;
}

pcms_status gather_values(const Grid *grid, const double *vals, int n_fields, double *svals,
                          hipStream_t s)
{
    k_scatter_vals<<<grid_blocks(grid->n_src, 256), 256, 0, s>>>(vals, grid->iperm, grid->n_src,
                                                                n_fields, svals);
    PCMS_HIP(hipGetLastError());
    return PCMS_OK;
}

}  // namespace pcms
