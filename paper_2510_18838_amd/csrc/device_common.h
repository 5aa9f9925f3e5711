// Declarations shared by the kernels and their host emulation build.
//
// Everything here is plain arithmetic on plain pointers, marked host+device,
// so the same code runs inside the HIP kernels and in the CPU emulation that
// the test-suite builds with address sanitising to check indexing.
#pragma once

#include <stdint.h>

#ifdef PCMS_HOST_EMULATION
#include <algorithm>
#include <cmath>
#define PCMS_HD
#define PCMS_INLINE inline
using std::exp;
using std::fabs;
using std::floor;
using std::fmax;
using std::fmin;
using std::isinf;
using std::isnan;
using std::max;
using std::min;
using std::nextafter;
using std::pow;
using std::rint;
using std::log2;
using std::ldexp;
using std::ceil;
using std::sqrt;
// Called by the emulation build when a lane addresses LDS words outside its own.
[[noreturn]] void pcms_emu_lds_fault(int e, int words);
// The HIP vector type the walks load records with.
struct alignas(16) float4 {
    float x, y, z, w;
};
// Work counters of the emulation build (rows walked, candidates tested, walks,
// candidates of FP32 walks that needed their FP64 record, LBVH records read).
extern thread_local long long pcms_emu_rows, pcms_emu_cands, pcms_emu_walks, pcms_emu_exact,
    pcms_emu_nodes;
// Collective operations of a lane group, provided by the emulation driver:
// the G lanes of a group run as G threads meeting at a barrier per operation.
struct EmuGroup;
unsigned pcms_emu_ballot(EmuGroup *g, int q, bool p);
double pcms_emu_sum(EmuGroup *g, int q, double x);
float pcms_emu_sum(EmuGroup *g, int q, float x);
int pcms_emu_sum(EmuGroup *g, int q, int x);
double pcms_emu_min(EmuGroup *g, int q, double x);
int pcms_emu_min(EmuGroup *g, int q, int x);
void pcms_emu_sync(EmuGroup *g, int q);
#else
#include <hip/hip_runtime.h>
#define PCMS_HD __host__ __device__
#define PCMS_INLINE __forceinline__
#endif

#include "pcms_mls.h"

namespace pcms {

constexpr int kMaxDim = PCMS_MAX_DIM;
// Slices of dimension 0 per bucket width in the grids the library builds.
constexpr int kRowSlices = 4;
constexpr int kMaxKcap = PCMS_MAX_KCAP;

// Device-resident description of a uniform grid.  Bucket coordinates of a
// point x are c_k = clamp(floor((x_k - lo_k) * inv_w_k), 0, n_k - 1); the
// linear bucket id is row-major with dimension 0 fastest, so the buckets of
// one "row" (fixed c_1..c_{d-1}) are contiguous in sorted order.  Dimension
// 0 is cut `sub` times finer than the others (w_0 = w / sub in metric
// units): a search pays per row it visits, not per bucket, so the finer
// slices narrow each row's range to the ball's chord at no cost in rows.
struct GridParams {
    int dim;
    int sub;    // slices of dimension 0 per bucket width (1: cubic buckets)
    int n_cells;
    int n[kMaxDim];
    int stride[kMaxDim];
    double lo[kMaxDim];
    double hi[kMaxDim];     // upper corner of the sources' bounding box
    double w[kMaxDim];      // bucket width, raw coordinates
    double inv_w[kMaxDim];  // 1 / w
    double g[kMaxDim];      // metric factors
    double qs[kMaxDim];     // quantum of the 32-bit source records (a power of two)
    double iqs[kMaxDim];    // 1 / qs
    double density;         // sources per unit metric volume of the bounding box
};

PCMS_HD PCMS_INLINE int bucket_of(const GridParams &p, int k, double x)
{
    double f = floor((x - p.lo[k]) * p.inv_w[k]);
    f = fmax(f, 0.0);                     // also maps NaN to 0
    f = fmin(f, (double)(p.n[k] - 1));
    return (int)f;
}

// Bucket sizing from the bounding box [lo, hi]: width cell_width (metric
// units) if > 0, else sized for about pts_per_cell sources per cubic bucket
// of that width; dimension 0 is then cut into `sub` slices per width (a
// power of two; 1 in one dimension).  Until the bucket count fits `cap`,
// sub halves first, then the width grows.
PCMS_HD inline void grid_params_compute(const double *lo, const double *hi, int dim, int64_t n,
                                        const double *g, double cell_width, double pts_per_cell,
                                        int cap, int sub, GridParams *out)
{
    GridParams p;
    p.dim = dim;
    p.sub = dim > 1 && sub > 1 ? sub : 1;
    double ext[kMaxDim];
    double vol = 1.0;
    int d_eff = 0;
    for (int k = 0; k < kMaxDim; ++k) {
        p.lo[k] = 0.0;
        p.hi[k] = 0.0;
        p.g[k] = 1.0;
        p.n[k] = 1;
        p.w[k] = 1.0;
        p.inv_w[k] = 1.0;
        p.stride[k] = 0;
        p.qs[k] = 1.0;
        p.iqs[k] = 1.0;
        ext[k] = 0.0;
    }
    for (int k = 0; k < dim; ++k) {
        p.g[k] = g[k];
        double l = lo[k], h = hi[k];
        if (!(l <= h)) {
            l = 0.0;
            h = 0.0;
        }
        p.lo[k] = l;
        p.hi[k] = h;
        // quantum 2^(E - 32) with 2^E just above the extent: every source of
        // the box maps to an integer in [0, 2^32)
        if (h > l) {
            const int e = (int)ceil(log2((h - l) * (1.0 + 1.0 / 1048576.0)));
            p.qs[k] = ldexp(1.0, e - 32);
            p.iqs[k] = ldexp(1.0, 32 - e);
        }
        ext[k] = (h - l) * p.g[k];
        if (ext[k] > 0.0) {
            vol *= ext[k];
            d_eff++;
        }
    }
    double wm;
    if (cell_width > 0.0) {
        wm = cell_width;
    } else {
        double ppc = pts_per_cell > 0.0 ? pts_per_cell : (double)(1 << dim);
        wm = d_eff > 0 ? pow(ppc * vol / (double)(n > 0 ? n : 1), 1.0 / d_eff) : 1.0;
        if (!(wm > 0.0) || !(wm < INFINITY)) wm = 1.0;
    }
    double total = 1.0;
    for (int it = 0; it < 4000; ++it) {
        total = 1.0;
        for (int k = 0; k < dim; ++k) {
            const double wk = k == 0 ? wm / p.sub : wm;
            if (ext[k] > 0.0) {
                double nk = floor(ext[k] / wk) + 1.0;
                nk = fmin(nk, 1073741824.0);
                p.n[k] = (int)nk;
                p.w[k] = wk / p.g[k];
            } else {
                p.n[k] = 1;
                p.w[k] = 1.0 / p.g[k];
            }
            p.inv_w[k] = 1.0 / p.w[k];
            total *= (double)p.n[k];
        }
        if (total <= (double)cap) break;
        if (p.sub > 1)
            p.sub /= 2;
        else
            wm *= 1.25;
    }
    if (total > (double)cap) {      // never exceed the allocated bucket count
        p.sub = 1;
        for (int k = 0; k < dim; ++k) {
            p.n[k] = 1;
            p.w[k] = (ext[k] > 0.0 ? 2.0 * ext[k] : 1.0) / p.g[k];
            p.inv_w[k] = 1.0 / p.w[k];
        }
    }
    int s = 1;
    for (int k = 0; k < dim; ++k) {
        p.stride[k] = s;
        s *= p.n[k];
    }
    p.n_cells = s;
    p.density = d_eff > 0 ? (double)n / vol : 0.0;
    *out = p;
}

// The buckets whose first sorted position is i (0 <= i <= n), from the n
// sorted bucket keys (each < n_cells): [lo, hi], none when hi < lo.
// Position 0 starts [0, key[0]], position i (0 < i < n) starts
// (key[i-1], key[i]] and the end n starts (key[n-1], n_cells].
PCMS_HD PCMS_INLINE void cell_run(const unsigned *keys, int n, int n_cells, int i, int &lo, int &hi)
{
    lo = i == 0 ? 0 : (int)keys[i - 1] + 1;
    hi = i == n ? n_cells : (int)keys[i];
}

PCMS_HD PCMS_INLINE unsigned bucket_key(const GridParams &p, const double *x)
{
    int id = 0;
    for (int k = 0; k < p.dim; ++k) id += bucket_of(p, k, x[k]) * p.stride[k];
    return (unsigned)id;
}

// Processing order of the targets: tiles of 8 cubic buckets per side (the
// slices of dimension 0 merged; tiled in every dimension with at least 16
// such buckets) in row-major order, and Morton order of the buckets inside
// a tile, so that a wave's consecutive targets cover a compact block of
// buckets.  Keys are below tile_key_bound(n_cells, dim).
PCMS_HD PCMS_INLINE unsigned target_key(const GridParams &p, const double *x)
{
    unsigned tile = 0, tstride = 1, local = 0;
    int nt = 0;   // tiled dimensions so far
    int tiled[kMaxDim], c[kMaxDim];
    int nk[kMaxDim];
    for (int k = 0; k < p.dim; ++k) {
        // the slices of dimension 0 are merged back into cubic buckets
        const int s = k == 0 ? p.sub : 1;
        c[k] = bucket_of(p, k, x[k]) / s;
        nk[k] = (p.n[k] + s - 1) / s;
        tiled[k] = nk[k] >= 16;
        nt += tiled[k];
    }
    int r = 0;
    for (int k = 0; k < p.dim; ++k) {
        const int sh = tiled[k] ? 3 : 0;
        tile += (unsigned)(c[k] >> sh) * tstride;
        tstride *= (unsigned)((nk[k] + (1 << sh) - 1) >> sh);
        if (tiled[k]) {
            for (int b = 0; b < 3; ++b) local |= (unsigned)((c[k] >> b) & 1) << (b * nt + r);
            ++r;
        }
    }
    return (tile << (3 * nt)) | local;
}

// Upper bound of the target keys: each tiled dimension rounds its bucket
// count up to a multiple of 8 (at most 23/16 of it, as it has >= 16).
inline double tile_key_bound(double n_cells, int dim)
{
    double f = 1.0;
    for (int k = 0; k < dim; ++k) f *= 23.0 / 16.0;
    return n_cells * f + 1.0;
}

// Sorted source coordinates are stored with an even stride (3-D points take
// four doubles), so that every point starts on a 16-byte boundary and loads
// as whole 16-byte words.
PCMS_HD PCMS_INLINE constexpr int padded_dim(int d) { return (d + 1) & ~1; }

template <int D>
PCMS_HD PCMS_INLINE void load_src(const double *__restrict__ spts, int p, double (&s)[D])
{
    constexpr int DP = padded_dim(D);
    const double *b = spts + (size_t)p * DP;
#ifdef PCMS_HOST_EMULATION
    for (int k = 0; k < D; ++k) s[k] = b[k];
#else
#pragma unroll
    for (int j = 0; j < DP / 2; ++j) {
        const double2 v = reinterpret_cast<const double2 *>(b)[j];
        s[2 * j] = v.x;
        if (2 * j + 1 < D) s[2 * j + 1] = v.y;
    }
#endif
}

// Sorted sources also keep an FP32 image of their coordinates relative to
// the grid origin, fl32(s_k - lo_k), packed with no padding (a 3-D point is
// 12 bytes and loads as one 12-byte word: ten records share a 128-byte line
// instead of eight); the mixed-precision searches classify candidates from it.
PCMS_HD PCMS_INLINE constexpr int padded_dim32(int d) { return d; }

template <int D>
PCMS_HD PCMS_INLINE void load_src32(const float *__restrict__ s32, int p, float (&s)[D])
{
    // adjacent scalar loads, which the compiler merges into one wide load
    const float *b = s32 + (size_t)p * D;
#pragma unroll
    for (int k = 0; k < D; ++k) s[k] = b[k];
}

// Sorted sources also keep a 32-bit fixed-point image of their coordinates,
// q_k = round((s_k - lo_k) / qs_k) with the power-of-two quantum qs_k of
// their box, packed with no padding (a 3-D point is 12 bytes, one load).  The
// mixed-precision fit passes read it instead of the FP64 record: it places
// the source within qs_k / 2 (about 1.2e-10 of the box) of its position, and
// (q_k - (t_k - lo_k) / qs_k) * qs_k is formed in FP64 without cancellation.
PCMS_HD PCMS_INLINE uint32_t quantize(double x, double lo, double iqs)
{
    const double v = rint((x - lo) * iqs);
    return (uint32_t)fmin(fmax(v, 0.0), 4294967295.0);
}

template <int D>
PCMS_HD PCMS_INLINE void load_srcq(const uint32_t *__restrict__ sq, int p, uint32_t (&q)[D])
{
    // adjacent scalar loads, which the compiler merges into one wide load
    const uint32_t *b = sq + (size_t)p * D;
#pragma unroll
    for (int k = 0; k < D; ++k) q[k] = b[k];
}

// Fused multiply-add in the arithmetic of its operands (__builtin_fma on
// floats would promote them and compute in FP64).
PCMS_HD PCMS_INLINE float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
PCMS_HD PCMS_INLINE double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Two consecutive doubles from a 16-byte aligned address, in one load.
PCMS_HD PCMS_INLINE void load_pair(const double *__restrict__ p, double &x, double &y)
{
#ifdef PCMS_HOST_EMULATION
    x = p[0];
    y = p[1];
#else
    const double2 v = *reinterpret_cast<const double2 *>(p);
    x = v.x;
    y = v.y;
#endif
}

// Two consecutive doubles to a 16-byte aligned address, in one store.
PCMS_HD PCMS_INLINE void store_pair(double *__restrict__ p, double x, double y)
{
#ifdef PCMS_HOST_EMULATION
    p[0] = x;
    p[1] = y;
#else
    *reinterpret_cast<double2 *>(p) = make_double2(x, y);
#endif
}

// Atomic add to a word of the block's LDS.
PCMS_HD PCMS_INLINE void lds_add(int *w, int v)
{
#ifdef PCMS_HOST_EMULATION
    __atomic_fetch_add(w, v, __ATOMIC_RELAXED);
#else
    atomicAdd(w, v);
#endif
}

// --- lane groups -----------------------------------------------------------
// G consecutive lanes of a wave (G a power of two, <= 16) cooperate on one
// target.  Group operations must be reached by all G lanes together (the
// control flow around them is uniform within the group).
template <int G>
struct Grp {
    int q;   // lane index inside the group
#ifdef PCMS_HOST_EMULATION
    EmuGroup *emu;
    unsigned ballot(bool p) const { return pcms_emu_ballot(emu, q, p); }
    template <class T>
    T sum(T x) const { return pcms_emu_sum(emu, q, x); }
    template <class T>
    T min(T x) const { return pcms_emu_min(emu, q, x); }
    void sync() const { pcms_emu_sync(emu, q); }
#else
    __device__ PCMS_INLINE unsigned ballot(bool p) const
    {
        const unsigned long long m = __ballot(p);
        const int base = (int)(__lane_id() & ~(unsigned)(G - 1));
        return (unsigned)(m >> base) & ((1u << G) - 1u);
    }
    // butterfly: every lane ends with the same value, summed in the same order
    template <class T>
    __device__ PCMS_INLINE T sum(T x) const
    {
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
            T y = __shfl_xor(x, off, 64);
            x = (q & off) ? y + x : x + y;
        }
        return x;
    }
    template <class T>
    __device__ PCMS_INLINE T min(T x) const
    {
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
            T y = __shfl_xor(x, off, 64);
            x = y < x ? y : x;
        }
        return x;
    }
    // orders this lane's LDS accesses against the group's (one wavefront)
    __device__ PCMS_INLINE void sync() const
    {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
#endif
    // lanes of mask m below this one
    PCMS_HD PCMS_INLINE int below(unsigned m) const
    {
        return __builtin_popcount(m & ((1u << q) - 1u));
    }
};

// --- pieces of the stable radix-sort scatter (one 8-bit digit per pass) ------
// Lanes of one wave holding the same digit: AND of the per-bit ballots.
PCMS_HD PCMS_INLINE unsigned long long digit_match(unsigned long long valid,
                                                   const unsigned long long (&bits)[8], int digit)
{
    unsigned long long mask = valid;
    for (int b = 0; b < 8; ++b) mask &= ((digit >> b) & 1) ? bits[b] : ~bits[b];
    return mask;
}

PCMS_HD PCMS_INLINE unsigned long long lanes_below(int lane)
{
    return lane == 0 ? 0ull : ((~0ull) >> (64 - lane));
}

// Output slot of an item: block running offset of its digit, plus the items
// of the same digit in earlier waves of this round, plus earlier lanes.
PCMS_HD PCMS_INLINE int scatter_slot(int running, const int (&wave_cnt)[4][256], int w, int digit,
                                     unsigned long long mask, int lane)
{
    int pos = running + __builtin_popcountll(mask & lanes_below(lane));
    for (int v = 0; v < w; ++v) pos += wave_cnt[v][digit];
    return pos;
}

}  // namespace pcms
