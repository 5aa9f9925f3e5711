// Linear bounding volume hierarchy (LBVH) over the sorted sources: the
// alternative to the uniform grid for localising the sources near a target
// (PCMS paper, Section 3.3, which compares the two).
//
// The sources are sorted by the Morton code of their position.  The binary
// radix tree over all sorted sources (keys: code, then sorted position, so
// all keys differ and the tree has depth <= 64) is cut into leaves: the
// largest subtrees holding at most max_leaf sources (kBvhLeaf by default).
// A leaf is therefore an aligned Morton cell (or a part of one, where sources
// share a code), never a run that straddles a cell boundary, and its box
// stays compact however the density varies.  A second radix tree over the leaves (keyed by their first
// source's code, ties by leaf index) gives the internal nodes.
//
// Records (floats, a stride of bvh_stride(D) each): the nl - 1 internal nodes
// (record 0 the root), then the nl leaves (record nl - 1 + l for leaf l).  A
// record holds its box (lower then upper corner, raw coordinates rounded
// outward to FP32), then as int bits its first child's record (-1 for a
// leaf), its rope, and the sorted-source range [begin, end) it covers.  The
// rope is the record to visit after the subtree: the largest subtree that
// starts at the next leaf, i.e. the second child of the node that splits
// between the two (-1 after the last leaf).  A tree of one leaf is that
// leaf's record.  The leaf count lives only on the device; the records need
// none of it to be walked.
//
// A walk goes through the records in depth-first order without a stack:
// into the first child when a node's box is within reach, along the rope
// otherwise (and after a leaf), so leaves -- and their sources -- reach the
// callback in ascending sorted order, as in the grid's row walks.
#pragma once

#include "device_common.h"

namespace pcms {

constexpr int kBvhLeaf = 4;       // default of the most sources per leaf
constexpr int kBvhLeafMax = 64;   // largest accepted

// Record stride: box, first child, rope, source range.
PCMS_HD PCMS_INLINE constexpr int bvh_stride(int d) { return ((2 * d + 4) + 3) & ~3; }

struct BvhView {
    const float *nodes;   // [2 n_leaves - 1][bvh_stride(dim)] records
};

PCMS_HD PCMS_INLINE int bvh_int(const float *rec, int j) { return __builtin_bit_cast(int, rec[j]); }

// Construction steps shared by the device build and its CPU emulation ---------

// Spreads the low b bits of v to every dim-th bit (bit j to bit j * dim).
PCMS_HD PCMS_INLINE uint32_t bvh_spread_bits(uint32_t v, int b, int dim)
{
    uint32_t r = 0;
    for (int j = 0; j < b; ++j) r |= ((v >> j) & 1u) << (j * dim);
    return r;
}

// Morton code of x in the (single-bucket) box of gp: 32 / D bits per
// coordinate, coordinate k in bits k, k + D, ...
template <int D>
PCMS_HD PCMS_INLINE uint32_t bvh_morton(const GridParams &gp, const double *x)
{
    constexpr int B = 32 / D;
    uint32_t code = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double ext = gp.n[k] * gp.w[k];
        double f = (x[k] - gp.lo[k]) / ext;
        f = fmin(fmax(f, 0.0), 1.0);   // also maps NaN to 0
        const uint32_t q = (uint32_t)fmin(f * (double)(1ull << B), (double)((1ull << B) - 1u));
        code |= bvh_spread_bits(q, B, D) << k;
    }
    return code;
}

// Internal node i (< n - 1) of the binary radix tree over n sorted keys
// key(0..n-1), ties broken by index (Karras's construction: the direction of
// the node's range from the neighbours' common-prefix lengths, its far end by
// exponential then binary search, the split where the prefix shared with i
// ends).  Returns the node's key range [first, last] and its split: the
// first child covers [first, split], the second [split + 1, last].
template <class K>
PCMS_HD PCMS_INLINE void bvh_karras(const K &key, int n, int i, int &first, int &last, int &split)
{
    // common-prefix length of the keys of a and b (64-bit keys: code, index)
    auto delta = [&](int a, int b) -> int {
        if (b < 0 || b >= n) return -1;
        const unsigned x = key(a), y = key(b);
        if (x != y) return __builtin_clz(x ^ y);
        return 32 + __builtin_clz((unsigned)(a ^ b));
    };
    const int d = delta(i, i + 1) - delta(i, i - 1) > 0 ? 1 : -1;
    const int dmin = delta(i, i - d);
    int lmax = 2;
    while (delta(i, i + lmax * d) > dmin) lmax *= 2;
    int l = 0;
    for (int t = lmax / 2; t >= 1; t /= 2)
        if (delta(i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = delta(i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (delta(i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    split = i + s * d + min(d, 0);
    first = min(i, j);
    last = max(i, j);
}

// Leaf cuts from internal node i of the tree over the n sorted sources: the
// node splits between sources split and split + 1, which fall into
// different leaves exactly when the node holds more than max_leaf sources
// (each split belongs to one node, so every cut[] entry is written once).
PCMS_HD PCMS_INLINE void bvh_point_cut(const unsigned *codes, int n, int i, int max_leaf, int *cut)
{
    int first, last, split;
    bvh_karras([&](int j) { return codes[j]; }, n, i, first, last, split);
    cut[split] = last - first + 1 > max_leaf;
}

// Internal node i (< nl - 1) of the tree over the nl leaves (leaf l starts
// at sorted source leaf_start[l]): writes the first child's record and the
// leaf range into the node's record, and for the later passes the parents
// of both children, the second child, and the second child as the rope of
// whatever ends at the split (split_right[split]).
template <int D>
PCMS_HD PCMS_INLINE void bvh_radix_node(const unsigned *codes, const int *leaf_start, int nl, int i,
                                        float *nodes, int *parent, int *child1, int *split_right)
{
    constexpr int S = bvh_stride(D);
    int first, last, split;
    bvh_karras([&](int l) { return codes[leaf_start[l]]; }, nl, i, first, last, split);
    // records: internal node x is x, leaf x is nl - 1 + x
    const int c0 = first == split ? nl - 1 + split : split;
    const int c1 = last == split + 1 ? nl - 1 + split + 1 : split + 1;
    float *nd = nodes + (size_t)i * S;
    nd[2 * D] = __builtin_bit_cast(float, c0);
    nd[2 * D + 2] = __builtin_bit_cast(float, first);   // leaf range, until bvh_rope
    nd[2 * D + 3] = __builtin_bit_cast(float, last);
    parent[c0] = i;
    parent[c1] = i;
    child1[i] = c1;
    split_right[split] = c1;
}

// Rope and source range of record r (after every bvh_radix_node).
template <int D>
PCMS_HD PCMS_INLINE void bvh_rope(int nl, int r, float *nodes, const int *leaf_start,
                                  const int *split_right)
{
    constexpr int S = bvh_stride(D);
    float *nd = nodes + (size_t)r * S;
    int first, last;
    if (r >= nl - 1) {
        first = last = r - (nl - 1);
        nd[2 * D] = __builtin_bit_cast(float, -1);
    } else {
        first = bvh_int(nd, 2 * D + 2);
        last = bvh_int(nd, 2 * D + 3);
    }
    nd[2 * D + 1] = __builtin_bit_cast(float, last < nl - 1 ? split_right[last] : -1);
    nd[2 * D + 2] = __builtin_bit_cast(float, leaf_start[first]);
    nd[2 * D + 3] = __builtin_bit_cast(float, leaf_start[last + 1]);
}

PCMS_HD PCMS_INLINE float bvh_round_down(double x)
{
    const float f = (float)x;
    return (double)f > x ? nextafterf(f, -INFINITY) : f;
}

PCMS_HD PCMS_INLINE float bvh_round_up(double x)
{
    const float f = (float)x;
    return (double)f < x ? nextafterf(f, INFINITY) : f;
}

// FP32 box of the sorted sources [beg, end) (FP64 records, rounded outward).
template <int D>
PCMS_HD PCMS_INLINE void bvh_leaf_box(const double *spts, int beg, int end, float (&lo)[D],
                                      float (&hi)[D])
{
    constexpr int DP = padded_dim(D);
    double a[D], b[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        a[k] = INFINITY;
        b[k] = -INFINITY;
    }
    for (int p = beg; p < end; ++p)
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double x = spts[(size_t)p * DP + k];
            a[k] = fmin(a[k], x);
            b[k] = fmax(b[k], x);
        }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lo[k] = bvh_round_down(a[k]);
        hi[k] = bvh_round_up(b[k]);
    }
}

// Squared metric distance from t to the box [lo, hi] (0 inside), with the
// gaps widened by 1e-7 of the box so that the FP32 rounding of the bounds
// (already outward) and of this sum cannot exclude a source.
template <int D, bool UNIT>
PCMS_HD PCMS_INLINE double box_dist2(const GridParams &gp, const double (&t)[D], const float *lo,
                                     const float *hi)
{
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double l = (double)lo[k], h = (double)hi[k];
        double gap = fmax(fmax(l - t[k], t[k] - h), 0.0);
        gap = fmax(gap - 1e-7 * (h - l), 0.0);
        if (!UNIT) gap *= gp.g[k];
        acc = __builtin_fma(gap, gap, acc);
    }
    return acc;
}

// Conservative FP32 form of box_dist2 <= rho2 for the walks: t in FP32
// (tf), each gap shrunk by 2^-20 of |tf| + gap before it is scaled and
// squared, and the limit rounded up with a relative and an absolute slack,
// so that rounding (and underflow, which only lowers the sum) can make a box
// pass that the exact test would reject but never the reverse.  rho2 may be
// +inf.
template <int D, bool UNIT>
struct BoxTest32 {
    float tf[D], g[D], lim;
    PCMS_HD BoxTest32(const GridParams &gp, const double (&t)[D], double rho2)
    {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            tf[k] = (float)t[k];
            g[k] = UNIT ? 1.0f : (float)gp.g[k] * (1.0f + 1e-6f);
        }
        const double l = rho2 * (1.0 + 1e-5);
        float lf = (float)l;
        if ((double)lf < l) lf = nextafterf(lf, INFINITY);
        lim = lf + 1e-43f;
    }
    // rec: the record's box, lower then upper corner
    PCMS_HD PCMS_INLINE bool operator()(const float *rec) const
    {
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            float gap = fmaxf(fmaxf(rec[k] - tf[k], tf[k] - rec[D + k]), 0.0f);
            gap = fmaxf(gap - 9.5367431640625e-07f * (fabsf(tf[k]) + gap), 0.0f);
            if (!UNIT) gap *= g[k];
            acc = fmaf(gap, gap, acc);
        }
        return acc <= lim;
    }
};

// Calls leaf(beg, end) for the sorted-source ranges of the leaves whose box
// is within reach of the ball D < rho2 around t (a superset of the sources
// inside it), in ascending order.  Records are read as 16-byte vectors (the
// stride is a multiple of four floats on 256-byte aligned storage) and
// tested in FP32 (BoxTest32).
template <int D, bool UNIT, class L>
PCMS_HD PCMS_INLINE void bvh_leaves(const GridParams &gp, const BvhView &bv, const double (&t)[D],
                                    double rho2, L &&leaf)
{
    constexpr int S = bvh_stride(D);
    const BoxTest32<D, UNIT> within(gp, t, rho2);
    int r = 0;
    while (r >= 0) {
#ifdef PCMS_HOST_EMULATION
        ++pcms_emu_nodes;
#endif
        float rec[S];
        const float4 *q = reinterpret_cast<const float4 *>(bv.nodes + (size_t)r * S);
#pragma unroll
        for (int j = 0; j < S / 4; ++j) {
            const float4 v = q[j];
            rec[4 * j] = v.x;
            rec[4 * j + 1] = v.y;
            rec[4 * j + 2] = v.z;
            rec[4 * j + 3] = v.w;
        }
        const bool hit = within(rec);
        const int c0 = bvh_int(rec, 2 * D), rope = bvh_int(rec, 2 * D + 1);
        if (c0 < 0) {
            if (hit) leaf(bvh_int(rec, 2 * D + 2), bvh_int(rec, 2 * D + 3));
            r = rope;
        } else {
            r = hit ? c0 : rope;
        }
    }
}

// Radius of a ball expected to hold k sources: the distance from t to the
// box of the smallest subtree on the way to t (descending toward the child
// whose box is nearer) that still holds at least 4k sources, plus the radius
// holding k sources at that subtree's density (its count over its box).
template <int D, bool UNIT>
PCMS_HD PCMS_INLINE double bvh_radius_guess(const GridParams &gp, const BvhView &bv,
                                            const double (&t)[D], int k)
{
    constexpr int S = bvh_stride(D);
    const float *nd = bv.nodes;
    for (int c0 = bvh_int(nd, 2 * D); c0 >= 0; c0 = bvh_int(nd, 2 * D)) {
        const float *n0 = bv.nodes + (size_t)c0 * S;
        // the second child: the first child's rope
        const float *n1 = bv.nodes + (size_t)bvh_int(n0, 2 * D + 1) * S;
        const float *nc =
            box_dist2<D, UNIT>(gp, t, n1, n1 + D) < box_dist2<D, UNIT>(gp, t, n0, n0 + D) ? n1 : n0;
        if (bvh_int(nc, 2 * D + 3) - bvh_int(nc, 2 * D + 2) < 4 * k) break;
        nd = nc;
    }
    const int count = bvh_int(nd, 2 * D + 3) - bvh_int(nd, 2 * D + 2);
    double vol = 1.0, gap2 = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const double lo = nd[j], hi = nd[D + j];
        vol *= fmax(hi - lo, 1e-300) * gp.g[j];
        const double gap = fmax(fmax(lo - t[j], t[j] - hi), 0.0) * gp.g[j];
        gap2 += gap * gap;
    }
    const double vball = D == 1 ? 2.0 : D == 2 ? M_PI : D == 3 ? 4.18879020478639098
                       : D == 4 ? 4.93480220054467931 : 5.26378901489003940;
    return sqrt(gap2) + pow((double)k * vol / ((double)max(count, 1) * vball), 1.0 / D);
}

}  // namespace pcms
