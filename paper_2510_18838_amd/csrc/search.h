// Per-target neighbour search on the uniform grid, G lanes per target.
//
// Selection follows the PCMS paper, Section 3.2.1: the source set of target
// t is { s_j : phi(s_j, t) > 0 }, i.e. the sources strictly inside the
// support radius.  The distance is the metric
//     D = fma(u_{d-1}, u_{d-1}, ... fma(u_1, u_1, u_0 * u_0)),
//     u_k = (t_k - s_k) * g_k,
// evaluated in FP64 in this exact order, so the predicate D < r^2 is bit
// reproducible.  The radius is fixed, grown by doubling r^2 until a minimum
// count is met (Section 3.2.1), or set to the k-th smallest D.  Above k_cap
// sources the k_cap smallest by (D, source index) are kept.
//
// Stencil walk: buckets are row-major with dimension 0 fastest, so for every
// row (c_1..c_{d-1}) the buckets c_0 in [a, b] form one contiguous range of
// sorted sources.  Rows whose slab is farther than the radius are skipped and
// each row's c_0 range is narrowed to the chord of the ball in that slab.
// The G lanes of a target walk the same rows (uniform control flow) and take
// the candidates of a row in an interleaved order, so their loads are
// contiguous; candidates reach the per-step callback in ascending sorted
// order, which the ordered ballot compaction of the lists preserves.
#pragma once

#include "bvh.h"
#include "device_common.h"

namespace pcms {

// Candidates per walk step whose loads are issued together: FP64 records
// (two 16-byte loads each) and FP32 records (one).
#ifndef PCMS_WALK_BATCH64
#define PCMS_WALK_BATCH64 4
#endif
#ifndef PCMS_WALK_BATCH32
#define PCMS_WALK_BATCH32 4
#endif
constexpr int kBatch64 = PCMS_WALK_BATCH64, kBatch32 = PCMS_WALK_BATCH32;

template <int D, bool UNIT>
PCMS_HD PCMS_INLINE double metric_d2(const double (&t)[D], const double *__restrict__ s,
                                     const GridParams &p)
{
    double u = UNIT ? (t[0] - s[0]) : (t[0] - s[0]) * p.g[0];
    double acc = u * u;
#pragma unroll
    for (int k = 1; k < D; ++k) {
        u = UNIT ? (t[k] - s[k]) : (t[k] - s[k]) * p.g[k];
        acc = __builtin_fma(u, u, acc);
    }
    return acc;
}

// Fraction of the unit d-ball's volume beyond the hyperplane at distance x
// (0 <= x <= 1) from its centre: the integral of (1 - s^2)^((d-1)/2) over
// [x, 1] over its integral over [-1, 1] (d = 1, 2, 3).
template <int D>
PCMS_HD PCMS_INLINE double ball_beyond(double x)
{
    static_assert(D >= 1 && D <= 3, "closed forms for 1-3 dimensions");
    auto P = [](double s) {
        if constexpr (D == 1) return s;
        else if constexpr (D == 2) return 0.5 * (s * sqrt(fmax(1.0 - s * s, 0.0)) + asin(s));
        else return s - s * s * s / 3.0;
    };
    x = fmin(fmax(x, 0.0), 1.0);
    return (P(1.0) - P(x)) / (P(1.0) - P(-1.0));
}

// Rows of a stencil walk: for radius rho around t, yields the rows (bucket
// coordinates c_1..c_{d-1}) whose slab is within reach, with each row's
// linear id and the c_0 range of the ball's chord in that slab.
template <int D, bool UNIT>
struct RowIter {
    const GridParams &gp;
    const double (&t)[D];
    double rho2;
    int a[D], b[D], c[D];
    bool done;

    PCMS_HD PCMS_INLINE RowIter(const GridParams &gp_, const double (&t_)[D], double rho2_)
        : gp(gp_), t(t_), rho2(rho2_), done(false)
    {
        const double rho = sqrt(rho2);
#pragma unroll
        for (int k = 1; k < D; ++k) {
            double half = (UNIT ? rho : rho / gp.g[k]) * (1.0 + 1e-9) + fabs(t[k]) * 1e-15 + 1e-300;
            a[k] = bucket_of(gp, k, t[k] - half);
            b[k] = bucket_of(gp, k, t[k] + half);
            c[k] = a[k];
        }
    }

    // Next row within reach; false when the stencil is exhausted.
    PCMS_HD PCMS_INLINE bool next(int &row, int &a0, int &b0)
    {
        while (!done) {
            // squared metric distance from t to this row's slab (boxes widened
            // slightly so rounding in the bucket assignment cannot hide a source)
            double m2 = 0.0;
            row = 0;
#pragma unroll
            for (int k = 1; k < D; ++k) {
                double blo = gp.lo[k] + (double)c[k] * gp.w[k];
                double bhi = blo + gp.w[k];
                double pad = 1e-7 * gp.w[k];
                // the first and last buckets also hold clamped coordinates
                if (c[k] == 0) blo = -INFINITY;
                if (c[k] == gp.n[k] - 1) bhi = INFINITY;
                double dlt = fmax(fmax(blo - pad - t[k], t[k] - bhi - pad), 0.0);
                if (!UNIT) dlt *= gp.g[k];
                m2 = __builtin_fma(dlt, dlt, m2);
                row += c[k] * gp.stride[k];
            }
            const bool reach = m2 <= rho2 * (1.0 + 1e-9);
            if (reach) {
                double rem2 = fmax(rho2 - m2 * (1.0 - 1e-9), 0.0);
                double half0 = (UNIT ? sqrt(rem2) : sqrt(rem2) / gp.g[0]) * (1.0 + 1e-9) +
                               fabs(t[0]) * 1e-15 + 1e-300;
                a0 = bucket_of(gp, 0, t[0] - half0);
                b0 = bucket_of(gp, 0, t[0] + half0);
            }
            // odometer over c_1..c_{d-1}, unrolled so c stays in registers
            bool carry = true;
#pragma unroll
            for (int k = 1; k < D; ++k) {
                if (carry) {
                    if (c[k] < b[k]) {
                        c[k]++;
                        carry = false;
                    } else {
                        c[k] = a[k];
                    }
                }
            }
            if (carry) done = true;
            if (reach) return true;
        }
        return false;
    }
};

// Candidate measures of the walks.  Exact64 loads a source's FP64 record
// and returns the D of the exact predicate.
template <int D, bool UNIT>
struct Exact64 {
    using E = double;
    const GridParams &gp;
    const double *__restrict__ spts;
    const double (&t)[D];
    PCMS_HD PCMS_INLINE void load(int p, double (&s)[D]) const { load_src<D>(spts, p, s); }
    PCMS_HD PCMS_INLINE double d2(const double (&s)[D]) const { return metric_d2<D, UNIT>(t, s, gp); }
};

// Image32 loads a source's FP32 record s32_k = fl32(s_k - lo_k) and returns
// the FP32 image of D: with the target split as t_k - lo_k = th_k + tl_k (two
// floats),
//     v_k = (th_k - s32_k) + tl_k,   u_k = v_k * fl32(g_k),   D32 = sum u_k^2
// (the sum as an fma chain).  It differs from the FP64 D by at most
//     m = alpha + beta * D32.
// Derivation: each u_k is within A_k + B |u_k| of its FP64 counterpart, where
// A_k = g_k |th_k| a (a >= 2^-24: rounding of the source image, plus the
// target split) and B >= 4 * 2^-24 + 2^-24 (the FP32 roundings of u_k and of
// g_k, and the source image through |s32_k| <= |th_k| + |v_k|).  Summing
// |u32_k^2 - u64_k^2| <= (A_k + B |u_k|)(A_k + (2 + B) |u_k|) over k, with
// sum_k A_k |u_k| <= |A| sqrt(D) and sqrt(D) <= (D / c + c) / 2 for any c > 0,
// and adding the d roundings of the FP32 sum, gives alpha and beta (times a
// safety factor of 1.5).  c is chosen near the thresholds of the walk, where
// the bound is tightest.  Coordinates beyond the FP32 range give a non-finite
// m, which the callers treat as "unknown".
template <int D, bool UNIT>
struct Image32 {
    using E = float;
    const float *__restrict__ s32;
    float th[D], tl[D], g[D];
    double alpha, beta;

    PCMS_HD PCMS_INLINE Image32(const GridParams &gp, const float *s32_, const double (&t)[D],
                                double c)
        : s32(s32_)
    {
        constexpr double kA = 6.0e-8, kB = 3.1e-7, kR = 6.0e-8, kSafe = 1.5;
        double a2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double x = t[k] - gp.lo[k];
            th[k] = (float)x;
            tl[k] = (float)(x - (double)th[k]);
            g[k] = UNIT ? 1.0f : (float)gp.g[k];
            const double ak = (UNIT ? 1.0 : gp.g[k]) * fabs((double)th[k]) * kA;
            a2 += ak * ak;
        }
        const double A = sqrt(a2);
        c = fmin(fmax(c, 1e-150), 1e150);
        alpha = kSafe * (A * A + (1.0 + kB) * A * c) + 1e-36;
        beta = kSafe * ((1.0 + kB) * A / c + 2.0 * kB + kB * kB + D * kR) * (1.0 + 1e-6);
    }
    PCMS_HD PCMS_INLINE void load(int p, float (&s)[D]) const { load_src32<D>(s32, p, s); }
    PCMS_HD PCMS_INLINE float d2(const float (&s)[D]) const
    {
        float v = (th[0] - s[0]) + tl[0];
        float u = UNIT ? v : v * g[0];
        float acc = u * u;
#pragma unroll
        for (int k = 1; k < D; ++k) {
            v = (th[k] - s[k]) + tl[k];
            u = UNIT ? v : v * g[k];
            acc = __builtin_fmaf(u, u, acc);
        }
        return acc;
    }
    // bound on |D - D32|; not finite (or NaN) when D32 cannot be trusted
    PCMS_HD PCMS_INLINE double bound(float d32) const { return alpha + beta * (double)d32; }
};

// Classification of D by equal-width bins: -1 below lo, j for D in the j-th
// of nb bins of [lo, hi), nb at or above hi (nb = 0, hi = lo: inside or not).
// Monotone non-decreasing in D.
struct Bins {
    double lo, hi, ibw;
    int nb;
    PCMS_HD PCMS_INLINE int operator()(double d2) const
    {
        return d2 < lo ? -1 : d2 < hi ? min((int)((d2 - lo) * ibw), nb - 1) : nb;
    }
};

// The same classification from an FP32 image: y = (D32 - lo) * ibw in FP32
// is within mb = a + b * D32 bin widths of (D - lo) * ibw (the image's bound
// plus the three FP32 roundings of y, plus 1e-9 for the FP64 rounding of the
// exact classification's own edges), so when y lies farther than mb from
// every edge its bin is the bin of D.  y is clamped to [-0.5, nb + 0.5]
// first: beyond the outer edges only the side matters.
struct Bins32 {
    float lo, ibw, top, a, b;

    template <int D, bool UNIT>
    PCMS_HD PCMS_INLINE Bins32(const Bins &k, const Image32<D, UNIT> &im)
    {
        constexpr double kU = 5.97e-8;   // 2^-24, rounded up
        lo = (float)k.lo;
        ibw = (float)k.ibw;
        top = (float)k.nb + 0.5f;
        a = (float)((k.ibw * (im.alpha + 4.04 * kU * fabs(k.lo)) + 1e-9) * 1.01);
        b = (float)(k.ibw * (im.beta + 3.03 * kU) * 1.01);
    }
    // the bin of D when `sure`; NaN or overflowed images are never sure
    PCMS_HD PCMS_INLINE int operator()(float d32, bool &sure) const
    {
        const float y = fminf(fmaxf((d32 - lo) * ibw, -0.5f), top);
        const float fl = floorf(y), fr = y - fl;
        const float mb = __builtin_fmaf(b, d32, a);
        sure = (fr > mb) & (fr + mb < 1.0f);
        return (int)fl;
    }
};

// Calls f(p, x, valid) for the sorted sources p of [beg, end), x being the
// measure's value (D, or its FP32 image), kBatch * G candidates per step (the
// loads of a step are issued together); every lane of the group calls f the
// same number of times, with valid = false on the padding slots past the end.
template <int D, int G, int kBatch, class Meas, class F>
PCMS_HD PCMS_INLINE void walk_range(const Meas &meas, int beg, int end, int q, F &&f)
{
    for (int p0 = beg; p0 < end; p0 += kBatch * G) {
        // slot j of lane q is candidate p0 + j*G + q: the group's loads of
        // one slot are contiguous
        typename Meas::E sb[kBatch][D];
        int pp[kBatch];
        bool ok[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            pp[j] = p0 + j * G + q;
            ok[j] = pp[j] < end;
            meas.load(ok[j] ? pp[j] : beg, sb[j]);
        }
#pragma unroll
        for (int j = 0; j < kBatch; ++j) f(pp[j], meas.d2(sb[j]), ok[j]);
    }
}

// walk_range over every sorted source in the buckets that can hold a source
// with D < rho2 (a superset of the ball).  rho2 may be +inf.  The next row's
// bucket offsets are loaded while the current row is processed.
template <int D, bool UNIT, int G, int kBatch, class Meas, class F>
PCMS_HD PCMS_INLINE void walk(const GridParams &gp, const int *__restrict__ cs, const Meas &meas,
                              const double (&t)[D], double rho2, int q, F &&f)
{
#ifdef PCMS_HOST_EMULATION
    if (q == 0) ++pcms_emu_walks;
#endif
    RowIter<D, UNIT> it(gp, t, rho2);
    int row, a0, b0;
    bool have = it.next(row, a0, b0);
    int beg = 0, end = 0;
    if (have) {
        beg = cs[row + a0];
        end = cs[row + b0 + 1];
    }
    while (have) {
        int nbeg = 0, nend = 0;
        const bool nhave = it.next(row, a0, b0);
        if (nhave) {
            nbeg = cs[row + a0];
            nend = cs[row + b0 + 1];
        }
#ifdef PCMS_HOST_EMULATION
        if (q == 0) {
            ++pcms_emu_rows;
            pcms_emu_cands += end - beg;
        }
#endif
        walk_range<D, G, kBatch>(meas, beg, end, q, f);
        beg = nbeg;
        end = nend;
        have = nhave;
    }
}

// Search state of one target, shared by its G lanes.  The target's `words`
// LDS words L[0..words) hold the kept list (k_cap entries) and, during the
// radius search, a buffer of words / 2 doubles (double j in words 2j, 2j+1).
// The walk over the sources that can lie inside a ball: the grid's row walk,
// or with BVH the leaves of the tree within reach (bvh.h).
template <int D, bool UNIT, int G, bool BVH, int kBatch, class Meas, class F>
PCMS_HD PCMS_INLINE void walk_any(const GridParams &gp, const int *__restrict__ cs,
                                  const BvhView &bv, const Meas &meas, const double (&t)[D],
                                  double rho2, int q, F &&f)
{
    if constexpr (BVH) {
#ifdef PCMS_HOST_EMULATION
        if (q == 0) ++pcms_emu_walks;
#endif
        bvh_leaves<D, UNIT>(gp, bv, t, rho2, [&](int beg, int end) {
#ifdef PCMS_HOST_EMULATION
            if (q == 0) {
                ++pcms_emu_rows;
                pcms_emu_cands += end - beg;
            }
#endif
            walk_range<D, G, kBatch>(meas, beg, end, q, f);
        });
    } else {
        walk<D, UNIT, G, kBatch>(gp, cs, meas, t, rho2, q, f);
    }
}

template <int D, bool UNIT, int G, bool BVH = false>
struct Search {
    const GridParams &gp;
    const int *__restrict__ cs;
    const double *__restrict__ spts;
    const float *__restrict__ spts32;   // FP32 records (used by the F32 walks)
    const int *__restrict__ perm;
    double t[D];
    int *L;     // this target's LDS words
    int k_cap;
    int words;  // >= max(k_cap, 2)
    Grp<G> g;
    BvhView bv; // the tree (BVH only)

    PCMS_HD PCMS_INLINE int &at(int e)
    {
#ifdef PCMS_HOST_EMULATION
        if (e < 0 || e >= words) pcms_emu_lds_fault(e, words);
#endif
        return L[e];
    }
    PCMS_HD PCMS_INLINE void dstore(int j, double v)
    {
        unsigned long long bits = __builtin_bit_cast(unsigned long long, v);
        at(2 * j) = (int)(unsigned)(bits & 0xffffffffull);
        at(2 * j + 1) = (int)(unsigned)(bits >> 32);
    }
    PCMS_HD PCMS_INLINE double dload(int j)
    {
        unsigned long long lo = (unsigned)at(2 * j);
        unsigned long long hi = (unsigned)at(2 * j + 1);
        return __builtin_bit_cast(double, (hi << 32) | lo);
    }
    template <class F>
    PCMS_HD PCMS_INLINE void each(double rho2, F &&f)
    {
        walk_any<D, UNIT, G, BVH, kBatch64>(gp, cs, bv, Exact64<D, UNIT>{gp, spts, t}, t, rho2, g.q,
                                            f);
    }

    // Calls f(p, bins(D), valid) for the candidates of the walk over rho2.
    // Without F32 the class comes from the FP64 D.  With F32 the walk reads
    // the FP32 records (kBatch32 per step) and a candidate takes the class of
    // its image when that is certain, else loads its FP64 record; either way
    // f sees the same classes.  c: the distance scale of the thresholds (any
    // positive value is correct; the bound is tightest near it).
    template <bool F32, class F>
    PCMS_HD PCMS_INLINE void each_key(double rho2, double c, const Bins &bins, F &&f)
    {
        if (!F32) {
            each(rho2, [&](int p, double d2, bool ok) { f(p, bins(d2), ok); });
            return;
        }
        const Image32<D, UNIT> im(gp, spts32, t, c);
        const Bins32 b32(bins, im);
        walk_any<D, UNIT, G, BVH, kBatch32>(gp, cs, bv, im, t, rho2, g.q, [&](int p, float d32, bool ok) {
            bool sure;
            int kk = b32(d32, sure);
            if (ok && !sure) {
#ifdef PCMS_HOST_EMULATION
                ++pcms_emu_exact;
#endif
                kk = bins(d2_of(p));
            }
            f(p, kk, ok);
        });
    }

    // Squared metric distance from t to the farthest corner of the bucket
    // box; every source lies closer, so a larger radius covers all sources.
    PCMS_HD double far2() const
    {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double lo = gp.lo[k], hi = gp.lo[k] + gp.n[k] * gp.w[k];
            double dd = fmax(fabs(t[k] - lo), fabs(hi - t[k])) * gp.g[k];
            acc += dd * dd;
        }
        return acc * (1.0 + 1e-6) + 1e-300;
    }

    // Collects every source with D < r2 into the list (up to k_cap, in walk
    // order); returns the count (the same on every lane of the group).
    template <bool F32 = false>
    PCMS_HD int collect(double r2)
    {
        int n = 0;
        each_key<F32>(r2, sqrt(r2), Bins{r2, r2, 1.0 / r2, 0}, [&](int p, int kk, bool ok) {
            // bitwise '&': the key is needed whatever ok is, so the compiler
            // keeps the batch's loads together instead of sinking one into a
            // branch
            const bool acc = ok & (kk < 0);
            const unsigned m = g.ballot(acc);
            if (acc) {
                const int pos = n + g.below(m);
                if (pos < k_cap) at(pos) = p;
            }
            n += __builtin_popcount(m);
        });
        g.sync();
        return n;
    }

    // Radius of a ball expected to hold k sources, from the bucket counts
    // around t (no point loads): the 3^d block of bucket widths around t's
    // bucket, which in dimension 0 spans sub + sub/2 slices to each side.
    PCMS_HD double knn_radius_guess(int k) const
    {
        if constexpr (BVH) return box_corrected(bvh_radius_guess<D, UNIT>(gp, bv, t, k));
        int a[D], b[D], c[D];
        double vol = 1.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const int h = j == 0 ? gp.sub + gp.sub / 2 : 1;
            int cj = bucket_of(gp, j, t[j]);
            a[j] = max(cj - h, 0);
            b[j] = min(cj + h, gp.n[j] - 1);
            c[j] = a[j];
            vol *= (double)(b[j] - a[j] + 1) * gp.w[j] * gp.g[j];
        }
        long long count = 0;
        for (;;) {
            int row = 0;
#pragma unroll
            for (int j = 1; j < D; ++j) row += c[j] * gp.stride[j];
            count += cs[row + b[0] + 1] - cs[row + a[0]];
            bool carry = true;
#pragma unroll
            for (int j = 1; j < D; ++j) {
                if (carry) {
                    if (c[j] < b[j]) {
                        c[j]++;
                        carry = false;
                    } else {
                        c[j] = a[j];
                    }
                }
            }
            if (carry) break;
        }
        // unit-ball volume pi^(D/2) / Gamma(D/2 + 1)
        const double vball = D == 1 ? 2.0 : D == 2 ? M_PI : D == 3 ? 4.18879020478639098
                           : D == 4 ? 4.93480220054467931 : 5.26378901489003940;
        if (count <= 0) {
            double half = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) half = fmax(half, 1.5 * gp.w[j] * gp.g[j]);
            return 2.0 * half;
        }
        return box_corrected(pow((double)k * vol / ((double)count * vball), 1.0 / D));
    }

    // Every source lies in the bounding box, so the part of a ball beyond a
    // face holds none: the radius g0 expected to hold k sources at the local
    // density is grown until the part inside the box is expected to hold k
    // (faces taken one at a time, two fixed-point steps; a face behind the
    // target cuts nothing here).  Each dimension keeps at least half of the
    // ball, as at a face: a box thinner than the ball (flat or coincident
    // sources) holds a lower-dimensional cloud, which this model does not
    // describe, so the radius grows at most 2x.  In 1-3 dimensions (where
    // knn_select narrows the grid's window to match).
    PCMS_HD double box_corrected(double g0) const
    {
        if constexpr (D > 3) {
            return g0;
        } else {
            double gr = g0;
            for (int it = 0; it < 2; ++it) {
                double f = 1.0;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const double s = (UNIT ? 1.0 : gp.g[j]) / gr;
                    f *= fmax(1.0 - ball_beyond<D>((t[j] - gp.lo[j]) * s) -
                                  ball_beyond<D>((gp.hi[j] - t[j]) * s),
                              0.5);
                }
                gr = g0 * pow(f, -1.0 / D);
            }
            return gr < INFINITY ? gr : g0;
        }
    }

    // Appends the values D in [lo, hi) to the buffer (ordered compaction,
    // at most cb kept); returns (group-uniform) the counts below lo and in
    // [lo, hi).
    PCMS_HD void buffer_bracket(double lo, double hi, int cb, int &c_lo, int &n_in)
    {
        int below = 0, n = 0;
        each(hi, [&](int, double d2, bool ok) {
            below += ok & (d2 < lo);
            const bool in = ok & (d2 >= lo) & (d2 < hi);
            const unsigned m = g.ballot(in);
            if (in) {
                const int pos = n + g.below(m);
                if (pos < cb) dstore(pos, d2);
            }
            n += __builtin_popcount(m);
        });
        g.sync();
        c_lo = g.sum(below);
        n_in = n;
    }

    // r-th smallest (1-based) of the n doubles in the buffer; the lanes rank
    // interleaved entries and the group takes the minimum found.
    PCMS_HD double buffer_rank(int n, int r)
    {
        double ans = INFINITY;
        for (int a0 = 0; a0 < n; a0 += G) {
            const int a = a0 + g.q;
            if (a < n) {
                const double v = dload(a);
                int less = 0, le = 0;
                for (int b = 0; b < n; ++b) {
                    const double x = dload(b);
                    less += x < v;
                    le += x <= v;
                }
                if (less < r && r <= le) ans = v;
            }
        }
        return g.min(ans);
    }

    // D of sorted source p
    PCMS_HD PCMS_INLINE double d2_of(int p) const
    {
        double sb[D];
        load_src<D>(spts, p, sb);
        return metric_d2<D, UNIT>(t, sb, gp);
    }

    // kNN selection in two walks, for k <= k_cap + 1: select_window over the
    // window [(a g)^2, (b g)^2), g the estimate of the radius.  With the
    // grid's estimate corrected for the bounding box (1-3 dimensions) the
    // window is [0.8 g, 1.18 g); else, and for the LBVH's noisier estimate,
    // [0.78 g, 1.3 g).  On success r2 is the k-th smallest D, the list holds
    // every source with D < r2 and n_found their count (< k).  When the k-th
    // lies outside the window, one more window beside it is tried,
    // [b g, 1.5 b g) or [0.6 a g, a g): two walks instead of the general
    // path's bracketing.  False leaves the general path to the caller.
    template <bool F32 = false>
    PCMS_HD bool knn_select(int k, double &r2, int &n_found)
    {
        constexpr bool kTight = !BVH && D <= 3;
        constexpr double a = kTight ? 0.8 : 0.78, b = kTight ? 1.18 : 1.3;
        const double gr = knn_radius_guess(k);
        double lo = (a * gr) * (a * gr), hi = (b * gr) * (b * gr);
        // one call site, so that the selection is inlined once
        for (int attempt = 0; attempt < 2; ++attempt) {
            int side = 0;
            if (select_window<F32, false>(k, lo, hi, r2, n_found, &side)) return true;
            if (side > 0) {
                lo = hi;
                hi = (1.5 * b * gr) * (1.5 * b * gr);
            } else if (side < 0) {
                hi = lo;
                lo = (0.6 * a * gr) * (0.6 * a * gr);
            } else {
                return false;
            }
        }
        return false;
    }

    // The k-th smallest D in two walks, given a window [lo, hi) expected to
    // hold it.  The first walk, over the ball D < hi, counts the sources
    // below lo and histograms those in [lo, hi) into nb bins of equal width
    // in D (the target's first nb words serve as the bins).  The second walk
    // lists, in walk order, every source of a lower bin (or below lo) and
    // keeps the indices of the bin holding the k-th at the end of the words;
    // the k-th is ranked among them (their D recomputed) and those below it
    // complete the list.  Both walks classify a source with the same
    // expression of its D, so their counts agree exactly (with F32 the walks
    // read the FP32 records and still obtain that exact classification).  On
    // success v is the k-th smallest D and the list holds every source with
    // D < v, n their count (< k); with TIES the list is then completed to k
    // entries with sources at D = v, smallest source index first, and n = k.
    // Returns false when the k-th lies outside [lo, hi) or its bin does not
    // fit the words; then *side (if given) is -1 if the k-th lies below lo,
    // +1 if at or above hi, 0 otherwise.
    template <bool F32, bool TIES>
    PCMS_HD bool select_window(int k, double lo, double hi, double &v, int &n_out,
                               int *side = nullptr)
    {
        const int nb = words < 64 ? words : 64;
        const double bw = (hi - lo) / nb, ibw = 1.0 / bw;
        // -1 below lo, the bin in [lo, hi), nb at or above hi
        const Bins key{lo, hi, ibw, nb};
        for (int j = g.q; j < nb; j += G) at(j) = 0;
        g.sync();
        int below = 0;
        each_key<F32>(hi, sqrt(hi), key, [&](int, int kk, bool ok) {
            below += ok & (kk < 0);
            if (ok & (kk >= 0) & (kk < nb)) lds_add(&at(kk), 1);
        });
        g.sync();
        const int c_lo = g.sum(below);
        int b = -1, c_b = 0, n_b = 0;
        if (c_lo < k) {
            int cum = c_lo;
            for (int j = 0; j < nb; ++j) {
                const int cj = at(j);
                if (b < 0 && cum + cj >= k) {
                    b = j;
                    c_b = cum;
                    n_b = cj;
                }
                cum += cj;
            }
        }
        g.sync();   // every lane has read the bins before the list overwrites them
        if (b < 0 || c_b + n_b > words) {
            if (side) *side = b >= 0 ? 0 : c_lo >= k ? -1 : 1;
            return false;
        }
        // bin entry j sits in word words - n_b + j
        const int base = words - n_b;
        const double rho2 = b == nb - 1 ? hi : fmin(hi, (lo + (double)(b + 1) * bw) * (1.0 + 1e-12));
        int n = 0, m = 0;
        each_key<F32>(rho2, sqrt(rho2), key, [&](int p, int kk, bool ok) {
            const bool in = ok & (kk < b);
            const bool bb = ok & (kk == b);
            const unsigned mi = g.ballot(in), mb = g.ballot(bb);
            if (in) {
                const int pos = n + g.below(mi);
                if (pos < c_b) at(pos) = p;
            }
            if (bb) {
                const int j = m + g.below(mb);
                if (j < n_b) at(base + j) = p;
            }
            n += __builtin_popcount(mi);
            m += __builtin_popcount(mb);
        });
        g.sync();
        if (n != c_b || m != n_b) return false;   // cannot happen: same sources, same key
        // r-th smallest (1-based) of the bin, ranked by the lanes in turn
        const int r = k - c_b;
        double ans = INFINITY;
        for (int a0 = 0; a0 < n_b; a0 += G) {
            const int a = a0 + g.q;
            if (a < n_b) {
                const double x0 = d2_of(at(base + a));
                int less = 0, le = 0;
                for (int j = 0; j < n_b; ++j) {
                    const double x = d2_of(at(base + j));
                    less += x < x0;
                    le += x <= x0;
                }
                if (less < r && r <= le) ans = x0;
            }
        }
        v = g.min(ans);
        if (TIES) {
            // the k - (c_b + #(bin entries below v)) sources at D = v of
            // smallest source index join the list: each round marks the next
            // one (its word holds ~p until it is appended)
            int below_v = 0;
            for (int j0 = 0; j0 < n_b; j0 += G) {
                const int j = j0 + g.q;
                below_v += j < n_b && d2_of(at(base + j)) < v;
            }
            int prev = -1;
            for (int need = k - c_b - g.sum(below_v); need > 0; --need) {
                int best = 0x7fffffff, bj = -1;
                for (int j0 = 0; j0 < n_b; j0 += G) {
                    const int j = j0 + g.q;
                    if (j < n_b) {
                        const int x = at(base + j);
                        if (x >= 0) {
                            const int idx = perm[x];
                            if (idx > prev && idx < best && d2_of(x) == v) {
                                best = idx;
                                bj = j;
                            }
                        }
                    }
                }
                const int gb = g.min(best);
                g.sync();
                if (best == gb && bj >= 0) at(base + bj) = ~at(base + bj);
                g.sync();
                prev = gb;
            }
        }
        // append the bin's sources below v (and the marked ones) in walk
        // order; entry j is read before position c_b + j (<= base + j) can
        // be written
        int cnt = c_b;
        for (int j0 = 0; j0 < n_b; j0 += G) {
            const int j = j0 + g.q;
            const int x = j < n_b ? at(base + j) : 0;
            const int p = x < 0 ? ~x : x;
            const bool take = j < n_b && (x < 0 || d2_of(p) < v);
            const unsigned mt = g.ballot(take);
            g.sync();
            if (take) at(cnt + g.below(mt)) = p;
            cnt += __builtin_popcount(mt);
        }
        g.sync();
        n_out = cnt;
        return true;
    }

    // Squared distance of the k-th nearest source.  One walk counts the
    // sources below lo = ((1 - h) g)^2 and buffers those in
    // [lo, hi = ((1 + h) g)^2), g the bucket-count estimate of the radius;
    // when the k-th falls in the buffered interval it is ranked there,
    // otherwise the general bracketing search continues from what the walk
    // established.
    PCMS_HD double knn_r2(int k)
    {
        const double gr = knn_radius_guess(k);
        const int cb = words / 2;
        // expected count in the window k ((1 + h)^D - (1 - h)^D) ~ 2 D h k,
        // sized to about 3/4 of the buffer
        const double h = fmin(0.15, fmax(0.02, 0.75 * (double)cb / (2.0 * D * (double)k)));
        const double lo = (1.0 - h) * (1.0 - h) * gr * gr, hi = (1.0 + h) * (1.0 + h) * gr * gr;
        int c_lo, n_in;
        buffer_bracket(lo, hi, cb, c_lo, n_in);
        if (c_lo < k && k <= c_lo + n_in && n_in <= cb) return buffer_rank(n_in, k - c_lo);
        if (c_lo >= k) return kth(k, 0.0, 0, lo, cb);
        if (c_lo + n_in < k) return kth(k, hi, c_lo + n_in, 4.0 * hi, cb);
        return kth(k, lo, c_lo, hi, cb);
    }

    // Exact k-th smallest D (1-based) over all sources, given a bracket:
    // #(D < lo) = c_lo < k, and hi a first guess for an upper bound (grown
    // when #(D < hi) < k).  Each round counts the sources of [lo, hi) into 8
    // sub-intervals with one walk; once the interval holding the k-th has at
    // most `sb` (<= words / 2) sources they are copied into the buffer and
    // ranked.
    PCMS_HD double kth(int k, double lo, int c_lo, double hi, int sb)
    {
        constexpr int NB = 8;
        const double farr = far2();
        for (int it = 0; it < 400; ++it) {
            double sp[NB];
            const bool from_zero = (lo == 0.0);
#pragma unroll
            for (int j = 0; j < NB - 1; ++j) {
                // from zero: equal expected counts, ((j + 1) / NB)^(2 / D) of
                // the interval; otherwise linear in D
                const double x = (double)(j + 1) / NB;
                const double f0 = D == 1 ? x * x : D == 2 ? x : D == 3 ? cbrt(x * x)
                                : D == 4 ? sqrt(x) : pow(x, 0.4);
                const double f = from_zero ? f0 : x;
                sp[j] = fmin(fmax(lo + (hi - lo) * f, lo), hi);
            }
            sp[NB - 1] = hi;
            int cnt[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) cnt[j] = 0;
            const double l0 = lo, h0 = hi;
            double vmin = h0;   // smallest D in [lo, hi) and its multiplicity
            int neq = 0;
            each(h0, [&](int, double d2, bool ok) {
                if (ok & (d2 >= l0) & (d2 < h0)) {
#pragma unroll
                    for (int j = 0; j < NB; ++j) cnt[j] += d2 < sp[j];
                    if (d2 < vmin) {
                        vmin = d2;
                        neq = 0;
                    }
                    neq += d2 == vmin;
                }
            });
#pragma unroll
            for (int j = 0; j < NB; ++j) cnt[j] = g.sum(cnt[j]);
            {
                const double gmin = g.min(vmin);
                neq = g.sum(vmin == gmin ? neq : 0);
                vmin = gmin;
            }
            if (c_lo + cnt[NB - 1] < k) {     // the k-th lies at or above hi
                // every source has D < farr, so the count reaches k there
                // (k <= n_src); nothing above it is left to search
                if (!(hi < farr)) return hi;
                c_lo += cnt[NB - 1];
                lo = hi;
                hi = fmin(fmax(hi * 16.0, farr * 1e-12), farr);
                continue;
            }
            // #(D < vmin) = c_lo: the k-th is vmin when its copies reach rank k
            if (c_lo + neq >= k) return vmin;
            int bsel = NB - 1;
#pragma unroll
            for (int j = NB - 1; j >= 0; --j)
                if (c_lo + cnt[j] >= k) bsel = j;
            int below = 0;
            double nlo = lo, nhi = hi;
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                if (j + 1 == bsel) {
                    below = cnt[j];
                    nlo = sp[j];
                }
                if (j == bsel) nhi = sp[j];
            }
            int nin = cnt[bsel] - below;
            lo = nlo;
            hi = nhi;
            c_lo += below;
            if (nin == cnt[NB - 1] && vmin >= lo) {
                // no split separated the values (many equal ones): step past
                // the smallest, whose copies all rank below k
                lo = nextafter(vmin, INFINITY);
                c_lo += neq;
                nin -= neq;
            }
            if (nin <= sb) {
                int cl, n;
                buffer_bracket(lo, hi, sb, cl, n);
                const double ans = buffer_rank(min(n, sb), k - c_lo);
                return ans < INFINITY ? ans : hi;
            }
            // a single representable value left in [lo, hi): it is the answer
            if (!(nextafter(lo, INFINITY) < hi)) return lo;
        }
        return hi;
    }

    // Keeps the k_cap smallest (D, source index) among D < r2 in the list
    // (called when more than k_cap sources are inside); returns the number of
    // list entries written.
    template <bool F32 = false>
    PCMS_HD int cap_collect(double r2)
    {
        // usually two walks: the k_cap-th lies in the window [0, r2)
        double vw;
        int nw;
        if (select_window<F32, true>(k_cap, 0.0, r2, vw, nw)) return nw;
        const double v = kth(k_cap, 0.0, 0, r2, words / 2);
        const double vnext = nextafter(v, INFINITY);
        int n = 0, c_eq = 0;
        each(vnext, [&](int p, double d2, bool ok) {
            const bool acc = ok & (d2 < v);
            const unsigned m = g.ballot(acc);
            if (acc) {
                const int pos = n + g.below(m);
                if (pos < k_cap) at(pos) = p;
            }
            n += __builtin_popcount(m);
            c_eq += ok & (d2 == v);
        });
        g.sync();
        c_eq = g.sum(c_eq);
        const int need = k_cap - n;
        if (need <= 0) return k_cap;
        int jthr = 0x7fffffff;
        if (need < c_eq) {        // ties at v: the smallest source indices win
            int prev = -1;
            for (int r = 0; r < need; ++r) {
                int best = 0x7fffffff;
                each(vnext, [&](int p, double d2, bool ok) {
                    if (ok & (d2 == v)) {
                        const int j = perm[p];
                        if (j > prev && j < best) best = j;
                    }
                });
                prev = g.min(best);
            }
            jthr = prev;
        }
        each(vnext, [&](int p, double d2, bool ok) {
            const bool acc = ok & (d2 == v) && perm[p] <= jthr;
            const unsigned m = g.ballot(acc);
            if (acc) {
                const int pos = n + g.below(m);
                if (pos < k_cap) at(pos) = p;
            }
            n += __builtin_popcount(m);
        });
        g.sync();
        return min(n, k_cap);
    }
};

}  // namespace pcms
