// Per-target work of the neighbour-list and field-transfer kernels, written
// as host+device functions of (arguments, target slot, the target's LDS
// words, lane group) so the CPU emulation build runs exactly this code.  The
// G lanes of a target split the walks' candidates and the neighbours of the
// fit passes; group sums combine their partial moments.
//
// Field transfer (PCMS paper, Section 3.2.1, Eq. 1): for target t with kept
// sources s_e, weights w_e = phi(q_e), q_e = sqrt(D_e) / r, and monomials
// p_e = p(xi_e) of total degree <= P in xi_e = (s_e - t) * g / r, the fitted
// value is fhat = e_0^T G^{-1} B with G = sum_e w_e p_e p_e^T + lambda I and
// B = sum_e w_e p_e f_e^T.  It is evaluated in shape-function form: one
// Cholesky factorisation of G, one solve y = G^{-1} e_0, then
// fhat_l = sum_e (w_e p_e . y) f_e,l for every field l, which shares the
// factorisation across all fields.
//
// Precision: FP64 assembles G in FP64.  MIXED forms xi_e and w_e in FP32 and
// accumulates G in FP32; the factorisation, the solve and the evaluation
// pass are FP64 (FP64 per-neighbour data).  MIXED_REFINE assembles its FP32
// moments from the sources' fixed-point records (one load each) and adds
// FP64 iterative refinement y += G32^{-1}(e_0 - G y) with the residual formed
// from FP64 per-neighbour data, which converges to the FP64 result (one step
// unless the target is ill-conditioned).  In the mixed modes with lambda = 0
// field values are centred on the first kept neighbour's value.
#pragma once

#include <type_traits>

#include "device_common.h"
#include "search.h"

namespace pcms {

constexpr int kFieldChunk = 8;
constexpr int kMaxRefine = 4;

template <int D, int P>
struct Basis {
    static constexpr int M = P == 0 ? 1 : P == 1 ? 1 + D : 1 + D + D * (D + 1) / 2;
    static constexpr int MM = M * (M + 1) / 2;
};

// Monomials of total degree <= P in graded-lex order:
// 1; x_0 .. x_{D-1}; x_a x_b for a <= b, lexicographic in (a, b).
template <int D, int P, typename T>
PCMS_HD PCMS_INLINE void monomials(const T (&xi)[D], T (&p)[Basis<D, P>::M])
{
    int m = 0;
    p[m++] = T(1);
    if (P >= 1) {
#pragma unroll
        for (int a = 0; a < D; ++a) p[m++] = xi[a];
    }
    if (P >= 2) {
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = a; b < D; ++b) p[m++] = xi[a] * xi[b];
    }
}

// Radial weights of q = r / r_c (Table 1, a = 2; Wendland C2 is the default),
// given q < 1 and o = 1 - q.
template <typename T>
PCMS_HD PCMS_INLINE T weight_in(int kind, T q, T o)
{
    switch (kind) {
    case PCMS_WEIGHT_C4: {
        T o2 = o * o;
        T o6 = o2 * o2 * o2;
        T poly = ((((T(5) * q + T(30)) * q + T(72)) * q + T(82)) * q + T(36)) * q + T(6);
        return poly * o6;
    }
    case PCMS_WEIGHT_GAUSSIAN: return exp(-(T(2) * q) * (T(2) * q));
    case PCMS_WEIGHT_CONST:
    case PCMS_WEIGHT_NO_OP: return T(1);
    case PCMS_WEIGHT_IMQ: return T(1) / sqrt(T(1) + (T(2) * q) * (T(2) * q));
    default: {
        T o2 = o * o;
        return o2 * o2 * (T(4) * q + T(1));
    }
    }
}

template <typename T>
PCMS_HD PCMS_INLINE T weight_of(int kind, T q)
{
    return q < T(1) ? weight_in<T>(kind, q, T(1) - q) : T(0);
}

// Packed upper-triangular index of (a, b), a <= b.
template <int M>
PCMS_HD PCMS_INLINE constexpr int tri(int a, int b)
{
    return a * M - a * (a - 1) / 2 + (b - a);
}

// Singularity floors of the Cholesky pivots, relative to max diag: 1e-13 for
// moments accumulated in FP64 (and for the FP32 factor of MIXED_REFINE, whose
// refinement judges convergence itself); 4e-6 (64 units of FP32 rounding) for
// FP32-accumulated moments factored without refinement, whose pivots below
// that carry no information (an exactly singular G gets pivots of FP32
// rounding size instead of zero).
constexpr double kPivotFloor = 1e-13;
constexpr double kPivotFloorF32 = 4e-6;

// In-place Cholesky of the packed SPD matrix A (upper triangle rows), in T,
// overwriting it with the factor R = L^T (A = R^T R).  Returns false when a
// pivot is not above tau_rel * max diag(A).
template <int M, typename T>
PCMS_HD PCMS_INLINE bool cholesky(T (&A)[M * (M + 1) / 2], T (&inv_diag)[M], double tau_rel)
{
    T maxd = T(0);
#pragma unroll
    for (int i = 0; i < M; ++i) maxd = fmax(maxd, A[tri<M>(i, i)]);
    const T tau = T(tau_rel) * maxd;
    bool ok = maxd > T(0);
#pragma unroll
    for (int j = 0; j < M; ++j) {
        T s = A[tri<M>(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) s = fma_t(-A[tri<M>(k, j)], A[tri<M>(k, j)], s);
        ok = ok && (s > tau);
        T d = sqrt(fmax(s, sizeof(T) == sizeof(double) ? T(1e-300) : T(1e-30)));
        T id = T(1) / d;
        A[tri<M>(j, j)] = d;
        inv_diag[j] = id;
#pragma unroll
        for (int i = j + 1; i < M; ++i) {
            T x = A[tri<M>(j, i)];
#pragma unroll
            for (int k = 0; k < j; ++k) x = fma_t(-A[tri<M>(k, j)], A[tri<M>(k, i)], x);
            A[tri<M>(j, i)] = x * id;
        }
    }
    return ok;
}

// Solves R^T R x = b in place with the packed factor R (entries of type T),
// in FP64 arithmetic.
template <int M, typename T>
PCMS_HD PCMS_INLINE void chol_solve(const T (&R)[M * (M + 1) / 2], const T (&inv_diag)[M],
                                    double (&x)[M])
{
#pragma unroll
    for (int i = 0; i < M; ++i) {
        double s = x[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s = __builtin_fma(-(double)R[tri<M>(k, i)], x[k], s);
        x[i] = s * (double)inv_diag[i];
    }
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
        double s = x[i];
#pragma unroll
        for (int k = i + 1; k < M; ++k) s = __builtin_fma(-(double)R[tri<M>(i, k)], x[k], s);
        x[i] = s * (double)inv_diag[i];
    }
}

// The same solve in T arithmetic throughout (the refinement corrections of
// MIXED_REFINE, which need only the relative accuracy of the FP32 factor).
template <int M, typename T>
PCMS_HD PCMS_INLINE void chol_solve_in(const T (&R)[M * (M + 1) / 2], const T (&inv_diag)[M],
                                       T (&x)[M])
{
#pragma unroll
    for (int i = 0; i < M; ++i) {
        T s = x[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s = fma_t(-R[tri<M>(k, i)], x[k], s);
        x[i] = s * inv_diag[i];
    }
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
        T s = x[i];
#pragma unroll
        for (int k = i + 1; k < M; ++k) s = fma_t(-R[tri<M>(i, k)], x[k], s);
        x[i] = s * inv_diag[i];
    }
}

struct KArgs {
    const GridParams *gp;
    const int *cs;
    const double *spts;
    const float *spts32;   // FP32 records of the sorted sources (mixed-precision walks)
    const uint32_t *sq;    // fixed-point records of the sorted sources (mixed-precision fits)
    const float *bvh_nodes;  // LBVH records (the BVH kernels)
    const int *perm;
    const double *tgt;
    const int *tperm;
    int n_tgt;
    int mode;
    int k;
    int n_min;
    int max_iter;
    double r;
    int k_cap;
    int words;             // LDS words of a target's list/buffer (>= max(k_cap, 2))
    int stride;            // LDS words between consecutive targets of a block (odd)
    int n_blocks;          // logical blocks (before XCD padding)
    // transfer only
    const double *svals;   // [n_src][nfs], sorted order, zero padded
    int nf;
    int nfs;               // padded_dim(nf): 16-byte aligned value records
    int weight;
    double lambda;
    double *out;           // [nf][n_tgt]
    double *stage;         // [n_tgt][nfs] by original target index, or NULL: the
                           // fields of a target are written as one record
                           // (whole 16-byte words) and transposed into out by a
                           // later kernel, instead of nf scattered 8-byte stores
    // operator emission only: [width][n_tgt] weights and source indices, counts
    double *op_w;
    int32_t *op_c;
    int32_t *op_n;
    // outputs
    int32_t *nbr;
    int32_t *n_kept;
    int32_t *n_found;
    double *r2;
    uint8_t *status;
    int32_t *summary;
};

// LDS words of a target: its kept list (at most k_cap entries; in kNN mode
// with k <= k_cap at most k - 1, since every kept D is below the k-th
// smallest), which also holds the histogram and buffers of the radius search,
// plus 8 for the bin of the k-th smallest D (kNN) or, where the cap is
// expected to bind (growing radii, kNN beyond the cap), of the k_cap-th.  A
// fixed radius keeps k_cap words: its rare capped targets take the general
// bracketing path.
PCMS_HD inline int target_words(int mode, int k, int k_cap)
{
    if (mode == PCMS_RADIUS_KNN && k + 8 < k_cap) return k + 8;
    if (mode == PCMS_RADIUS_FIXED) return k_cap < 2 ? 2 : k_cap;
    return k_cap + 8;
}

// Radius and kept list for one target; returns the status bits, the count
// inside the radius, the number of kept list entries and r^2 (all uniform
// across the group).  F32: the walks classify candidates from the FP32
// records (same lists).
template <int D, bool UNIT, int G, bool F32 = false, class S_>
PCMS_HD PCMS_INLINE int select_target(S_ &S, const KArgs &a, int &n_found,
                                      int &n_kept, double &r2)
{
    int st = PCMS_TGT_OK;
    if (a.mode == PCMS_RADIUS_FIXED) {
        r2 = a.r * a.r;
        n_found = S.template collect<F32>(r2);
    } else if (a.mode == PCMS_RADIUS_GROW) {
        r2 = a.r * a.r;
        n_found = S.template collect<F32>(r2);
        int it = 0;
        while (n_found < a.n_min && it < a.max_iter) {
            r2 = 2.0 * r2;
            ++it;
            n_found = S.template collect<F32>(r2);
        }
        if (n_found < a.n_min) st = PCMS_TGT_RADIUS_EXHAUSTED;
    } else {
        // n_found < k <= k_cap + 1 on the two-walk path, so no cap applies
        if (!(a.k <= a.k_cap + 1 && S.template knn_select<F32>(a.k, r2, n_found))) {
            r2 = S.knn_r2(a.k);
            n_found = S.collect(r2);
        }
    }
    n_kept = min(n_found, a.k_cap);
    if (n_found > a.k_cap) {
        st |= PCMS_TGT_CAPPED;
        n_kept = S.template cap_collect<F32>(r2);
    }
    return st;
}

template <int D>
PCMS_HD PCMS_INLINE void load_point(const double *__restrict__ x, int i, double (&t)[D])
{
#pragma unroll
    for (int k = 0; k < D; ++k) t[k] = x[(size_t)i * D + k];
}

// Neighbour list of the target at sorted slot i (original indices, ascending).
template <int D, bool UNIT, int G, bool BVH = false>
PCMS_HD PCMS_INLINE int nbr_target(const KArgs &a, const GridParams &gp, int i, int *L, Grp<G> g)
{
    const int ti = a.tperm[i];
    Search<D, UNIT, G, BVH> S{gp, a.cs, a.spts, a.spts32, a.perm, {}, L, a.k_cap, a.words, g,
                              {a.bvh_nodes}};
    load_point<D>(a.tgt, ti, S.t);
    int n_found, n;
    double r2;
    const int st = select_target<D, UNIT, G>(S, a, n_found, n, r2);
    for (int e = g.q; e < n; e += G) S.at(e) = a.perm[S.at(e)];
    g.sync();
    // source indices are distinct: each entry's rank is its output slot
    int32_t *row = a.nbr + (size_t)ti * a.k_cap;
    for (int e = g.q; e < n; e += G) {
        const int v = S.at(e);
        int rank = 0;
        for (int x = 0; x < n; ++x) rank += S.at(x) < v;
        row[rank] = v;
    }
    if (g.q == 0) {
        a.n_kept[ti] = n;
        if (a.n_found) a.n_found[ti] = n_found;
        if (a.r2) a.r2[ti] = r2;
        if (a.status) a.status[ti] = (uint8_t)st;
    }
    return st;
}

// Coordinates of the kept sources in the fit passes.  With Q false they come
// from the FP64 records and u = (t - s) g is the FP64 offset of the exact
// predicate; with Q true (the mixed precisions) from the fixed-point records
// (one load of 4 D bytes instead of two 16-byte ones), u = (tq - q) qs g with
// tq = (t - lo) / qs formed once per target, which is the offset of the
// source's fixed-point position lo + q qs, within qs / 2 of its own.
template <int D, bool UNIT, bool Q>
struct FitPts {
    using Rec = typename std::conditional<Q, uint32_t, double>::type;
    const double *__restrict__ spts;
    const uint32_t *__restrict__ sq;
    double t[D];    // the target, or its fixed-point image
    double sc[D];   // g, or qs g

    PCMS_HD PCMS_INLINE FitPts(const KArgs &a, const GridParams &gp, const double (&tt)[D])
        : spts(a.spts), sq(a.sq)
    {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            t[k] = Q ? (tt[k] - gp.lo[k]) * gp.iqs[k] : tt[k];
            sc[k] = Q ? (UNIT ? gp.qs[k] : gp.qs[k] * gp.g[k]) : gp.g[k];
        }
    }
    PCMS_HD PCMS_INLINE void load(int p, Rec (&r)[D]) const
    {
        if constexpr (Q)
            load_srcq<D>(sq, p, r);
        else
            load_src<D>(spts, p, r);
    }
    PCMS_HD PCMS_INLINE void offsets(const Rec (&r)[D], double (&u)[D]) const
    {
#pragma unroll
        for (int k = 0; k < D; ++k)
            u[k] = Q ? (t[k] - (double)r[k]) * sc[k] : (UNIT ? t[k] - r[k] : (t[k] - r[k]) * sc[k]);
    }
};

// Loads the records of kept neighbours e0 + j G (j < B) of this lane at once,
// with their sorted indices; slots past n repeat neighbour 0 and are flagged
// invalid.
template <int D, int G, int B, class S_, class FP>
PCMS_HD PCMS_INLINE void load_neighbours(S_ &S, const FP &fp, int e0, int n,
                                         typename FP::Rec (&sb)[B][D], bool (&ok)[B], int (&pe)[B])
{
#pragma unroll
    for (int j = 0; j < B; ++j) {
        const int e = e0 + j * G;
        ok[j] = e < n;
        pe[j] = S.at(ok[j] ? e : 0);
    }
#pragma unroll
    for (int j = 0; j < B; ++j) fp.load(pe[j], sb[j]);
}

// Per-neighbour local data from its offset u = (t - s) g: monomials p of
// xi = -u / h and the weight w, in T.
template <int D, int P, typename T>
PCMS_HD PCMS_INLINE void neighbour_data(const double (&u)[D], double inv_h, double inv_r2,
                                        int weight, T (&p)[Basis<D, P>::M], T &w)
{
    double d2 = u[0] * u[0];
    T xi[D];
    xi[0] = (T)(-u[0] * inv_h);
#pragma unroll
    for (int k = 1; k < D; ++k) {
        d2 = __builtin_fma(u[k], u[k], d2);
        xi[k] = (T)(-u[k] * inv_h);
    }
    if constexpr (sizeof(T) == sizeof(double)) {
        T q = sqrt((T)(d2 * inv_r2));
        w = weight_of<T>(weight, q);
    } else {
        // FP32 weights: 1 - q from 1 - q^2 formed in FP64, so that the weight
        // keeps its relative accuracy up to the support boundary (1 - q in
        // FP32 would round to 0 or 2^-24 steps there)
        const double x = d2 * inv_r2;
        const T q = sqrt((T)x);
        w = x < 1.0 ? weight_in<T>(weight, q, (T)(1.0 - x) / (T(1) + q)) : T(0);
    }
    monomials<D, P, T>(xi, p);
}

// Reference values of fields [l0, l0 + kFieldChunk) for a centred sum: the
// first kept source's values in the mixed modes (centring leaves the fit
// unchanged only without regularisation), else zero.
template <bool MIXED, int FC = kFieldChunk, class S_>
PCMS_HD PCMS_INLINE void field_refs(S_ &S, const KArgs &a, int l0, double (&fref)[FC])
{
    const double *sv0 = a.svals + (size_t)S.at(0) * a.nfs;
#pragma unroll
    for (int l = 0; l < FC; ++l)
        fref[l] = (MIXED && a.lambda == 0.0 && l0 + l < a.nf) ? sv0[l0 + l] : 0.0;
}

// One pass over the n kept sources with the coefficients y: acc[l] = sum_e
// w_e (p_e . y) (f_{e, l0 + l} - fref[l]), per lane (the caller sums over the
// group).  B neighbours' loads are issued together.
template <int D, int P, int G, int B, class S_, class FP>
PCMS_HD PCMS_INLINE void field_pass(S_ &S, const KArgs &a, const FP &fp, int n, double inv_h,
                                    double inv_r2, const double (&y)[Basis<D, P>::M], int l0,
                                    const double (&fref)[kFieldChunk], double (&acc)[kFieldChunk])
{
    constexpr int M = Basis<D, P>::M;
#pragma unroll
    for (int l = 0; l < kFieldChunk; ++l) acc[l] = 0.0;
    for (int e0 = S.g.q; e0 < n; e0 += G * B) {
        typename FP::Rec sb[B][D];
        bool ok[B];
        int pe[B];
        load_neighbours<D, G, B>(S, fp, e0, n, sb, ok, pe);
        double fv[B][kFieldChunk];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const double *sv = a.svals + (size_t)pe[j] * a.nfs + l0;
#pragma unroll
            for (int h = 0; h < kFieldChunk / 2; ++h) {
                fv[j][2 * h] = fv[j][2 * h + 1] = 0.0;
                if (l0 + 2 * h < a.nfs) load_pair(sv + 2 * h, fv[j][2 * h], fv[j][2 * h + 1]);
            }
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            double u[D], p[M], w;
            fp.offsets(sb[j], u);
            neighbour_data<D, P, double>(u, inv_h, inv_r2, a.weight, p, w);
            double py = 0.0;
#pragma unroll
            for (int v = 0; v < M; ++v) py = __builtin_fma(p[v], y[v], py);
            const double N = ok[j] ? w * py : 0.0;
#pragma unroll
            for (int l = 0; l < kFieldChunk; ++l) acc[l] = __builtin_fma(N, fv[j][l] - fref[l], acc[l]);
        }
    }
}

// Adds the refinement correction d of step `step` to y and applies the
// stopping rule: the correction predicts the next one as rho |d|, rho the
// observed contraction (|d| / |y| for step 0, whose correction is the FP32
// solution's error).  Returns 0 once that prediction is below 1e-9 |y|, or
// the correction itself is below 1e-8 |y| (converged); 1 to take another
// step; 2 when the corrections stop shrinking (at the last step, or above
// half of |y|) without having reached 1e-5 |y| (singular at FP32 accuracy).
template <int M, typename TA>
PCMS_HD PCMS_INLINE int refine_update(double (&y)[M], const TA (&d)[M], int step, double &nd_prev)
{
    double ny = 0.0, nd = 0.0;
#pragma unroll
    for (int u = 0; u < M; ++u) {
        ny = fmax(ny, fabs(y[u]));
        nd = fmax(nd, fabs((double)d[u]));
        y[u] += (double)d[u];
    }
    const double rho = step == 0 ? nd / ny : nd / nd_prev;
    nd_prev = nd;
    if (nd <= 1e-8 * ny || rho * nd <= 1e-9 * ny) return 0;
    if (!(nd <= 0.5 * ny) || step == kMaxRefine - 1) return nd <= 1e-5 * ny ? 0 : 2;
    return 1;
}

// The correction d = R^{-1} R^{-T} (e_0 - lambda y + res) of a residual
// partial sum res = -sum_e w_e (p_e . y) p_e (summed over the group here),
// solved in the arithmetic of the factor.
template <int M, int G, typename TA>
PCMS_HD PCMS_INLINE void refine_correction(const TA (&R)[M * (M + 1) / 2], const TA (&idg)[M],
                                           const double (&y)[M], const double (&res)[M],
                                           double lambda, Grp<G> g, TA (&d)[M])
{
#pragma unroll
    for (int u = 0; u < M; ++u) d[u] = (TA)(g.sum(res[u]) + ((u == 0 ? 1.0 : 0.0) - lambda * y[u]));
    chol_solve_in<M, TA>(R, idg, d);
}

// Refinement steps step0, step0 + 1, ... of y = (G + lambda I)^{-1} e_0 with
// the factor R of the FP32 moments as preconditioner: each step is one pass
// over the n kept sources forming the residual from FP64 data, then
// refine_update.  nd_prev: the previous correction's size.  Returns false
// when the target is singular at FP32 accuracy.
template <int D, int P, int G, int K, class S_, class FP, typename TA>
PCMS_HD PCMS_INLINE bool refine_steps(S_ &S, const KArgs &a, const FP &fp, int n, double inv_h,
                                      double inv_r2, const TA (&R)[Basis<D, P>::MM],
                                      const TA (&idg)[Basis<D, P>::M], double (&y)[Basis<D, P>::M],
                                      int step0, double nd_prev)
{
    constexpr int M = Basis<D, P>::M;
    for (int step = step0; step < kMaxRefine; ++step) {
        double res[M];
#pragma unroll
        for (int u = 0; u < M; ++u) res[u] = 0.0;
        for (int e0 = S.g.q; e0 < n; e0 += G * K) {
            typename FP::Rec sb[K][D];
            bool okn[K];
            int pe[K];
            load_neighbours<D, G, K>(S, fp, e0, n, sb, okn, pe);
#pragma unroll
            for (int j = 0; j < K; ++j) {
                double uo[D], p[M], w;
                fp.offsets(sb[j], uo);
                neighbour_data<D, P, double>(uo, inv_h, inv_r2, a.weight, p, w);
                double py = 0.0;
#pragma unroll
                for (int u = 0; u < M; ++u) py = __builtin_fma(p[u], y[u], py);
                const double c = okn[j] ? -w * py : 0.0;
#pragma unroll
                for (int u = 0; u < M; ++u) res[u] = __builtin_fma(c, p[u], res[u]);
            }
        }
        TA d[M];
        refine_correction<M, G, TA>(R, idg, y, res, a.lambda, S.g, d);
        const int r = refine_update<M, TA>(y, d, step, nd_prev);
        if (r == 0) return true;
        if (r == 2) return false;
    }
    return true;
}

// field_pass with the first refinement step folded in: besides the field
// sums acc with the coefficients y, the same pass forms the residual partial
// sum res = -sum_e w_e (p_e . y) p_e and, in FP32, the moments of the
// centred fields Bm[u][l] = sum_e w_e p_e,u (f_{e, l0 + l} - fref[l]).  The
// correction d of the residual then moves every fitted value by d . Bm[.][l]
// (the fit is linear in y), which needs no further pass; Bm only has to be
// accurate relative to that correction.
template <int D, int P, int G, int B, int FC, class S_, class FP>
PCMS_HD PCMS_INLINE void field_pass_fused(S_ &S, const KArgs &a, const FP &fp, int n, double inv_h,
                                          double inv_r2, const double (&y)[Basis<D, P>::M], int l0,
                                          const double (&fref)[FC], double (&acc)[FC],
                                          double (&res)[Basis<D, P>::M],
                                          float (&Bm)[Basis<D, P>::M][FC])
{
    constexpr int M = Basis<D, P>::M;
#pragma unroll
    for (int l = 0; l < FC; ++l) acc[l] = 0.0;
#pragma unroll
    for (int u = 0; u < M; ++u) {
        res[u] = 0.0;
#pragma unroll
        for (int l = 0; l < FC; ++l) Bm[u][l] = 0.0f;
    }
    for (int e0 = S.g.q; e0 < n; e0 += G * B) {
        typename FP::Rec sb[B][D];
        bool ok[B];
        int pe[B];
        load_neighbours<D, G, B>(S, fp, e0, n, sb, ok, pe);
        double fv[B][FC];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const double *sv = a.svals + (size_t)pe[j] * a.nfs + l0;
#pragma unroll
            for (int h = 0; h < FC / 2; ++h) {
                fv[j][2 * h] = fv[j][2 * h + 1] = 0.0;
                if (l0 + 2 * h < a.nfs) load_pair(sv + 2 * h, fv[j][2 * h], fv[j][2 * h + 1]);
            }
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            double u[D], p[M], w;
            fp.offsets(sb[j], u);
            neighbour_data<D, P, double>(u, inv_h, inv_r2, a.weight, p, w);
            w = ok[j] ? w : 0.0;
            double py = 0.0;
#pragma unroll
            for (int v = 0; v < M; ++v) py = __builtin_fma(p[v], y[v], py);
            const double N = w * py;
            float wf[FC];
#pragma unroll
            for (int l = 0; l < FC; ++l) {
                const double df = fv[j][l] - fref[l];
                acc[l] = __builtin_fma(N, df, acc[l]);
                wf[l] = (float)(w * df);
            }
#pragma unroll
            for (int v = 0; v < M; ++v) {
                res[v] = __builtin_fma(-N, p[v], res[v]);
                const float pv = (float)p[v];
#pragma unroll
                for (int l = 0; l < FC; ++l) Bm[v][l] = fma_t(pv, wf[l], Bm[v][l]);
            }
        }
    }
}

// Group sums of a field chunk, written to the target's outputs (or to its
// staged record, whose padding past nf receives zeros).
template <int G, int FC = kFieldChunk>
PCMS_HD PCMS_INLINE void write_fields(const KArgs &a, int ti, int l0, const double (&acc)[FC],
                                      const double (&fref)[FC], Grp<G> g)
{
    double v[FC];
#pragma unroll
    for (int l = 0; l < FC; ++l) v[l] = g.sum(acc[l]) + fref[l];
    if (a.stage) {
        double *rec = a.stage + (size_t)ti * a.nfs + l0;
#pragma unroll
        for (int h = 0; h < FC / 2; ++h)
            if (l0 + 2 * h < a.nfs && (h % G) == g.q) store_pair(rec + 2 * h, v[2 * h], v[2 * h + 1]);
        return;
    }
#pragma unroll
    for (int l = 0; l < FC; ++l)
        if (l0 + l < a.nf && (l % G) == g.q) a.out[(size_t)(l0 + l) * a.n_tgt + ti] = v[l];
}

// Field transfer of the target at sorted slot i; returns its status.
//
// EMIT (the precomputed transfer operator): instead of evaluating fields,
// write the shape functions N_e = w_e p_e . y of the kept sources with their
// sorted positions, slot e of sorted target i at [e * n_tgt + i], and the
// kept count at op_n[i] (-1 for a failed target); then fhat = sum_e N_e f_e
// for any field.
template <int D, int P, int PREC, bool UNIT, int G, bool EMIT = false, bool BVH = false>
PCMS_HD PCMS_INLINE int xfer_target(const KArgs &a, const GridParams &gp, int i, int *L, Grp<G> g)
{
    constexpr bool MIXED = PREC != PCMS_FP64;
    constexpr bool REFINE = PREC == PCMS_MIXED_REFINE;
    constexpr int M = Basis<D, P>::M;
    constexpr int MM = Basis<D, P>::MM;
    using TA = typename std::conditional<MIXED, float, double>::type;   // assembly type
    // neighbours per lane whose loads are issued together, per pass (fewer
    // where the pass holds more live registers)
    constexpr int kAsm = MIXED ? 4 : 2, kRef = MIXED ? 2 : 1, kApply = 2;
    // The FP32 moments of MIXED_REFINE, which only precondition the
    // refinement, are assembled from the fixed-point records (one load per
    // source); every other pass reads the FP64 records, so the weights that
    // enter the result are those of the exact positions (a weight near the
    // edge of the support, (1 - q)^4 with 1 - q ~ 1e-7, is too sensitive to
    // the position for any rounding of it).
    using FQ = FitPts<D, UNIT, REFINE>;
    using FP = FitPts<D, UNIT, false>;
    using RecQ = typename FQ::Rec;
    // small bases: the first refinement step of MIXED_REFINE rides on the
    // evaluation pass of the first kFused fields (their FP32 field moments
    // fit in registers)
    constexpr int kFused = 4;
    constexpr bool FUSED = REFINE && !EMIT && M <= 6;
    using Rec = typename FP::Rec;
    const int ti = a.tperm[i];
    Search<D, UNIT, G, BVH> S{gp, a.cs, a.spts, a.spts32, a.perm, {}, L, a.k_cap, a.words, g,
                              {a.bvh_nodes}};
    load_point<D>(a.tgt, ti, S.t);
    int n_found, n;
    double r2;
    // FP32 walks where they save loads: a point's FP32 record is one load (at
    // most 16 bytes) and its FP64 record is two (3-D and 4-D)
    int st = select_target<D, UNIT, G, MIXED && D >= 3 && D <= 4>(S, a, n_found, n, r2);
    if ((st & 0xF) == PCMS_TGT_OK && n < M) st |= PCMS_TGT_UNDERDETERMINED;
    double y[M];
    if ((st & 0xF) == PCMS_TGT_OK) {
        const double inv_h = 1.0 / sqrt(r2);
        const double inv_r2 = 1.0 / r2;
        const FP fp(a, gp, S.t);
        const FQ fq(a, gp, S.t);
        // moment matrix G = sum w p p^T (upper triangle, in TA); lane q takes
        // the neighbours e = q, q + G, ... and the group sums the partials
        TA Gm[MM];
#pragma unroll
        for (int j = 0; j < MM; ++j) Gm[j] = TA(0);
        for (int e0 = g.q; e0 < n; e0 += G * kAsm) {
            RecQ sb[kAsm][D];
            bool ok[kAsm];
            int pe[kAsm];
            load_neighbours<D, G, kAsm>(S, fq, e0, n, sb, ok, pe);
#pragma unroll
            for (int j = 0; j < kAsm; ++j) {
                double uo[D];
                fq.offsets(sb[j], uo);
                TA p[M], w;
                neighbour_data<D, P, TA>(uo, inv_h, inv_r2, a.weight, p, w);
                w = ok[j] ? w : TA(0);
#pragma unroll
                for (int u = 0; u < M; ++u) {
                    TA wp = w * p[u];
#pragma unroll
                    for (int v = u; v < M; ++v)
                        Gm[tri<M>(u, v)] = fma_t(wp, p[v], Gm[tri<M>(u, v)]);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < MM; ++j) Gm[j] = g.sum(Gm[j]);
        bool ok;
        TA idg[M];   // inverse diagonal of the FP32 factor (MIXED_REFINE)
#pragma unroll
        for (int u = 0; u < M; ++u) y[u] = u == 0 ? 1.0 : 0.0;
        if (!REFINE) {
            // FP64 factor of G + lambda I and the solve y = G^{-1} e_0
            double R[MM], idd[M];
#pragma unroll
            for (int j = 0; j < MM; ++j) R[j] = (double)Gm[j];
#pragma unroll
            for (int u = 0; u < M; ++u) R[tri<M>(u, u)] += a.lambda;
            ok = cholesky<M, double>(R, idd, MIXED ? kPivotFloorF32 : kPivotFloor);
            chol_solve<M, double>(R, idd, y);
        } else {
            // Iterative refinement with an FP32 factor of the FP32 moments as
            // the preconditioner: y += G32^{-1} (e_0 - (G + lambda I) y), the
            // residual formed entirely in FP64 (FP64 weights and monomials),
            // so y converges to the FP64 solution; the correction itself is
            // solved in FP32, the accuracy of the factor.  Each step's
            // correction d predicts the next one as rho |d|, rho the observed
            // contraction (|d| / |y| for the first step, whose correction is
            // the FP32 solution's error); refinement stops once that
            // prediction is below 1e-9 |y| (usually after one step), or the
            // correction itself is below 1e-8 |y|.  Ill-conditioned targets
            // take up to kMaxRefine steps, and a correction that does not
            // shrink marks the target singular at FP32 accuracy.
#pragma unroll
            for (int u = 0; u < M; ++u) Gm[tri<M>(u, u)] += (TA)a.lambda;
            ok = cholesky<M, TA>(Gm, idg, kPivotFloor);
            {
                TA y0[M];
#pragma unroll
                for (int u = 0; u < M; ++u) y0[u] = u == 0 ? TA(1) : TA(0);
                chol_solve_in<M, TA>(Gm, idg, y0);
#pragma unroll
                for (int u = 0; u < M; ++u) y[u] = (double)y0[u];
            }
            // with FUSED the first step is taken inside the evaluation pass
            if (!FUSED && ok)
                ok = refine_steps<D, P, G, kRef>(S, a, fp, n, inv_h, inv_r2, Gm, idg, y, 0, 0.0);
        }
        if (!ok) st |= PCMS_TGT_SINGULAR;
        if (EMIT) {
            if ((st & 0xF) == PCMS_TGT_OK) {
                for (int e0 = g.q; e0 < n; e0 += G * kApply) {
                    Rec sb[kApply][D];
                    bool okn[kApply];
                    int pe[kApply];
                    load_neighbours<D, G, kApply>(S, fp, e0, n, sb, okn, pe);
#pragma unroll
                    for (int j = 0; j < kApply; ++j) {
                        double uo[D], p[M], w;
                        fp.offsets(sb[j], uo);
                        neighbour_data<D, P, double>(uo, inv_h, inv_r2, a.weight, p, w);
                        double py = 0.0;
#pragma unroll
                        for (int u = 0; u < M; ++u) py = __builtin_fma(p[u], y[u], py);
                        if (okn[j]) {
                            const size_t at = (size_t)(e0 + j * G) * a.n_tgt + i;
                            a.op_w[at] = w * py;
                            a.op_c[at] = pe[j];
                        }
                    }
                }
            }
        } else if ((st & 0xF) == PCMS_TGT_OK) {
            int l_begin = 0;
            if constexpr (FUSED) {
                // the first chunk of fields with the first refinement step:
                // when one step is enough, the chunk's values are those of
                // the refined y; otherwise refinement continues with passes
                // of its own and the chunk is evaluated again
                double acc[kFused], fref[kFused], res[M];
                float Bm[M][kFused];
                field_refs<MIXED, kFused>(S, a, 0, fref);
                field_pass_fused<D, P, G, 1, kFused>(S, a, fp, n, inv_h, inv_r2, y, 0, fref, acc,
                                                     res, Bm);
                TA d[M];
                refine_correction<M, G, TA>(Gm, idg, y, res, a.lambda, g, d);
                double nd = 0.0;
                const int r = refine_update<M, TA>(y, d, 0, nd);
                if (r == 0) {
#pragma unroll
                    for (int l = 0; l < kFused; ++l) {
                        double c = 0.0;
#pragma unroll
                        for (int u = 0; u < M; ++u) c = __builtin_fma((double)d[u], (double)Bm[u][l], c);
                        acc[l] += c;
                    }
                    write_fields<G, kFused>(a, ti, 0, acc, fref, g);
                    l_begin = kFused;
                } else if (r == 2 ||
                           !refine_steps<D, P, G, kRef>(S, a, fp, n, inv_h, inv_r2, Gm, idg, y, 1, nd)) {
                    st |= PCMS_TGT_SINGULAR;
                    l_begin = a.nf;
                }
            }
            for (int l0 = l_begin; l0 < a.nf; l0 += kFieldChunk) {
                double acc[kFieldChunk], fref[kFieldChunk];
                field_refs<MIXED>(S, a, l0, fref);
                field_pass<D, P, G, kApply>(S, a, fp, n, inv_h, inv_r2, y, l0, fref, acc);
                write_fields<G>(a, ti, l0, acc, fref, g);
            }
        }
    }
    if (EMIT) {
        if (g.q == 0) a.op_n[i] = (st & 0xF) == PCMS_TGT_OK ? n : -1;
    } else if ((st & 0xF) != PCMS_TGT_OK) {
        if (a.stage) {
            for (int h = g.q; 2 * h < a.nfs; h += G)
                store_pair(a.stage + (size_t)ti * a.nfs + 2 * h, NAN, NAN);
        } else {
            for (int l = g.q; l < a.nf; l += G) a.out[(size_t)l * a.n_tgt + ti] = NAN;
        }
    }
    if (a.status && g.q == 0) a.status[ti] = (uint8_t)st;
    return st;
}

}  // namespace pcms
