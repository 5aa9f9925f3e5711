/*
 * TEST INFRASTRUCTURE ONLY -- plain, slow, FP64 CPU oracle for the
 * point-cloud field transfer by local weighted polynomial fitting.
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * load this file.  It shares no code with the HIP library and must never be
 * used as a fallback for it.
 *
 * What it computes (PCMS paper, Section 3.2.1):
 *   For every target t_i, the source set s^i = { s_j : phi(s_j, t_i) > 0 }
 *   selected by a radius (the selection function of Section 3.2.1, with the
 *   radius fixed, grown from an initial value until a minimum count is met,
 *   or set to the distance of the k-th nearest source), and the value at t_i
 *   of the weighted, Tikhonov-regularised least-squares polynomial of Eq. 1:
 *       c* = argmin_c  sum_j w_j (p(xi_j).c - f_j)^2 + lambda |c|^2,
 *       fhat_i = p(0).c* = c*_0,
 *   with the basis p = monomials of total degree <= p in target-centred,
 *   radius-scaled coordinates xi.  It is solved by the normal equations
 *   G c = B, G = sum_j w_j p_j p_j^T + lambda I, B = sum_j w_j p_j f_j^T,
 *   with a textbook Cholesky factorisation.
 *
 * Readings taken where the paper is silent (each listed in the design notes):
 *   - distance D_ij = fma chain over dimensions of u_k = (t_k - s_jk) g_k,
 *     evaluated in FP64 in dimension order (bit-reproducible predicate);
 *   - selection is strict, D_ij < r_i^2 (phi > 0 only strictly inside);
 *   - the weight enters the normal equations once (W = diag(phi));
 *   - the default weight is Wendland C2, (1-q)^4 (4q+1); Table 1's C4,
 *     Gaussian, constant and inverse multiquadric are also provided;
 *   - a neighbour cap keeps the k_cap nearest by (D, j), lists are reported
 *     by ascending source index;
 *   - growing radius: per target, r^2 <- 2 r^2 until the count reaches n_min
 *     or max_iter doublings are spent;
 *   - k-nearest radius: r_i^2 = k-th smallest D_ij (so k-1 points are kept
 *     strictly inside, the k-th sits where the weight vanishes);
 *   - a target with fewer than m kept sources is underdetermined (the
 *     paper's error condition), a Cholesky pivot <= 1e-13 * max diag(G)
 *     marks it singular; both give NaN outputs.
 *
 * The search is a plain bucket grid: for a query ball, every source in the
 * covering box of buckets is tested with the exact predicate.  A brute-force
 * mode tests every source and exists to pin the bucket search.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXD 5
#define ORC_MAXM 21

enum { ORC_OK = 0, ORC_UNDERDET = 1, ORC_SINGULAR = 2, ORC_EXHAUSTED = 3, ORC_CAPPED = 0x10 };
enum { ORC_FIXED = 0, ORC_KNN = 1, ORC_GROW = 2 };
enum { W_WENDLAND_C2 = 0, W_C4 = 1, W_GAUSSIAN = 2, W_CONST = 3, W_IMQ = 4 };

typedef struct {
    int mode;
    double r;
    int k;
    int n_min;
    int max_iter;
} orc_radius;

/* ------------------------------------------------------------------ */
/* distance and weight                                                  */
/* ------------------------------------------------------------------ */

/* D = u_{d-1}^2 + ... + u_0^2 as a chain of fused multiply-adds. */
static double metric_d2(const double *t, const double *s, const double *g, int dim)
{
    double u = (t[0] - s[0]) * g[0];
    double acc = u * u;
    for (int k = 1; k < dim; ++k) {
        u = (t[k] - s[k]) * g[k];
        acc = fma(u, u, acc);
    }
    return acc;
}

/* Radial weight as a function of q = r / r_c (Table 1; Wendland C2 added). */
double orc_weight(int kind, double q)
{
    const double a = 2.0; /* shape parameter used for Table 1's plots */
    if (!(q < 1.0)) return 0.0;
    switch (kind) {
    case W_WENDLAND_C2: {
        double o = 1.0 - q;
        return o * o * o * o * (4.0 * q + 1.0);
    }
    case W_C4: {
        double o = 1.0 - q;
        double poly = 5.0 * pow(q, 5) + 30.0 * pow(q, 4) + 72.0 * pow(q, 3) + 82.0 * q * q + 36.0 * q + 6.0;
        return poly * pow(o, 6);
    }
    case W_GAUSSIAN: return exp(-(a * q) * (a * q));
    case W_CONST: return 1.0;
    case W_IMQ: return 1.0 / sqrt(1.0 + (a * q) * (a * q));
    default: return NAN;
    }
}

/* ------------------------------------------------------------------ */
/* bucket grid                                                          */
/* ------------------------------------------------------------------ */

typedef struct {
    int dim;
    double lo[ORC_MAXD];
    double width[ORC_MAXD]; /* bucket width in raw coordinates */
    int64_t n[ORC_MAXD];
    int64_t n_cells;
    int64_t *start;  /* [n_cells + 1] */
    int64_t *items;  /* source indices grouped by bucket */
} bucket_grid;

static int64_t bucket_of(const bucket_grid *bg, int k, double x)
{
    double f = floor((x - bg->lo[k]) / bg->width[k]);
    if (!(f >= 0.0)) return 0;
    if (f >= (double)(bg->n[k] - 1)) return bg->n[k] - 1;
    return (int64_t)f;
}

/* ball_r: typical query radius in metric units, used to size the buckets. */
static int grid_build(bucket_grid *bg, const double *src, int64_t n_src, int dim, const double *g,
                      double ball_r)
{
    memset(bg, 0, sizeof(*bg));
    bg->dim = dim;
    double hi[ORC_MAXD];
    for (int k = 0; k < dim; ++k) { bg->lo[k] = INFINITY; hi[k] = -INFINITY; }
    for (int64_t j = 0; j < n_src; ++j)
        for (int k = 0; k < dim; ++k) {
            double x = src[j * dim + k];
            if (x < bg->lo[k]) bg->lo[k] = x;
            if (x > hi[k]) hi[k] = x;
        }
    if (n_src == 0)
        for (int k = 0; k < dim; ++k) { bg->lo[k] = 0.0; hi[k] = 0.0; }
    if (!(ball_r > 0.0) || !isfinite(ball_r)) ball_r = 1.0;
    double scale = 1.0;
    for (;;) {
        double total = 1.0;
        for (int k = 0; k < dim; ++k) {
            bg->width[k] = ball_r * scale / g[k];
            double ext = hi[k] - bg->lo[k];
            double nk = floor(ext / bg->width[k]) + 1.0;
            if (nk < 1.0) nk = 1.0;
            bg->n[k] = (int64_t)fmin(nk, 1e9);
            total *= (double)bg->n[k];
        }
        if (total <= 4.0 * (double)n_src + 64.0) { bg->n_cells = (int64_t)total; break; }
        scale *= 1.5;
    }
    bg->start = (int64_t *)calloc((size_t)bg->n_cells + 1, sizeof(int64_t));
    bg->items = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_src > 0 ? n_src : 1));
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_src > 0 ? n_src : 1));
    if (!bg->start || !bg->items || !cell) { free(cell); return -1; }
    for (int64_t j = 0; j < n_src; ++j) {
        int64_t id = 0;
        for (int k = dim - 1; k >= 0; --k) id = id * bg->n[k] + bucket_of(bg, k, src[j * dim + k]);
        cell[j] = id;
        bg->start[id + 1]++;
    }
    for (int64_t c = 0; c < bg->n_cells; ++c) bg->start[c + 1] += bg->start[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)bg->n_cells);
    memcpy(fill, bg->start, sizeof(int64_t) * (size_t)bg->n_cells);
    for (int64_t j = 0; j < n_src; ++j) bg->items[fill[cell[j]]++] = j;
    free(fill);
    free(cell);
    return 0;
}

static void grid_free(bucket_grid *bg)
{
    free(bg->start);
    free(bg->items);
}

typedef struct {
    int64_t j;
    double d2;
} cand;

typedef struct {
    cand *v;
    int64_t n, cap;
} cand_vec;

static void cv_push(cand_vec *cv, int64_t j, double d2)
{
    if (cv->n == cv->cap) {
        cv->cap = cv->cap ? 2 * cv->cap : 256;
        cv->v = (cand *)realloc(cv->v, sizeof(cand) * (size_t)cv->cap);
    }
    cv->v[cv->n].j = j;
    cv->v[cv->n].d2 = d2;
    cv->n++;
}

/* All sources in the buckets covering the metric ball of radius rho (a superset
 * of the ball), or all sources when brute is set.  Candidate D values are exact. */
static void gather(const bucket_grid *bg, const double *src, int64_t n_src, const double *g,
                   const double *t, double rho, int brute, cand_vec *out)
{
    int dim = bg->dim;
    out->n = 0;
    if (brute) {
        for (int64_t j = 0; j < n_src; ++j) cv_push(out, j, metric_d2(t, src + j * dim, g, dim));
        return;
    }
    int64_t a[ORC_MAXD], b[ORC_MAXD], c[ORC_MAXD];
    for (int k = 0; k < dim; ++k) {
        double half = rho / g[k] * (1.0 + 1e-9) + 1e-300;
        a[k] = bucket_of(bg, k, t[k] - half);
        b[k] = bucket_of(bg, k, t[k] + half);
        c[k] = a[k];
    }
    for (;;) {
        int64_t id = 0;
        for (int k = dim - 1; k >= 0; --k) id = id * bg->n[k] + c[k];
        for (int64_t p = bg->start[id]; p < bg->start[id + 1]; ++p) {
            int64_t j = bg->items[p];
            cv_push(out, j, metric_d2(t, src + j * dim, g, dim));
        }
        int k = 0;
        while (k < dim) {
            if (c[k] < b[k]) { c[k]++; break; }
            c[k] = a[k];
            k++;
        }
        if (k == dim) break;
    }
}

static int cmp_d2(const void *x, const void *y)
{
    double a = ((const cand *)x)->d2, b = ((const cand *)y)->d2;
    return (a > b) - (a < b);
}

static int cmp_d2_j(const void *x, const void *y)
{
    const cand *p = (const cand *)x, *q = (const cand *)y;
    if (p->d2 != q->d2) return (p->d2 > q->d2) - (p->d2 < q->d2);
    return (p->j > q->j) - (p->j < q->j);
}

static int cmp_j(const void *x, const void *y)
{
    int64_t a = ((const cand *)x)->j, b = ((const cand *)y)->j;
    return (a > b) - (a < b);
}

static int64_t count_below(const cand_vec *cv, double r2)
{
    int64_t n = 0;
    for (int64_t i = 0; i < cv->n; ++i) n += cv->v[i].d2 < r2;
    return n;
}

static double unit_ball_volume(int d)
{
    return pow(M_PI, 0.5 * d) / tgamma(0.5 * d + 1.0);
}

typedef struct {
    const double *src;
    int64_t n_src;
    int dim;
    const double *g;
    const orc_radius *rs;
    int k_cap;
    int brute;
    bucket_grid bg;
    double ball_r;
} search_ctx;

/* Radius, selection and cap for one target.  On return `sel` holds the kept
 * candidates sorted by source index; returns the status bits. */
static int select_one(const search_ctx *sc, const double *t, cand_vec *cv, cand_vec *sel,
                      int64_t *n_found_out, double *r2_out)
{
    const orc_radius *rs = sc->rs;
    double r2 = 0.0;
    int status = ORC_OK;
    if (rs->mode == ORC_FIXED) {
        r2 = rs->r * rs->r;
        gather(&sc->bg, sc->src, sc->n_src, sc->g, t, rs->r, sc->brute, cv);
    } else if (rs->mode == ORC_GROW) {
        r2 = rs->r * rs->r;
        gather(&sc->bg, sc->src, sc->n_src, sc->g, t, sqrt(r2), sc->brute, cv);
        int it = 0;
        while (count_below(cv, r2) < rs->n_min && it < rs->max_iter) {
            r2 = 2.0 * r2;
            ++it;
            gather(&sc->bg, sc->src, sc->n_src, sc->g, t, sqrt(r2), sc->brute, cv);
        }
        if (count_below(cv, r2) < rs->n_min) status = ORC_EXHAUSTED;
    } else { /* KNN: k-th smallest D over all sources */
        double rho = sc->ball_r;
        for (;;) {
            gather(&sc->bg, sc->src, sc->n_src, sc->g, t, rho, sc->brute, cv);
            /* every source with D < rho^2 lies in the gathered set */
            if (sc->brute || count_below(cv, rho * rho) >= rs->k || cv->n == sc->n_src) {
                qsort(cv->v, (size_t)cv->n, sizeof(cand), cmp_d2);
                r2 = cv->v[rs->k - 1].d2;
                break;
            }
            rho *= 2.0;
        }
    }
    /* strict selection */
    sel->n = 0;
    for (int64_t i = 0; i < cv->n; ++i)
        if (cv->v[i].d2 < r2) cv_push(sel, cv->v[i].j, cv->v[i].d2);
    int64_t n_found = sel->n;
    if (n_found > sc->k_cap) {
        qsort(sel->v, (size_t)sel->n, sizeof(cand), cmp_d2_j);
        sel->n = sc->k_cap;
        status |= ORC_CAPPED;
    }
    qsort(sel->v, (size_t)sel->n, sizeof(cand), cmp_j);
    *n_found_out = n_found;
    *r2_out = r2;
    return status;
}

static double typical_radius(const double *src, int64_t n_src, int dim, const double *g,
                             const orc_radius *rs)
{
    if (rs->mode != ORC_KNN) return rs->r;
    double vol = 1.0;
    for (int k = 0; k < dim; ++k) {
        double lo = INFINITY, hi = -INFINITY;
        for (int64_t j = 0; j < n_src; ++j) {
            double x = src[j * dim + k];
            lo = fmin(lo, x);
            hi = fmax(hi, x);
        }
        double e = (hi - lo) * g[k];
        vol *= (e > 0.0 ? e : 1.0);
    }
    double dens = (double)n_src / vol;
    return pow((double)rs->k / (dens * unit_ball_volume(dim)), 1.0 / dim);
}

static int ctx_init(search_ctx *sc, const double *src, int64_t n_src, int dim, const double *g,
                    const orc_radius *rs, int k_cap, int brute)
{
    sc->src = src;
    sc->n_src = n_src;
    sc->dim = dim;
    sc->g = g;
    sc->rs = rs;
    sc->k_cap = k_cap;
    sc->brute = brute;
    sc->ball_r = typical_radius(src, n_src, dim, g, rs);
    return grid_build(&sc->bg, src, n_src, dim, g, sc->ball_r);
}

static int check_args(int64_t n_src, int dim, const orc_radius *rs, int k_cap)
{
    if (n_src < 1 || dim < 1 || dim > ORC_MAXD || k_cap < 1) return -1;
    if (rs->mode == ORC_KNN && (rs->k < 1 || rs->k > n_src)) return -1;
    if (rs->mode != ORC_KNN && !(rs->r > 0.0 && isfinite(rs->r))) return -1;
    if (rs->mode == ORC_GROW && rs->max_iter < 0) return -1;
    return 0;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Neighbour lists: nbr[i*k_cap + e] = kept source indices, ascending. */
int orc_neighbors(const double *src, int64_t n_src, int dim, const double *g_in, const double *tgt,
                  int64_t n_tgt, const orc_radius *rs, int k_cap, int brute, int nthreads,
                  int32_t *nbr, int32_t *n_kept, int32_t *n_found, double *r2, uint8_t *status)
{
    double g[ORC_MAXD];
    if (check_args(n_src, dim, rs, k_cap)) return -1;
    for (int k = 0; k < dim; ++k) g[k] = g_in ? g_in[k] : 1.0;
    search_ctx sc;
    if (ctx_init(&sc, src, n_src, dim, g, rs, k_cap, brute)) return -2;
    set_threads(nthreads);
#pragma omp parallel
    {
        cand_vec cv = {0}, sel = {0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n_tgt; ++i) {
            int64_t nf;
            double rr;
            int st = select_one(&sc, tgt + i * dim, &cv, &sel, &nf, &rr);
            for (int64_t e = 0; e < sel.n; ++e) nbr[i * k_cap + e] = (int32_t)sel.v[e].j;
            n_kept[i] = (int32_t)sel.n;
            if (n_found) n_found[i] = (int32_t)nf;
            if (r2) r2[i] = rr;
            if (status) status[i] = (uint8_t)st;
        }
        free(cv.v);
        free(sel.v);
    }
    grid_free(&sc.bg);
    return 0;
}

/* ------------------------------------------------------------------ */
/* local weighted polynomial fit                                        */
/* ------------------------------------------------------------------ */

int orc_num_monomials(int dim, int degree)
{
    int m = 1;
    if (degree >= 1) m += dim;
    if (degree >= 2) m += dim * (dim + 1) / 2;
    return m;
}

/* Monomials of total degree <= degree, graded-lex order:
 * 1; x_0..x_{d-1}; x_a x_b for a <= b in lexicographic order of (a, b). */
static void monomials(const double *xi, int dim, int degree, double *p)
{
    int m = 0;
    p[m++] = 1.0;
    if (degree >= 1)
        for (int a = 0; a < dim; ++a) p[m++] = xi[a];
    if (degree >= 2)
        for (int a = 0; a < dim; ++a)
            for (int b = a; b < dim; ++b) p[m++] = xi[a] * xi[b];
}

/* Textbook Cholesky of the m x m SPD matrix G (row-major, full storage),
 * lower factor written into L.  Returns 0, or 1 if a pivot is not above
 * tau * max diag (the matrix is taken as singular).  The smallest ratio
 * pivot / max diag is stored in *ratio. */
static int cholesky(const double *G, int m, double *L, double *ratio)
{
    double maxdiag = 0.0;
    for (int i = 0; i < m; ++i) maxdiag = fmax(maxdiag, G[i * m + i]);
    double minr = INFINITY;
    memset(L, 0, sizeof(double) * (size_t)(m * m));
    for (int j = 0; j < m; ++j) {
        double s = G[j * m + j];
        for (int k = 0; k < j; ++k) s -= L[j * m + k] * L[j * m + k];
        double r = (maxdiag > 0.0) ? s / maxdiag : -1.0;
        if (r < minr) minr = r;
        if (!(s > 1e-13 * maxdiag) || !(maxdiag > 0.0)) { *ratio = minr; return 1; }
        double d = sqrt(s);
        L[j * m + j] = d;
        for (int i = j + 1; i < m; ++i) {
            double t = G[i * m + j];
            for (int k = 0; k < j; ++k) t -= L[i * m + k] * L[j * m + k];
            L[i * m + j] = t / d;
        }
    }
    *ratio = minr;
    return 0;
}

/* Solve L L^T x = b in place. */
static void chol_solve(const double *L, int m, double *x)
{
    for (int i = 0; i < m; ++i) {
        double s = x[i];
        for (int k = 0; k < i; ++k) s -= L[i * m + k] * x[k];
        x[i] = s / L[i * m + i];
    }
    for (int i = m - 1; i >= 0; --i) {
        double s = x[i];
        for (int k = i + 1; k < m; ++k) s -= L[k * m + i] * x[k];
        x[i] = s / L[i * m + i];
    }
}

typedef struct {
    int degree;
    int weight;
    double lambda;
} fit_opts;

/* Fit one target from its kept list.  Writes n_fields values (or NaN), and the
 * shape functions N_e = w_e p_e^T G^{-1} e_0 when `shape` is given. */
static int fit_one(const search_ctx *sc, const fit_opts *fo, const double *t, const cand_vec *sel,
                   double r2, const double *vals, int n_fields, int64_t n_src, double *out_vals,
                   int64_t out_stride, double *shape, double *pivot_ratio)
{
    int dim = sc->dim;
    int m = orc_num_monomials(dim, fo->degree);
    double G[ORC_MAXM * ORC_MAXM], L[ORC_MAXM * ORC_MAXM], p[ORC_MAXM], xi[ORC_MAXD];
    double *B = (double *)calloc((size_t)(m * n_fields), sizeof(double));
    memset(G, 0, sizeof(G));
    double h = sqrt(r2);
    for (int64_t e = 0; e < sel->n; ++e) {
        const double *s = sc->src + sel->v[e].j * dim;
        for (int k = 0; k < dim; ++k) xi[k] = (s[k] - t[k]) * sc->g[k] / h;
        double q = sqrt(sel->v[e].d2 / r2);
        double w = orc_weight(fo->weight, q);
        monomials(xi, dim, fo->degree, p);
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) G[a * m + b] += w * p[a] * p[b];
        for (int l = 0; l < n_fields; ++l) {
            double f = vals[(int64_t)l * n_src + sel->v[e].j];
            for (int a = 0; a < m; ++a) B[a * n_fields + l] += w * p[a] * f;
        }
    }
    for (int a = 0; a < m; ++a) G[a * m + a] += fo->lambda;
    double ratio;
    int sing = cholesky(G, m, L, &ratio);
    if (pivot_ratio) *pivot_ratio = ratio;
    if (sing) {
        for (int l = 0; l < n_fields; ++l) out_vals[l * out_stride] = NAN;
        free(B);
        return ORC_SINGULAR;
    }
    double x[ORC_MAXM];
    for (int l = 0; l < n_fields; ++l) {
        for (int a = 0; a < m; ++a) x[a] = B[a * n_fields + l];
        chol_solve(L, m, x);
        out_vals[l * out_stride] = x[0];
    }
    if (shape) {
        double y[ORC_MAXM] = {0};
        y[0] = 1.0;
        chol_solve(L, m, y);
        for (int64_t e = 0; e < sel->n; ++e) {
            const double *s = sc->src + sel->v[e].j * dim;
            for (int k = 0; k < dim; ++k) xi[k] = (s[k] - t[k]) * sc->g[k] / h;
            double w = orc_weight(fo->weight, sqrt(sel->v[e].d2 / r2));
            monomials(xi, dim, fo->degree, p);
            double acc = 0.0;
            for (int a = 0; a < m; ++a) acc += p[a] * y[a];
            shape[e] = w * acc;
        }
    }
    free(B);
    return ORC_OK;
}

/* Field transfer: out[l*n_tgt + i] = fitted value of field l at target i.
 * nbr/n_kept (nullable) also report the lists, shape (nullable,
 * [n_tgt*k_cap]) the shape functions aligned with nbr. */
int orc_transfer(const double *src, int64_t n_src, int dim, const double *g_in, const double *vals,
                 int n_fields, const double *tgt, int64_t n_tgt, int degree, const orc_radius *rs,
                 int k_cap, int weight, double lambda, int brute, int nthreads, double *out,
                 uint8_t *status, double *pivot_ratio, int32_t *nbr, int32_t *n_kept, double *shape)
{
    double g[ORC_MAXD];
    if (check_args(n_src, dim, rs, k_cap)) return -1;
    if (degree < 0 || degree > 2 || n_fields < 1 || lambda < 0.0) return -1;
    int m = orc_num_monomials(dim, degree);
    if (k_cap < m) return -1;
    for (int k = 0; k < dim; ++k) g[k] = g_in ? g_in[k] : 1.0;
    search_ctx sc;
    if (ctx_init(&sc, src, n_src, dim, g, rs, k_cap, brute)) return -2;
    fit_opts fo = {degree, weight, lambda};
    set_threads(nthreads);
#pragma omp parallel
    {
        cand_vec cv = {0}, sel = {0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n_tgt; ++i) {
            int64_t nf;
            double rr, ratio = NAN;
            const double *t = tgt + i * dim;
            int st = select_one(&sc, t, &cv, &sel, &nf, &rr);
            if (nbr) {
                for (int64_t e = 0; e < sel.n; ++e) nbr[i * k_cap + e] = (int32_t)sel.v[e].j;
            }
            if (n_kept) n_kept[i] = (int32_t)sel.n;
            int base = st & ~ORC_CAPPED;
            if (base == ORC_OK && sel.n < m) base = ORC_UNDERDET;
            if (base != ORC_OK) {
                for (int l = 0; l < n_fields; ++l) out[(int64_t)l * n_tgt + i] = NAN;
            } else {
                base = fit_one(&sc, &fo, t, &sel, rr, vals, n_fields, n_src, out + i, n_tgt,
                               shape ? shape + i * k_cap : NULL, &ratio);
            }
            if (status) status[i] = (uint8_t)(base | (st & ORC_CAPPED));
            if (pivot_ratio) pivot_ratio[i] = ratio;
        }
        free(cv.v);
        free(sel.v);
    }
    grid_free(&sc.bg);
    return 0;
}

int orc_version(void) { return 1; }

/* Threads an OpenMP region of this library uses by default. */
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
