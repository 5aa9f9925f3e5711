// C entry points: argument validation (host only, before any HIP call),
// orchestration of the grid build, target ordering, search and fit kernels
// on the caller's stream, and the status/return-code plumbing.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <memory>
#include <functional>
#include <mutex>
#include <new>
#include <string>

#include "fit.h"
#include "bvh.h"
#include "internal.h"

namespace pcms {

namespace {
thread_local std::string g_last_error;

bool finite_pos(double x) { return x > 0.0 && std::isfinite(x); }

int num_monomials(int dim, int degree)
{
    return degree == 0 ? 1 : degree == 1 ? 1 + dim : 1 + dim + dim * (dim + 1) / 2;
}

double unit_ball_volume(int d)
{
    return pow(M_PI, 0.5 * d) / tgamma(0.5 * d + 1.0);
}

pcms_status arg_error(const std::string &m)
{
    set_error(m);
    return PCMS_ERR_ARG;
}

pcms_status check_radius(const pcms_radius *r, int64_t n_src)
{
    if (!r) return arg_error("radius is NULL");
    if (r->mode == PCMS_RADIUS_FIXED) {
        if (!finite_pos(r->r)) return arg_error("fixed radius must be finite and > 0");
    } else if (r->mode == PCMS_RADIUS_GROW) {
        if (!finite_pos(r->r)) return arg_error("initial radius must be finite and > 0");
        if (r->n_min < 1) return arg_error("n_min must be >= 1");
        if (r->max_iter < 0 || r->max_iter > 2000) return arg_error("max_iter must be in [0, 2000]");
    } else if (r->mode == PCMS_RADIUS_KNN) {
        if (r->k < 1 || (int64_t)r->k > n_src) return arg_error("KNN k must be in [1, n_src]");
    } else {
        return arg_error("unknown radius mode");
    }
    return PCMS_OK;
}

pcms_status check_scale(const double *g, int dim)
{
    if (!g) return PCMS_OK;
    for (int k = 0; k < dim; ++k)
        if (!finite_pos(g[k])) return arg_error("inv_scale entries must be finite and > 0");
    return PCMS_OK;
}

pcms_status check_opts(const pcms_mls_opts *o)
{
    if (!o) return PCMS_OK;
    if (o->weight < PCMS_WEIGHT_WENDLAND_C2 || o->weight > PCMS_WEIGHT_NO_OP)
        return arg_error("unknown weight function");
    if (o->precision < PCMS_FP64 || o->precision > PCMS_MIXED_REFINE)
        return arg_error("unknown precision");
    if (!(o->lambda >= 0.0) || !std::isfinite(o->lambda)) return arg_error("lambda must be finite and >= 0");
    if (o->block != 0 && o->block != 64 && o->block != 128 && o->block != 256)
        return arg_error("block must be 0, 64, 128 or 256");
    if ((o->flags & PCMS_ASYNC) && !o->summary)
        return arg_error("PCMS_ASYNC needs a device summary buffer");
    if (o->flags & ~(PCMS_ASYNC | PCMS_PROFILE | PCMS_LBVH)) return arg_error("unknown flag bits");
    return PCMS_OK;
}

// Cell sizing for a one-shot call: buckets a fixed fraction of the support
// radius wide (0.7 of the expected kNN radius, one fixed or initial radius);
// PCMS_CELL_FACTOR overrides the fraction.
void cell_spec(const pcms_radius *r, int dim, double *cell_width, double *pts_per_cell,
               double cf_override = 0.0)
{
    *cell_width = 0.0;
    *pts_per_cell = 0.0;
    const char *env = getenv("PCMS_CELL_FACTOR");
    double cf = cf_override > 0.0 ? cf_override
              : env ? atof(env) : (r->mode == PCMS_RADIUS_KNN ? 0.7 : 1.0);
    if (!(cf > 0.0)) cf = 1.0;
    if (r->mode == PCMS_RADIUS_KNN)
        *pts_per_cell = pow(cf, dim) * r->k / unit_ball_volume(dim);
    else
        *cell_width = cf * r->r;
}

// Leaf size of the LBVHs the one-shot calls build (PCMS_LBVH_LEAF overrides).
int lbvh_leaf_default()
{
    const char *env = getenv("PCMS_LBVH_LEAF");
    const int v = env ? atoi(env) : 0;
    return v >= 1 && v <= kBvhLeafMax ? v : kBvhLeaf;
}

// Reads {"block": B, "cell_factor": F} from a file written by pcms_autotune.
bool read_tune_cache(const char *path, int *block, double *cf)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char buf[512];
    const size_t n = std::fread(buf, 1, sizeof(buf) - 1, f);
    std::fclose(f);
    buf[n] = 0;
    const char *b = std::strstr(buf, "\"block\":");
    const char *c = std::strstr(buf, "\"cell_factor\":");
    if (!b || !c) return false;
    const int bv = std::atoi(b + 8);
    const double cv = std::atof(c + 14);
    if (bv != 64 && bv != 128 && bv != 256) return false;
    if (!(cv > 0.0 && cv <= 4.0)) return false;
    *block = bv;
    *cf = cv;
    return true;
}

struct Scratch {
    void *p = nullptr;
    hipStream_t s = nullptr;
    ~Scratch()
    {
        if (p) scratch_free(p, s);
    }
};

void grid_alloc_free(Grid *g)
{
    if (!g) return;
    if (g->params) (void)hipFree(g->params);
    if (g->cell_start) (void)hipFree(g->cell_start);
    if (g->perm) (void)hipFree(g->perm);
    if (g->iperm) (void)hipFree(g->iperm);
    if (g->spts) (void)hipFree(g->spts);
    if (g->spts32) (void)hipFree(g->spts32);
    if (g->bvh_nodes) (void)hipFree(g->bvh_nodes);
    delete g;
}

// Statuses -> return code (synchronous mode).
pcms_status finish(const int32_t *summary_dev, bool async, hipStream_t s, bool judge_underdet)
{
    if (async) return PCMS_OK;
    int32_t h[4] = {0, 0, 0, 0};
    PCMS_HIP(hipMemcpyAsync(h, summary_dev, sizeof(h), hipMemcpyDeviceToHost, s));
    PCMS_HIP(hipStreamSynchronize(s));
    if (judge_underdet && h[0] > 0) {
        set_error(std::to_string(h[0]) + " target(s) underdetermined");
        return PCMS_ERR_UNDERDETERMINED;
    }
    if (h[1] > 0) {
        set_error(std::to_string(h[1]) + " target(s) with a singular moment matrix");
        return PCMS_ERR_SINGULAR;
    }
    if (h[2] > 0) {
        set_error(std::to_string(h[2]) + " target(s) ran out of radius doublings");
        return PCMS_ERR_RADIUS_EXHAUSTED;
    }
    return PCMS_OK;
}

std::once_flag g_pool_once[64];

// Phase timing with HIP events (PCMS_PROFILE).
// Phase timing with HIP events (PCMS_PROFILE).  A profiled call records
// kPhases + 1 events on its stream and does not wait for them: its times are
// read once a later profiled call has been enqueued (so the device always has
// queued work), or when they are queried.  Two event sets alternate.
constexpr int kPhases = 5;
struct EventSet {
    hipEvent_t ev[kPhases + 1] = {};
    bool have[kPhases + 1] = {};
    bool pending = false;
};
struct Profiler {
    bool on = false;
    hipStream_t s = nullptr;
    EventSet set[2];
    int cur = 0;
    float last[kPhases] = {};
    double sum[kPhases] = {};
    int n_last = 0, calls = 0;

    pcms_status mark(int i)
    {
        if (!on) return PCMS_OK;
        EventSet &e = set[cur];
        if (!e.ev[i]) PCMS_HIP(hipEventCreate(&e.ev[i]));
        PCMS_HIP(hipEventRecord(e.ev[i], s));
        e.have[i] = true;
        return PCMS_OK;
    }
    // Waits for a pending set and adds its phase times to the statistics.
    pcms_status resolve(int k)
    {
        EventSet &e = set[k];
        if (!e.pending) return PCMS_OK;
        e.pending = false;
        int lastev = -1;
        for (int i = kPhases; i >= 0 && lastev < 0; --i)
            if (e.have[i]) lastev = i;
        if (lastev < 0) return PCMS_OK;
        PCMS_HIP(hipEventSynchronize(e.ev[lastev]));
        for (int i = 0; i < kPhases; ++i) {
            float ms = 0.0f;
            if (e.have[i] && e.have[i + 1]) PCMS_HIP(hipEventElapsedTime(&ms, e.ev[i], e.ev[i + 1]));
            last[i] = ms;
            sum[i] += ms;
        }
        n_last = kPhases;
        ++calls;
        return PCMS_OK;
    }
    pcms_status resolve_all()
    {
        const int older = cur ^ 1;
        pcms_status st = resolve(older);
        if (st != PCMS_OK) return st;
        return resolve(cur);
    }
};
thread_local Profiler g_prof;

pcms_status profile_begin(const pcms_mls_opts *o, hipStream_t s)
{
    g_prof.on = o && (o->flags & PCMS_PROFILE);
    if (!g_prof.on) return PCMS_OK;
    g_prof.cur ^= 1;
    // the set about to be reused belongs to the call before the previous one
    pcms_status st = g_prof.resolve(g_prof.cur);
    if (st != PCMS_OK) return st;
    g_prof.s = s;
    for (bool &h : g_prof.set[g_prof.cur].have) h = false;
    return g_prof.mark(0);
}

// After the call's work is enqueued: its events are pending, and the
// previous call's times are read (that call has completed or is completing
// ahead of this one on the device).
pcms_status profile_end()
{
    if (!g_prof.on) return PCMS_OK;
    g_prof.set[g_prof.cur].pending = true;
    g_prof.on = false;
    return g_prof.resolve(g_prof.cur ^ 1);
}

}  // namespace

void profile_off() { g_prof.on = false; }

void set_error(const std::string &msg) { g_last_error = msg; }

pcms_status hip_fail(hipError_t e, const char *what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? PCMS_ERR_NOMEM : PCMS_ERR_HIP;
}

pcms_status scratch_alloc(void **p, size_t bytes, hipStream_t s)
{
    int dev = 0;
    PCMS_HIP(hipGetDevice(&dev));
    if (dev >= 0 && dev < 64) {
        std::call_once(g_pool_once[dev], [dev]() {
            hipMemPool_t pool;
            if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
                uint64_t keep = UINT64_MAX;   // keep freed blocks cached in the pool
                (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
            }
        });
    }
    hipError_t e = hipMallocAsync(p, bytes > 0 ? bytes : 256, s);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync");
    return PCMS_OK;
}

void scratch_free(void *p, hipStream_t s)
{
    if (p) (void)hipFreeAsync(p, s);
}

namespace {
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
// workspace of a transfer on a grid:
// [summary | tperm | svals | staged outputs | sort buffers]
struct TransferWs {
    size_t off_tperm, off_svals, off_stage, off_sort, bytes;
    TransferWs(int64_t n_src, int n_fields, int64_t n_tgt)
    {
        off_tperm = 256;
        off_svals = off_tperm + align256(sizeof(int) * (size_t)n_tgt);
        off_stage = off_svals + align256(sizeof(double) * (size_t)n_src * padded_dim(n_fields));
        off_sort = off_stage + align256(sizeof(double) * (size_t)n_tgt * padded_dim(n_fields));
        bytes = off_sort + sort_targets_bytes(n_tgt);
    }
};
}  // namespace

// Arrays of a grid over n_src sources: parameters, cell starts, both
// permutations, FP64 and FP32 coordinate records; for an LBVH a single
// bucket and the tree's nodes.
struct GridLayout {
    size_t o_cs, o_perm, o_iperm, o_spts, o_s32, o_bvh, bytes;
    int cells;
    GridLayout(int64_t n_src, int dim, bool lbvh = false)
    {
        cells = lbvh ? 1 : cells_cap_for(n_src);
        o_cs = align256(sizeof(GridParams));
        o_perm = o_cs + align256(sizeof(int) * ((size_t)cells + 1));
        o_iperm = o_perm + align256(sizeof(int) * (size_t)n_src);
        o_spts = o_iperm + align256(sizeof(int) * (size_t)n_src);
        o_s32 = o_spts + align256(sizeof(double) * (size_t)n_src * padded_dim(dim));
        o_bvh = o_s32 + align256(sizeof(float) * 2 * (size_t)n_src * dim);   // FP32 + fixed-point
        bytes = o_bvh + (lbvh ? bvh_node_bytes(n_src, dim) : 0);
    }
    // Points g's arrays into the block at base.
    void place(Grid &g, void *base, bool lbvh) const
    {
        char *b = (char *)base;
        g.n_cells_cap = cells;
        g.params = (GridParams *)b;
        g.cell_start = (int *)(b + o_cs);
        g.perm = (int *)(b + o_perm);
        g.iperm = (int *)(b + o_iperm);
        g.spts = (double *)(b + o_spts);
        g.spts32 = (float *)(b + o_s32);
        g.sq = reinterpret_cast<uint32_t *>(g.spts32 + (size_t)g.n_src * g.dim);
        g.bvh_nodes = lbvh ? (float *)(b + o_bvh) : nullptr;
        g.lbvh = lbvh ? 1 : 0;
    }
};

// Scratch that build_lbvh_device takes while it runs.
size_t lbvh_build_scratch_bytes(int64_t n_src)
{
    return grid_build_scratch_bytes(n_src) + 256 + sizeof(int) * bvh_link_ints(n_src);
}

size_t transfer_ws_bytes(int64_t n_src, int n_fields, int64_t n_tgt)
{
    return TransferWs(n_src, n_fields, n_tgt).bytes;
}

void transfer_ws_order(void *ws, int64_t n_src, int n_fields, int64_t n_tgt, int **tperm,
                       void **sort_ws)
{
    const TransferWs L(n_src, n_fields, n_tgt);
    *tperm = (int *)((char *)ws + L.off_tperm);
    *sort_ws = (char *)ws + L.off_sort;
}

namespace {
// The calling thread's side stream on each device, with its fork and join
// events; created on first use and kept for the life of the thread (never
// destroyed: the runtime may already be gone when a thread's storage is).
struct Side {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
constexpr int kSideDevices = 64;
thread_local Side g_side[kSideDevices];

pcms_status side_stream(Side **out)
{
    int dev = 0;
    PCMS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kSideDevices) {
        set_error("device ordinal " + std::to_string(dev) + " beyond the supported 64");
        return PCMS_ERR_ARG;
    }
    Side &sd = g_side[dev];
    if (!sd.s) {
        PCMS_HIP(hipStreamCreateWithFlags(&sd.s, hipStreamNonBlocking));
        PCMS_HIP(hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming));
        PCMS_HIP(hipEventCreateWithFlags(&sd.join, hipEventDisableTiming));
    }
    *out = &sd;
    return PCMS_OK;
}
}  // namespace

pcms_status side_fork(hipStream_t s)
{
    Side *sd = nullptr;
    pcms_status st = side_stream(&sd);
    if (st != PCMS_OK) return st;
    PCMS_HIP(hipEventRecord(sd->fork, s));
    return PCMS_OK;
}

pcms_status order_targets_aside(const Grid *g, const double *tgt, int64_t n_tgt, int *tperm,
                                void *sort_ws, hipStream_t s, hipEvent_t *join, bool record_fork)
{
    Side *sd = nullptr;
    pcms_status st = side_stream(&sd);
    if (st != PCMS_OK) return st;
    if (record_fork) PCMS_HIP(hipEventRecord(sd->fork, s));
    PCMS_HIP(hipStreamWaitEvent(sd->s, sd->fork, 0));
    if ((st = sort_targets(g, tgt, n_tgt, tperm, sd->s, sort_ws)) != PCMS_OK) return st;
    PCMS_HIP(hipEventRecord(sd->join, sd->s));
    *join = sd->join;
    return PCMS_OK;
}

pcms_status transfer_on_grid(const Grid *g, const double *src_vals, int32_t n_fields,
                             const double *tgt, int64_t n_tgt, int32_t degree,
                             const pcms_radius *radius, int32_t k_cap, const pcms_mls_opts *opts,
                             hipStream_t s, double *tgt_vals, uint8_t *status, void *ws,
                             bool overlap, hipEvent_t ordered)
{
    pcms_mls_opts o;
    pcms_mls_opts_default(&o);
    if (opts) o = *opts;
    const bool async = (o.flags & PCMS_ASYNC) != 0;
    const TransferWs L(g->n_src, n_fields, n_tgt);
    Scratch sc;
    sc.s = s;
    pcms_status st;
    if (!ws) {
        if ((st = scratch_alloc(&sc.p, L.bytes, s)) != PCMS_OK) return st;
        ws = sc.p;
    }
    int32_t *summary = async ? o.summary : (int32_t *)ws;
    int *tperm = (int *)((char *)ws + L.off_tperm);
    double *svals = (double *)((char *)ws + L.off_svals);
    double *stage = (double *)((char *)ws + L.off_stage);
    if ((st = zero_ints(summary, 4, s)) != PCMS_OK) return st;
    if ((st = g_prof.mark(1)) != PCMS_OK) return st;
    // the target order: forked off already, forked off now (to overlap the
    // field gather), or in line
    hipEvent_t join = ordered;
    if (!join && overlap) {
        st = order_targets_aside(g, tgt, n_tgt, tperm, (char *)ws + L.off_sort, s, &join);
        if (st != PCMS_OK) return st;
    } else if (!join) {
        if ((st = sort_targets(g, tgt, n_tgt, tperm, s, (char *)ws + L.off_sort)) != PCMS_OK)
            return st;
    }
    if ((st = g_prof.mark(2)) != PCMS_OK) return st;
    if ((st = gather_values(g, src_vals, n_fields, svals, s)) != PCMS_OK) return st;
    if ((st = g_prof.mark(3)) != PCMS_OK) return st;
    if (join) PCMS_HIP(hipStreamWaitEvent(s, join, 0));
    LaunchSpec ls{g, tgt, tperm, n_tgt, *radius, k_cap, o.block, summary};
    st = launch_transfer(ls, svals, n_fields, degree, o.weight, o.precision, o.lambda, tgt_vals,
                         stage, status, s);
    if (st != PCMS_OK) return st;
    if ((st = g_prof.mark(4)) != PCMS_OK) return st;
    if ((st = unstage_fields(stage, n_tgt, n_fields, tgt_vals, s)) != PCMS_OK) return st;
    if ((st = g_prof.mark(5)) != PCMS_OK) return st;
    if ((st = profile_end()) != PCMS_OK) return st;
    return finish(summary, async, s, true);
}

pcms_status check_transfer_args(int64_t n_src, int32_t dim, const double *src_vals,
                                int32_t n_fields, const double *tgt, int64_t n_tgt, int32_t degree,
                                const pcms_radius *radius, int32_t k_cap,
                                const pcms_mls_opts *opts, double *tgt_vals)
{
    if (dim < 1 || dim > kMaxDim) return arg_error("dim must be in [1, 5]");
    if (degree < 0 || degree > 2) return arg_error("basis_degree must be in [0, 2]");
    if (n_fields < 1) return arg_error("n_fields must be >= 1");
    if (n_tgt < 0 || n_tgt >= ((int64_t)1 << 31) / 2) return arg_error("n_tgt must be in [0, 2^30)");
    const int m = num_monomials(dim, degree);
    if (k_cap < m || k_cap > kMaxKcap) return arg_error("k_cap must be in [m, 256]");
    pcms_status st = check_radius(radius, n_src);
    if (st != PCMS_OK) return st;
    if ((st = check_opts(opts)) != PCMS_OK) return st;
    if (n_tgt > 0 && (!src_vals || !tgt || !tgt_vals)) return arg_error("src_vals, tgt and tgt_vals are required");
    return PCMS_OK;
}

}  // namespace pcms

using namespace pcms;

extern "C" {

void pcms_mls_opts_default(pcms_mls_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->weight = PCMS_WEIGHT_WENDLAND_C2;
    o->precision = PCMS_FP64;
    o->lambda = 0.0;
}

int32_t pcms_version(void) { return 100; }

int32_t pcms_last_phase_ms(float *ms, int32_t n)
{
    if (!ms || n <= 0) return 0;
    if (g_prof.resolve_all() != PCMS_OK) return 0;
    int c = n < g_prof.n_last ? n : g_prof.n_last;
    for (int i = 0; i < c; ++i) ms[i] = g_prof.last[i];
    return c;
}

int32_t pcms_phase_ms_sum(double *sum_ms, int32_t n, int32_t reset)
{
    if (g_prof.resolve_all() != PCMS_OK) return -1;
    const int calls = g_prof.calls;
    if (sum_ms)
        for (int i = 0; i < n && i < kPhases; ++i) sum_ms[i] = g_prof.sum[i];
    if (reset) {
        for (double &x : g_prof.sum) x = 0.0;
        g_prof.calls = 0;
    }
    return calls;
}

const char *pcms_last_error(void) { return g_last_error.c_str(); }

static pcms_status grid_create(int64_t n_src, int32_t dim, const double *inv_scale, bool lbvh,
                               Grid **out)
{
    Grid *g = new (std::nothrow) Grid();
    if (!g) return PCMS_ERR_NOMEM;
    g->dim = dim;
    g->n_src = n_src;
    g->n_cells_cap = lbvh ? 1 : cells_cap_for(n_src);
    for (int k = 0; k < kMaxDim; ++k) g->g[k] = (inv_scale && k < dim) ? inv_scale[k] : 1.0;
    hipError_t e;
    if ((e = hipGetDevice(&g->device)) != hipSuccess ||
        (e = hipMalloc(&g->params, sizeof(GridParams))) != hipSuccess ||
        (e = hipMalloc(&g->cell_start, sizeof(int) * ((size_t)g->n_cells_cap + 1))) != hipSuccess ||
        (e = hipMalloc(&g->perm, sizeof(int) * (size_t)n_src)) != hipSuccess ||
        (e = hipMalloc(&g->iperm, sizeof(int) * (size_t)n_src)) != hipSuccess ||
        (e = hipMalloc(&g->spts, sizeof(double) * (size_t)n_src * padded_dim(dim))) != hipSuccess ||
        (e = hipMalloc(&g->spts32, sizeof(float) * 2 * (size_t)n_src * dim)) != hipSuccess ||
        (lbvh && (e = hipMalloc(&g->bvh_nodes, bvh_node_bytes(n_src, dim))) != hipSuccess)) {
        grid_alloc_free(g);
        return hip_fail(e, "hipMalloc(grid)");
    }
    g->sq = reinterpret_cast<uint32_t *>(g->spts32 + (size_t)n_src * dim);
    *out = g;
    return PCMS_OK;
}

pcms_status pcms_grid_build(const double *src, int64_t n_src, int32_t dim, const double *inv_scale,
                            double cell_width, double pts_per_cell, pcms_stream_t stream,
                            pcms_grid **out)
{
    if (!out) return arg_error("out is NULL");
    *out = nullptr;
    if (dim < 1 || dim > kMaxDim) return arg_error("dim must be in [1, 5]");
    if (n_src < 1 || n_src >= ((int64_t)1 << 31) / 2) return arg_error("n_src must be in [1, 2^30)");
    if (!src) return arg_error("src is NULL");
    if (!(cell_width >= 0.0) || !std::isfinite(cell_width)) return arg_error("cell_width must be finite and >= 0");
    if (!std::isfinite(pts_per_cell)) return arg_error("pts_per_cell must be finite");
    pcms_status st = check_scale(inv_scale, dim);
    if (st != PCMS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    Grid *g = nullptr;
    st = grid_create(n_src, dim, inv_scale, false, &g);
    if (st != PCMS_OK) return st;
    st = build_grid_device(g, src, cell_width, pts_per_cell, s);
    if (st != PCMS_OK) {
        grid_alloc_free(g);
        return st;
    }
    *out = reinterpret_cast<pcms_grid *>(g);
    return PCMS_OK;
}

pcms_status pcms_lbvh_build(const double *src, int64_t n_src, int32_t dim, const double *inv_scale,
                            int32_t max_leaf, pcms_stream_t stream, pcms_grid **out)
{
    if (!out) return arg_error("out is NULL");
    *out = nullptr;
    if (dim < 1 || dim > kMaxDim) return arg_error("dim must be in [1, 5]");
    if (n_src < 1 || n_src >= ((int64_t)1 << 31) / 2) return arg_error("n_src must be in [1, 2^30)");
    if (!src) return arg_error("src is NULL");
    if (max_leaf < 0 || max_leaf > kBvhLeafMax) return arg_error("max_leaf must be in [0, 64]");
    pcms_status st = check_scale(inv_scale, dim);
    if (st != PCMS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    Grid *g = nullptr;
    if ((st = grid_create(n_src, dim, inv_scale, true, &g)) != PCMS_OK) return st;
    if ((st = build_lbvh_device(g, src, max_leaf > 0 ? max_leaf : lbvh_leaf_default(), s)) !=
        PCMS_OK) {
        (void)hipStreamSynchronize(s);
        grid_alloc_free(g);
        return st;
    }
    *out = reinterpret_cast<pcms_grid *>(g);
    return PCMS_OK;
}

int32_t pcms_grid_is_lbvh(const pcms_grid *grid)
{
    return grid && reinterpret_cast<const Grid *>(grid)->lbvh ? 1 : 0;
}

pcms_status pcms_grid_free(pcms_grid *grid)
{
    if (!grid) return PCMS_OK;
    Grid *g = reinterpret_cast<Grid *>(grid);
    (void)hipDeviceSynchronize();
    grid_alloc_free(g);
    return PCMS_OK;
}

pcms_status pcms_neighbors(const pcms_grid *grid, const double *tgt, int64_t n_tgt,
                           const pcms_radius *radius, int32_t k_cap, pcms_stream_t stream,
                           int32_t *nbr, int32_t *n_kept, int32_t *n_found, double *r2,
                           uint8_t *status)
{
    if (!grid) return arg_error("grid is NULL");
    const Grid *g = reinterpret_cast<const Grid *>(grid);
    if (n_tgt < 0 || n_tgt >= ((int64_t)1 << 31) / 2) return arg_error("n_tgt must be in [0, 2^30)");
    if (k_cap < 1 || k_cap > kMaxKcap) return arg_error("k_cap must be in [1, 256]");
    pcms_status st = check_radius(radius, g->n_src);
    if (st != PCMS_OK) return st;
    if (n_tgt > 0 && (!tgt || !nbr || !n_kept)) return arg_error("tgt, nbr and n_kept are required");
    if (n_tgt == 0) return PCMS_OK;
    hipStream_t s = (hipStream_t)stream;
    Scratch sc;
    sc.s = s;
    st = scratch_alloc(&sc.p, sizeof(int) * (size_t)n_tgt + 64, s);
    if (st != PCMS_OK) return st;
    int32_t *summary = (int32_t *)sc.p;
    int *tperm = (int *)((char *)sc.p + 64);
    if ((st = zero_ints(summary, 4, s)) != PCMS_OK) return st;
    if ((st = sort_targets(g, tgt, n_tgt, tperm, s)) != PCMS_OK) return st;
    LaunchSpec ls{g, tgt, tperm, n_tgt, *radius, k_cap, 0, summary};
    if ((st = launch_neighbors(ls, nbr, n_kept, n_found, r2, status, s)) != PCMS_OK) return st;
    return finish(summary, false, s, false);
}

pcms_status pcms_workspace_query(int64_t n_src, int32_t dim, int32_t n_fields, int64_t n_tgt,
                                 pcms_workspace *out)
{
    if (!out) return arg_error("out is NULL");
    if (dim < 1 || dim > kMaxDim) return arg_error("dim must be in [1, 5]");
    if (n_src < 1 || n_src >= ((int64_t)1 << 31) / 2) return arg_error("n_src must be in [1, 2^30)");
    if (n_tgt < 0 || n_tgt >= ((int64_t)1 << 31) / 2) return arg_error("n_tgt must be in [0, 2^30)");
    if (n_fields < 1) return arg_error("n_fields must be >= 1");
    const GridLayout G(n_src, dim), B(n_src, dim, true);
    const size_t build = grid_build_scratch_bytes(n_src);
    const size_t bbuild = lbvh_build_scratch_bytes(n_src);
    const size_t xfer = transfer_ws_bytes(n_src, n_fields, n_tgt);
    out->grid_bytes = G.bytes;
    out->grid_build_bytes = build;
    out->transfer_grid_bytes = xfer;
    // the one-shot call keeps its grid for the whole call, and takes the
    // transfer's workspace before the build's scratch is released (the
    // target order runs beside the build)
    out->transfer_bytes = std::max(G.bytes + build + xfer, B.bytes + bbuild + xfer);
    out->operator_apply_bytes = sizeof(double) * (size_t)n_src * padded_dim(n_fields);
    out->noalloc_limit = PCMS_NOALLOC_SCRATCH_BYTES;
    out->lbvh_bytes = B.bytes;
    out->lbvh_build_bytes = bbuild;
    return PCMS_OK;
}

pcms_status pcms_mls_transfer(const double *src, int64_t n_src, int32_t dim, const double *src_vals,
                              int32_t n_fields, const double *tgt, int64_t n_tgt,
                              int32_t basis_degree, const pcms_radius *radius, int32_t k_cap,
                              const double *inv_scale, const pcms_mls_opts *opts,
                              pcms_stream_t stream, double *tgt_vals, uint8_t *status)
{
    if (n_src < 1 || n_src >= ((int64_t)1 << 31) / 2) return arg_error("n_src must be in [1, 2^30)");
    if (!src) return arg_error("src is NULL");
    pcms_status st = check_transfer_args(n_src, dim, src_vals, n_fields, tgt, n_tgt, basis_degree,
                                         radius, k_cap, opts, tgt_vals);
    if (st != PCMS_OK) return st;
    if ((st = check_scale(inv_scale, dim)) != PCMS_OK) return st;
    if (n_tgt == 0) return PCMS_OK;
    hipStream_t s = (hipStream_t)stream;
    if ((st = profile_begin(opts, s)) != PCMS_OK) return st;
    double cw, ppc;
    cell_spec(radius, dim, &cw, &ppc);
    const bool lbvh = opts && (opts->flags & PCMS_LBVH);
    // one-shot grid (or LBVH) in stream-ordered scratch
    Grid g{};
    g.dim = dim;
    g.n_src = n_src;
    for (int k = 0; k < kMaxDim; ++k) g.g[k] = (inv_scale && k < dim) ? inv_scale[k] : 1.0;
    PCMS_HIP(hipGetDevice(&g.device));
    Scratch sc, xs;
    sc.s = xs.s = s;
    const GridLayout L(n_src, dim, lbvh);
    if ((st = scratch_alloc(&sc.p, L.bytes, s)) != PCMS_OK) return st;
    L.place(g, sc.p, lbvh);
    // unprofiled calls order the targets on the side stream from the point
    // where the grid's parameters exist, overlapping the rest of the build
    // and the field gather (profiled calls run the phases in line, to time
    // them).  The fork point is marked there, but the side work is enqueued
    // after the build's, so the build's kernels are not held up behind the
    // host's launches of the sort.
    hipEvent_t ordered = nullptr;
    std::function<pcms_status()> fork = [&]() { return side_fork(s); };
    if (!g_prof.on) {
        if ((st = scratch_alloc(&xs.p, transfer_ws_bytes(n_src, n_fields, n_tgt), s)) != PCMS_OK)
            return st;
    }
    const std::function<pcms_status()> *hook = g_prof.on ? nullptr : &fork;
    st = lbvh ? build_lbvh_device(&g, src, lbvh_leaf_default(), s, hook)
              : build_grid_device(&g, src, cw, ppc, s, hook);
    if (st != PCMS_OK) return st;
    if (!g_prof.on) {
        int *tperm;
        void *sort_ws;
        transfer_ws_order(xs.p, n_src, n_fields, n_tgt, &tperm, &sort_ws);
        if ((st = order_targets_aside(&g, tgt, n_tgt, tperm, sort_ws, s, &ordered, false)) != PCMS_OK)
            return st;
    }
    return transfer_on_grid(&g, src_vals, n_fields, tgt, n_tgt, basis_degree, radius, k_cap, opts,
                            s, tgt_vals, status, xs.p, !g_prof.on, ordered);
}

pcms_status pcms_mls_transfer_grid(const pcms_grid *grid, const double *src_vals, int32_t n_fields,
                                   const double *tgt, int64_t n_tgt, int32_t basis_degree,
                                   const pcms_radius *radius, int32_t k_cap,
                                   const pcms_mls_opts *opts, pcms_stream_t stream,
                                   double *tgt_vals, uint8_t *status)
{
    if (!grid) return arg_error("grid is NULL");
    const Grid *g = reinterpret_cast<const Grid *>(grid);
    pcms_status st = check_transfer_args(g->n_src, g->dim, src_vals, n_fields, tgt, n_tgt,
                                         basis_degree, radius, k_cap, opts, tgt_vals);
    if (st != PCMS_OK) return st;
    if (n_tgt == 0) return PCMS_OK;
    if ((st = profile_begin(opts, (hipStream_t)stream)) != PCMS_OK) return st;
    if ((st = g_prof.mark(1)) != PCMS_OK) return st;   // no grid build in this call
    return transfer_on_grid(g, src_vals, n_fields, tgt, n_tgt, basis_degree, radius, k_cap, opts,
                            (hipStream_t)stream, tgt_vals, status, nullptr, !g_prof.on);
}

pcms_status pcms_operator_build(const double *src, int64_t n_src, int32_t dim, const double *tgt,
                                int64_t n_tgt, int32_t basis_degree, const pcms_radius *radius,
                                int32_t k_cap, const double *inv_scale, const pcms_mls_opts *opts,
                                pcms_stream_t stream, uint8_t *status, pcms_operator **out)
{
    if (!out) return arg_error("out is NULL");
    *out = nullptr;
    if (n_src < 1 || n_src >= ((int64_t)1 << 31) / 2) return arg_error("n_src must be in [1, 2^30)");
    if (!src) return arg_error("src is NULL");
    // the operator needs no field values: validate as a one-field transfer
    double *fake = const_cast<double *>(src);   // only checked for NULL
    pcms_status st = check_transfer_args(n_src, dim, fake, 1, tgt, n_tgt, basis_degree, radius, k_cap,
                                         opts, fake);
    if (st != PCMS_OK) return st;
    if (n_tgt > 0 && !tgt) return arg_error("tgt is required");
    if ((st = check_scale(inv_scale, dim)) != PCMS_OK) return st;
    pcms_mls_opts o;
    pcms_mls_opts_default(&o);
    if (opts) o = *opts;
    const bool async = (o.flags & PCMS_ASYNC) != 0;
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<Operator> op(new (std::nothrow) Operator());
    if (!op) return PCMS_ERR_NOMEM;
    op->n_src = n_src;
    op->n_tgt = n_tgt;
    // one-shot grid (or LBVH) in stream-ordered scratch
    double cw, ppc;
    cell_spec(radius, dim, &cw, &ppc);
    const bool lbvh = (o.flags & PCMS_LBVH) != 0;
    Grid g{};
    g.dim = dim;
    g.n_src = n_src;
    g.n_cells_cap = lbvh ? 1 : cells_cap_for(n_src);
    for (int k = 0; k < kMaxDim; ++k) g.g[k] = (inv_scale && k < dim) ? inv_scale[k] : 1.0;
    PCMS_HIP(hipGetDevice(&g.device));
    LaunchSpec ls{&g, tgt, nullptr, n_tgt, *radius, k_cap, o.block, nullptr};
    op->width = operator_width(ls);
    const size_t nt = (size_t)std::max<int64_t>(n_tgt, 1);
    const size_t o_opp = 256 + ((sizeof(int) * nt + 255) & ~(size_t)255);
    const size_t o_opi = o_opp + ((sizeof(int) * (size_t)n_src + 255) & ~(size_t)255);
    const size_t o_n = o_opi + ((sizeof(int) * (size_t)n_src + 255) & ~(size_t)255);
    const size_t o_c = o_n + ((sizeof(int32_t) * nt + 255) & ~(size_t)255);
    const size_t o_w = o_c + ((sizeof(int32_t) * nt * op->width + 255) & ~(size_t)255);
    const size_t bytes = o_w + sizeof(double) * nt * op->width;
    hipError_t he = hipMalloc(&op->mem, bytes);
    if (he != hipSuccess) return hip_fail(he, "hipMalloc(operator)");
    op->tperm = (int *)((char *)op->mem + 256);
    op->perm = (int *)((char *)op->mem + o_opp);
    op->iperm = (int *)((char *)op->mem + o_opi);
    op->op_n = (int32_t *)((char *)op->mem + o_n);
    op->op_c = (int32_t *)((char *)op->mem + o_c);
    op->op_w = (double *)((char *)op->mem + o_w);
    auto fail = [&](pcms_status e) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(op->mem);
        return e;
    };
    Scratch sc;
    sc.s = s;
    const GridLayout L(n_src, dim, lbvh);
    const size_t o_sum = align256(L.bytes);
    if ((st = scratch_alloc(&sc.p, o_sum + 64, s)) != PCMS_OK) return fail(st);
    L.place(g, sc.p, lbvh);
    int32_t *summary = async ? o.summary : (int32_t *)((char *)sc.p + o_sum);
    if ((st = zero_ints(summary, 4, s)) != PCMS_OK) return fail(st);
    st = lbvh ? build_lbvh_device(&g, src, lbvh_leaf_default(), s)
              : build_grid_device(&g, src, cw, ppc, s);
    if (st != PCMS_OK) return fail(st);
    he = hipMemcpyAsync(op->perm, g.perm, sizeof(int) * (size_t)n_src, hipMemcpyDeviceToDevice, s);
    if (he == hipSuccess)
        he = hipMemcpyAsync(op->iperm, g.iperm, sizeof(int) * (size_t)n_src, hipMemcpyDeviceToDevice, s);
    if (he != hipSuccess) return fail(hip_fail(he, "hipMemcpyAsync(operator permutation)"));
    if (n_tgt > 0) {
        if ((st = sort_targets(&g, tgt, n_tgt, op->tperm, s)) != PCMS_OK) return fail(st);
        ls.tperm = op->tperm;
        ls.summary = summary;
        if ((st = launch_operator(ls, basis_degree, o.weight, o.precision, o.lambda, op->op_w,
                                  op->op_c, op->op_n, status, s)) != PCMS_OK)
            return fail(st);
    }
    st = finish(summary, async, s, true);
    if (st != PCMS_OK && st != PCMS_ERR_UNDERDETERMINED && st != PCMS_ERR_SINGULAR &&
        st != PCMS_ERR_RADIUS_EXHAUSTED)
        return fail(st);
    *out = reinterpret_cast<pcms_operator *>(op.release());
    return st;
}

pcms_status pcms_operator_apply(const pcms_operator *op, const double *src_vals, int32_t n_fields,
                                pcms_stream_t stream, double *tgt_vals)
{
    if (!op) return arg_error("operator is NULL");
    const Operator &o = *reinterpret_cast<const Operator *>(op);
    if (n_fields < 1) return arg_error("n_fields must be >= 1");
    if (o.n_tgt > 0 && (!src_vals || !tgt_vals)) return arg_error("src_vals and tgt_vals are required");
    return operator_apply(o, src_vals, n_fields, tgt_vals, (hipStream_t)stream);
}

pcms_status pcms_operator_export(const pcms_operator *op, int32_t stride, pcms_stream_t stream,
                                 int32_t *n_kept, int32_t *cols, double *weights)
{
    if (!op) return arg_error("operator is NULL");
    const Operator &o = *reinterpret_cast<const Operator *>(op);
    if (stride < 1 || stride < o.width)
        return arg_error("stride must be >= pcms_operator_width(op) (" + std::to_string(o.width) + ")");
    if (o.n_tgt > 0 && !n_kept) return arg_error("n_kept is required");
    return operator_export(o, stride, n_kept, cols, weights, (hipStream_t)stream);
}

int32_t pcms_operator_width(const pcms_operator *op)
{
    return op ? reinterpret_cast<const Operator *>(op)->width : 0;
}

pcms_status pcms_operator_free(pcms_operator *op)
{
    if (!op) return PCMS_OK;
    Operator *o = reinterpret_cast<Operator *>(op);
    (void)hipDeviceSynchronize();
    if (o->mem) (void)hipFree(o->mem);
    delete o;
    return PCMS_OK;
}

void pcms_batch_opts_default(pcms_batch_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->weight = PCMS_WEIGHT_WENDLAND_C2;
    o->precision = PCMS_MIXED_REFINE;
}

pcms_status pcms_batch_plan_create(const pcms_problem *problems, int32_t n,
                                   const pcms_batch_opts *opts, pcms_batch_plan **out)
{
    if (!out) return arg_error("out is NULL");
    *out = nullptr;
    if (n < 1 || !problems) return arg_error("a batch needs n >= 1 problems");
    pcms_batch_opts o;
    pcms_batch_opts_default(&o);
    if (opts) o = *opts;
    pcms_mls_opts mo;
    pcms_mls_opts_default(&mo);
    mo.weight = o.weight;
    mo.precision = o.precision;
    mo.lambda = o.lambda;
    pcms_status st = check_opts(&mo);
    if (st != PCMS_OK) return st;
    if (o.block != 0 && o.block != 64 && o.block != 128 && o.block != 256)
        return arg_error("block must be 0, 64, 128 or 256");
    if (!(o.cell_factor >= 0.0 && o.cell_factor <= 4.0)) return arg_error("cell_factor must be 0 or in (0, 4]");
    int block = o.block;
    double cf = o.cell_factor;
    if ((block == 0 || cf == 0.0) && o.tune_cache) {
        int tb = 0;
        double tcf = 0.0;
        if (read_tune_cache(o.tune_cache, &tb, &tcf)) {
            if (block == 0) block = tb;
            if (cf == 0.0) cf = tcf;
        }
    }
    if (block == 0) block = 256;
    std::unique_ptr<BatchPlan> p(new (std::nothrow) BatchPlan());
    if (!p) return PCMS_ERR_NOMEM;
    p->n = n;
    p->weight = o.weight;
    p->precision = o.precision;
    p->lambda = o.lambda;
    p->block = block;
    p->cell_factor = cf;
    p->hp.assign(n, BatchProb{});
    for (int q = 0; q < n; ++q) {
        const pcms_problem &P = problems[q];
        const std::string at = "problem " + std::to_string(q) + ": ";
        if (P.n_src < 1 || P.n_src >= ((int64_t)1 << 31) / 2) return arg_error(at + "n_src must be in [1, 2^30)");
        if (!P.src) return arg_error(at + "src is NULL");
        st = check_transfer_args(P.n_src, P.dim, P.src_vals, P.n_fields, P.tgt, P.n_tgt, P.basis_degree,
                                 &P.radius, P.k_cap, &mo, P.tgt_vals);
        if (st != PCMS_OK) return arg_error(at + pcms_last_error());
        if ((st = check_scale(P.inv_scale, P.dim)) != PCMS_OK) return arg_error(at + pcms_last_error());
        BatchProb &B = p->hp[q];
        B.src = P.src;
        B.vals = P.src_vals;
        B.tgt = P.tgt;
        B.out = P.tgt_vals;
        B.status = P.status;
        B.n_src = (int)P.n_src;
        B.n_tgt = (int)P.n_tgt;
        B.dim = P.dim;
        B.degree = P.basis_degree;
        B.nf = P.n_fields;
        B.nfs = padded_dim(P.n_fields);
        B.k_cap = P.k_cap;
        B.words = target_words(P.radius.mode, P.radius.k, P.k_cap);
        B.stride = B.words | 1;
        B.mode = P.radius.mode;
        B.k = P.radius.k;
        B.n_min = P.radius.n_min;
        B.max_iter = P.radius.max_iter;
        B.r = P.radius.r;
        B.cells_cap = cells_cap_for(P.n_src);
        B.unit = 1;
        for (int k = 0; k < kMaxDim; ++k) {
            B.g[k] = (P.inv_scale && k < P.dim) ? P.inv_scale[k] : 1.0;
            if (B.g[k] != 1.0) B.unit = 0;
        }
        cell_spec(&P.radius, P.dim, &B.cell_width, &B.pts_per_cell, cf);
    }
    // the per-target LDS of one block must fit a workgroup
    int max_stride = 1;
    for (const BatchProb &B : p->hp) max_stride = std::max(max_stride, B.stride);
    while (p->block > 64 && (size_t)p->block * max_stride * sizeof(int) > 65536) p->block >>= 1;
    if ((st = batch_setup(*p)) != PCMS_OK) return st;
    *out = reinterpret_cast<pcms_batch_plan *>(p.release());
    return PCMS_OK;
}

pcms_status pcms_batch_plan_exec(pcms_batch_plan *plan, pcms_stream_t stream, int32_t *summary)
{
    if (!plan) return arg_error("plan is NULL");
    BatchPlan &p = *reinterpret_cast<BatchPlan *>(plan);
    hipStream_t s = (hipStream_t)stream;
    pcms_status st;
    if (!s) {
        // the legacy null stream cannot be captured: plain enqueue
        if ((st = batch_enqueue(p, s)) != PCMS_OK) return st;
    } else {
        if (!p.exec) {
            PCMS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            st = batch_enqueue(p, s);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(s, &g);
            if (st != PCMS_OK) {
                if (e == hipSuccess && g) (void)hipGraphDestroy(g);
                return st;
            }
            PCMS_HIP(e);
            e = hipGraphInstantiate(&p.exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(g);
                p.exec = nullptr;
                return hip_fail(e, "hipGraphInstantiate");
            }
            p.graph = g;
        }
        PCMS_HIP(hipGraphLaunch(p.exec, s));
    }
    if (summary) return batch_copy_summary(p.summary, summary, s);
    return finish(p.summary, false, s, true);
}

pcms_status pcms_batch_plan_free(pcms_batch_plan *plan)
{
    if (!plan) return PCMS_OK;
    BatchPlan *p = reinterpret_cast<BatchPlan *>(plan);
    (void)hipDeviceSynchronize();
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->ws) (void)hipFree(p->ws);
    delete p;
    return PCMS_OK;
}

pcms_status pcms_autotune(const pcms_problem *sample, int32_t n, const pcms_batch_opts *opts,
                          const char *cache_path, pcms_stream_t stream, pcms_tune_result *out)
{
    if (!out) return arg_error("out is NULL");
    pcms_batch_opts o;
    pcms_batch_opts_default(&o);
    if (opts) o = *opts;
    o.tune_cache = nullptr;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PCMS_HIP(hipEventCreate(&e0));
    PCMS_HIP(hipEventCreate(&e1));
    const int blocks[3] = {64, 128, 256};
    const double cfs[4] = {0.6, 0.7, 0.85, 1.0};
    pcms_tune_result best{0, 0.0, INFINITY};
    pcms_status st = PCMS_OK;
    int32_t *sum = nullptr;
    hipError_t he = hipMalloc(&sum, sizeof(int32_t) * 4);
    if (he != hipSuccess) st = hip_fail(he, "hipMalloc(summary)");
    for (int bi = 0; bi < 3 && st == PCMS_OK; ++bi) {
        for (int ci = 0; ci < 4 && st == PCMS_OK; ++ci) {
            o.block = blocks[bi];
            o.cell_factor = cfs[ci];
            pcms_batch_plan *plan = nullptr;
            if ((st = pcms_batch_plan_create(sample, n, &o, &plan)) != PCMS_OK) break;
            // first execution captures the graph; then three timed replays
            st = pcms_batch_plan_exec(plan, stream, sum);
            float ms = 0.0f;
            if (st == PCMS_OK && hipEventRecord(e0, s) == hipSuccess) {
                for (int r = 0; r < 3 && st == PCMS_OK; ++r) st = pcms_batch_plan_exec(plan, stream, sum);
                if (st == PCMS_OK && (hipEventRecord(e1, s) != hipSuccess ||
                                      hipEventSynchronize(e1) != hipSuccess ||
                                      hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    st = hip_fail(hipGetLastError(), "autotune timing");
            }
            pcms_batch_plan_free(plan);
            ms /= 3.0f;
            if (st == PCMS_OK && ms < best.ms) best = pcms_tune_result{blocks[bi], cfs[ci], ms};
        }
    }
    if (sum) (void)hipFree(sum);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != PCMS_OK) return st;
    *out = best;
    if (cache_path) {
        FILE *f = std::fopen(cache_path, "w");
        if (!f) {
            set_error(std::string("cannot write ") + cache_path);
            return PCMS_ERR_ARG;
        }
        std::fprintf(f, "{\"block\": %d, \"cell_factor\": %.17g, \"ms\": %.6g}\n", best.block,
                     best.cell_factor, (double)best.ms);
        std::fclose(f);
    }
    return PCMS_OK;
}

}  // extern "C"
