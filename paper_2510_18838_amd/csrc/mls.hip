// Neighbour-list and field-transfer kernels: one lane per target, targets in
// tiled Morton order so that the lanes of a wave search overlapping stencils.  The
// per-target work (search, moment assembly, Cholesky, evaluation) is in
// fit.h / search.h; this file holds the kernels and their launchers.
#include <hip/hip_runtime.h>
#include <math.h>

#include "fit.h"
#include "internal.h"
#include "launch_common.h"

namespace pcms {

namespace {

// Lanes per target (G consecutive lanes of a wave); the block's targets are
// consecutive in processing order and each owns `stride` LDS words.
#ifndef PCMS_LANES_PER_TARGET
#define PCMS_LANES_PER_TARGET 1
#endif
constexpr int kGroup = PCMS_LANES_PER_TARGET;

template <int D, bool UNIT, int G>
__global__ void __launch_bounds__(256) k_neighbors(KArgs a)
{
    extern __shared__ int lds[];
    const int lb = logical_block(a.n_blocks);
    if (lb >= a.n_blocks) return;
    const int slot = (int)threadIdx.x / G;
    const int i = lb * ((int)blockDim.x / G) + slot;
    const bool active = i < a.n_tgt;   // uniform within a group
    const Grp<G> g{(int)(threadIdx.x & (G - 1))};
    int st = 0;
    if (active) {
        const GridParams gp = *a.gp;
        st = nbr_target<D, UNIT, G>(a, gp, i, lds + slot * a.stride, g);
    }
    add_summary(a.summary, st, active && g.q == 0);
}

// Three waves per SIMD: the register allocator fits 168 VGPRs (the fit's
// moment and factor arrays spill a little around the refinement pass), which
// measured faster than two waves without spills.
template <int D, int P, bool MIXED, bool UNIT, int G>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_transfer(KArgs a)
{
    extern __shared__ int lds[];
    const int lb = logical_block(a.n_blocks);
    if (lb >= a.n_blocks) return;
    const int slot = (int)threadIdx.x / G;
    const int i = lb * ((int)blockDim.x / G) + slot;
    const bool active = i < a.n_tgt;   // uniform within a group
    const Grp<G> g{(int)(threadIdx.x & (G - 1))};
    int st = 0;
    if (active) {
        const GridParams gp = *a.gp;
        st = xfer_target<D, P, MIXED, UNIT, G>(a, gp, i, lds + slot * a.stride, g);
    }
    add_summary(a.summary, st, active && g.q == 0);
}

__global__ void k_zero_ints(int32_t *p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

using KernelFn = void (*)(KArgs);

template <int D, bool UNIT>
KernelFn pick_nbr()
{
    return k_neighbors<D, UNIT, kGroup>;
}

template <int D, int P, bool UNIT>
KernelFn pick_xfer(bool mixed)
{
    return mixed ? (KernelFn)k_transfer<D, P, true, UNIT, kGroup>
                 : (KernelFn)k_transfer<D, P, false, UNIT, kGroup>;
}

template <bool UNIT>
KernelFn xfer_table(int d, int p, bool mixed)
{
#define PCMS_CASE(DD)                                               \
    case DD:                                                        \
        return p == 0 ? pick_xfer<DD, 0, UNIT>(mixed)               \
             : p == 1 ? pick_xfer<DD, 1, UNIT>(mixed)               \
                      : pick_xfer<DD, 2, UNIT>(mixed);
    switch (d) {
        PCMS_CASE(1)
        PCMS_CASE(2)
        PCMS_CASE(3)
        PCMS_CASE(4)
        PCMS_CASE(5)
    }
#undef PCMS_CASE
    return nullptr;
}

template <bool UNIT>
KernelFn nbr_table(int d)
{
    switch (d) {
    case 1: return pick_nbr<1, UNIT>();
    case 2: return pick_nbr<2, UNIT>();
    case 3: return pick_nbr<3, UNIT>();
    case 4: return pick_nbr<4, UNIT>();
    case 5: return pick_nbr<5, UNIT>();
    }
    return nullptr;
}

bool unit_metric(const Grid *g)
{
    for (int k = 0; k < g->dim; ++k)
        if (g->g[k] != 1.0) return false;
    return true;
}

// LDS words of a target (target_words); the per-target stride is odd so
// neighbouring targets start in different banks.
int lane_words(const LaunchSpec &ls) { return target_words(ls.radius.mode, ls.radius.k, ls.k_cap); }
int target_stride(const LaunchSpec &ls) { return lane_words(ls) | 1; }

// Threads per block (kGroup lanes per target); the targets' LDS must fit
// 64 KiB per workgroup.
int pick_block(int requested, const LaunchSpec &ls)
{
    int b = requested > 0 ? requested : 256;
    while (b > 64 && (size_t)(b / kGroup) * target_stride(ls) * sizeof(int) > 65536) b >>= 1;
    return b;
}

KArgs base_args(const LaunchSpec &ls, int block)
{
    KArgs a{};
    a.gp = ls.grid->params;
    a.cs = ls.grid->cell_start;
    a.spts = ls.grid->spts;
    a.perm = ls.grid->perm;
    a.tgt = ls.tgt;
    a.tperm = ls.tperm;
    a.n_tgt = (int)ls.n_tgt;
    a.mode = ls.radius.mode;
    a.k = ls.radius.k;
    a.n_min = ls.radius.n_min;
    a.max_iter = ls.radius.max_iter;
    a.r = ls.radius.r;
    a.k_cap = ls.k_cap;
    const int tpb = block / kGroup;
    a.n_blocks = (int)((ls.n_tgt + tpb - 1) / tpb);
    a.words = lane_words(ls);
    a.stride = target_stride(ls);
    a.summary = ls.summary;
    return a;
}

}  // namespace

pcms_status zero_ints(int32_t *p, int n, hipStream_t s)
{
    k_zero_ints<<<(n + 255) / 256, 256, 0, s>>>(p, n);
    PCMS_HIP(hipGetLastError());
    return PCMS_OK;
}

pcms_status launch_neighbors(const LaunchSpec &ls, int32_t *nbr, int32_t *n_kept,
                             int32_t *n_found, double *r2, uint8_t *status, hipStream_t s)
{
    if (ls.n_tgt == 0) return PCMS_OK;
    const int block = pick_block(ls.block, ls);
    KArgs a = base_args(ls, block);
    a.nbr = nbr;
    a.n_kept = n_kept;
    a.n_found = n_found;
    a.r2 = r2;
    a.status = status;
    KernelFn fn = unit_metric(ls.grid) ? nbr_table<true>(ls.grid->dim) : nbr_table<false>(ls.grid->dim);
    const int launch = ((a.n_blocks + 7) / 8) * 8;
    const size_t shm = (size_t)(block / kGroup) * target_stride(ls) * sizeof(int);
    hipLaunchKernelGGL(fn, dim3(launch), dim3(block), shm, s, a);
    PCMS_HIP(hipGetLastError());
    return PCMS_OK;
}

pcms_status launch_transfer(const LaunchSpec &ls, const double *svals, int n_fields, int degree,
                            int weight, int precision, double lambda, double *out,
                            uint8_t *status, hipStream_t s)
{
    if (ls.n_tgt == 0) return PCMS_OK;
    const int block = pick_block(ls.block, ls);
    KArgs a = base_args(ls, block);
    a.svals = svals;
    a.nf = n_fields;
    a.nfs = padded_dim(n_fields);
    a.weight = weight;
    a.refine = precision == PCMS_MIXED_REFINE;
    a.lambda = lambda;
    a.out = out;
    a.status = status;
    const bool mixed = precision != PCMS_FP64;
    KernelFn fn = unit_metric(ls.grid) ? xfer_table<true>(ls.grid->dim, degree, mixed)
                                       : xfer_table<false>(ls.grid->dim, degree, mixed);
    const int launch = ((a.n_blocks + 7) / 8) * 8;
    const size_t shm = (size_t)(block / kGroup) * target_stride(ls) * sizeof(int);
    hipLaunchKernelGGL(fn, dim3(launch), dim3(block), shm, s, a);
    PCMS_HIP(hipGetLastError());
    return PCMS_OK;
}

}  // namespace pcms
