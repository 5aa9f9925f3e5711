// Launchers of the one-problem neighbour-list and field-transfer kernels
// (kernels.h): LDS sizing, block choice, XCD-aware grid, variant dispatch.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "internal.h"
#include "kernels.h"

namespace pcms {

namespace {

__global__ void k_zero_ints(int32_t *p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

KernelFn xfer_for(int d, int p, int precision, bool unit, bool bvh)
{
    if (bvh) {
        switch (d) {
        case 1: return transfer_kernel_bvh<1>(p, precision, unit);
        case 2: return transfer_kernel_bvh<2>(p, precision, unit);
        case 3: return transfer_kernel_bvh<3>(p, precision, unit);
        case 4: return transfer_kernel_bvh<4>(p, precision, unit);
        case 5: return transfer_kernel_bvh<5>(p, precision, unit);
        }
        return nullptr;
    }
    switch (d) {
    case 1: return transfer_kernel<1>(p, precision, unit);
    case 2: return transfer_kernel<2>(p, precision, unit);
    case 3: return transfer_kernel<3>(p, precision, unit);
    case 4: return transfer_kernel<4>(p, precision, unit);
    case 5: return transfer_kernel<5>(p, precision, unit);
    }
    return nullptr;
}

KernelFn op_for(int d, int p, int precision, bool unit, bool bvh)
{
    if (bvh) {
        switch (d) {
        case 1: return operator_kernel_bvh<1>(p, precision, unit);
        case 2: return operator_kernel_bvh<2>(p, precision, unit);
        case 3: return operator_kernel_bvh<3>(p, precision, unit);
        case 4: return operator_kernel_bvh<4>(p, precision, unit);
        case 5: return operator_kernel_bvh<5>(p, precision, unit);
        }
        return nullptr;
    }
    switch (d) {
    case 1: return operator_kernel<1>(p, precision, unit);
    case 2: return operator_kernel<2>(p, precision, unit);
    case 3: return operator_kernel<3>(p, precision, unit);
    case 4: return operator_kernel<4>(p, precision, unit);
    case 5: return operator_kernel<5>(p, precision, unit);
    }
    return nullptr;
}

KernelFn nbr_for(int d, bool unit, bool bvh)
{
    if (bvh) {
        switch (d) {
        case 1: return nbr_kernel_bvh<1>(unit);
        case 2: return nbr_kernel_bvh<2>(unit);
        case 3: return nbr_kernel_bvh<3>(unit);
        case 4: return nbr_kernel_bvh<4>(unit);
        case 5: return nbr_kernel_bvh<5>(unit);
        }
        return nullptr;
    }
    switch (d) {
    case 1: return nbr_kernel<1>(unit);
    case 2: return nbr_kernel<2>(unit);
    case 3: return nbr_kernel<3>(unit);
    case 4: return nbr_kernel<4>(unit);
    case 5: return nbr_kernel<5>(unit);
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
    a.spts32 = ls.grid->spts32;
    a.sq = ls.grid->sq;
    a.bvh_nodes = ls.grid->bvh_nodes;
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
    KernelFn fn = nbr_for(ls.grid->dim, unit_metric(ls.grid), ls.grid->lbvh != 0);
    const int launch = ((a.n_blocks + 7) / 8) * 8;
    const size_t shm = (size_t)(block / kGroup) * target_stride(ls) * sizeof(int);
    hipLaunchKernelGGL(fn, dim3(launch), dim3(block), shm, s, a);
    PCMS_HIP(hipGetLastError());
    return PCMS_OK;
}

pcms_status launch_transfer(const LaunchSpec &ls, const double *svals, int n_fields, int degree,
                            int weight, int precision, double lambda, double *out,
                            double *stage, uint8_t *status, hipStream_t s)
{
    if (ls.n_tgt == 0) return PCMS_OK;
    const int block = pick_block(ls.block, ls);
    KArgs a = base_args(ls, block);
    a.svals = svals;
    a.nf = n_fields;
    a.nfs = padded_dim(n_fields);
    a.weight = weight;
    a.lambda = lambda;
    a.out = out;
    a.stage = stage;
    a.status = status;
    KernelFn fn = xfer_for(ls.grid->dim, degree, precision, unit_metric(ls.grid),
                           ls.grid->lbvh != 0);
    const int launch = ((a.n_blocks + 7) / 8) * 8;
    const size_t shm = (size_t)(block / kGroup) * target_stride(ls) * sizeof(int);
    hipLaunchKernelGGL(fn, dim3(launch), dim3(block), shm, s, a);
    PCMS_HIP(hipGetLastError());
    return PCMS_OK;
}

pcms_status launch_operator(const LaunchSpec &ls, int degree, int weight, int precision,
                            double lambda, double *op_w, int32_t *op_c, int32_t *op_n,
                            uint8_t *status, hipStream_t s)
{
    if (ls.n_tgt == 0) return PCMS_OK;
    const int block = pick_block(ls.block, ls);
    KArgs a = base_args(ls, block);
    a.weight = weight;
    a.lambda = lambda;
    a.op_w = op_w;
    a.op_c = op_c;
    a.op_n = op_n;
    a.status = status;
    KernelFn fn = op_for(ls.grid->dim, degree, precision, unit_metric(ls.grid),
                         ls.grid->lbvh != 0);
    const int launch = ((a.n_blocks + 7) / 8) * 8;
    const size_t shm = (size_t)(block / kGroup) * target_stride(ls) * sizeof(int);
    hipLaunchKernelGGL(fn, dim3(launch), dim3(block), shm, s, a);
    PCMS_HIP(hipGetLastError());
    return PCMS_OK;
}

// Slots per target of an operator: every kept list fits its LDS words and
// holds at most k_cap entries.
int operator_width(const LaunchSpec &ls) { return std::min(lane_words(ls), ls.k_cap); }

}  // namespace pcms
