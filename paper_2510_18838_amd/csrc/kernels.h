// The one-problem neighbour-list and field-transfer kernels (one lane per
// target, targets in tiled Morton order so that the lanes of a wave search
// overlapping stencils), instantiated per dimension in mls_d1.hip ..
// mls_d5.hip so that the variants compile in parallel.  The per-target work
// (search, moment assembly, Cholesky, evaluation) is in fit.h / search.h.
#pragma once

#include <hip/hip_runtime.h>

#include "fit.h"
#include "launch_common.h"

namespace pcms {

// Lanes per target (G consecutive lanes of a wave); the block's targets are
// consecutive in processing order and each owns `stride` LDS words.
#ifndef PCMS_LANES_PER_TARGET
#define PCMS_LANES_PER_TARGET 1
#endif
constexpr int kGroup = PCMS_LANES_PER_TARGET;

using KernelFn = void (*)(KArgs);

// Kernel of dimension D for (degree, precision, unit metric); defined in
// mls_d<D>.hip, and the same on an LBVH in bvh_d<D>.hip.
template <int D>
KernelFn transfer_kernel(int degree, int precision, bool unit);
template <int D>
KernelFn nbr_kernel(bool unit);
template <int D>
KernelFn transfer_kernel_bvh(int degree, int precision, bool unit);
template <int D>
KernelFn nbr_kernel_bvh(bool unit);
// The operator-emission variant of transfer_kernel; defined in op_d<D>.hip,
// and on an LBVH in bvh_op_d<D>.hip.
template <int D>
KernelFn operator_kernel(int degree, int precision, bool unit);
template <int D>
KernelFn operator_kernel_bvh(int degree, int precision, bool unit);

namespace {

template <int D, bool UNIT, int G, bool BVH = false>
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
        st = nbr_target<D, UNIT, G, BVH>(a, gp, i, lds + slot * a.stride, g);
    }
    add_summary(a.summary, st, active && g.q == 0);
}

// Waves per SIMD the register allocator targets (168 VGPRs for 3, 256 for
// 2): three, except for MIXED_REFINE in 4-D and 5-D (240-1100 bytes of
// spill per lane under 168 VGPRs) and the 4-D and 5-D quadratic bases in
// any precision (1-2 KB), which get two.  Measured: the 5-D linear
// MIXED_REFINE kernel went from 3-6 % slower than FP64 to level with it
// (74.3 against 76.1 ms, means of three runs).  The low-dimensional
// kernels need the third wave for latency even where they spill a little:
// at two, the 3-D quadratic MIXED_REFINE kernel (52 bytes of spill) slows
// from 7.0 to 9.2 ms and the 2-D quadratic one (132 bytes) from 0.43 to
// 0.48 ms.
template <int PREC, int D, int P>
constexpr int waves_for()
{
    return D >= 4 && (PREC == PCMS_MIXED_REFINE || P == 2) ? 2 : 3;
}

template <int D, int P, int PREC, bool UNIT, int G, bool BVH = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(waves_for<PREC, D, P>())))
k_transfer(KArgs a)
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
        st = xfer_target<D, P, PREC, UNIT, G, false, BVH>(a, gp, i, lds + slot * a.stride, g);
    }
    add_summary(a.summary, st, active && g.q == 0);
}

// The same kernel writing the transfer operator instead of field values.
template <int D, int P, int PREC, bool UNIT, int G, bool BVH = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(waves_for<PREC, D, P>())))
k_operator(KArgs a)
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
        st = xfer_target<D, P, PREC, UNIT, G, true, BVH>(a, gp, i, lds + slot * a.stride, g);
    }
    add_summary(a.summary, st, active && g.q == 0);
}

template <int D, int P, bool UNIT, bool BVH = false>
KernelFn pick_prec(int precision)
{
    return precision == PCMS_FP64  ? (KernelFn)k_transfer<D, P, PCMS_FP64, UNIT, kGroup, BVH>
         : precision == PCMS_MIXED ? (KernelFn)k_transfer<D, P, PCMS_MIXED, UNIT, kGroup, BVH>
                                   : (KernelFn)k_transfer<D, P, PCMS_MIXED_REFINE, UNIT, kGroup, BVH>;
}

template <int D, int P, bool UNIT, bool BVH = false>
KernelFn pick_prec_op(int precision)
{
    return precision == PCMS_FP64  ? (KernelFn)k_operator<D, P, PCMS_FP64, UNIT, kGroup, BVH>
         : precision == PCMS_MIXED ? (KernelFn)k_operator<D, P, PCMS_MIXED, UNIT, kGroup, BVH>
                                   : (KernelFn)k_operator<D, P, PCMS_MIXED_REFINE, UNIT, kGroup, BVH>;
}

}  // namespace

// Body of the per-dimension definitions.
#define PCMS_DEFINE_DIM_KERNELS(DD)                                                    \
    template <>                                                                        \
    KernelFn transfer_kernel<DD>(int degree, int precision, bool unit)                 \
    {                                                                                  \
        if (unit)                                                                      \
            return degree == 0 ? pick_prec<DD, 0, true>(precision)                     \
                 : degree == 1 ? pick_prec<DD, 1, true>(precision)                     \
                               : pick_prec<DD, 2, true>(precision);                    \
        return degree == 0 ? pick_prec<DD, 0, false>(precision)                        \
             : degree == 1 ? pick_prec<DD, 1, false>(precision)                        \
                           : pick_prec<DD, 2, false>(precision);                       \
    }                                                                                  \
    template <>                                                                        \
    KernelFn nbr_kernel<DD>(bool unit)                                                 \
    {                                                                                  \
        return unit ? (KernelFn)k_neighbors<DD, true, kGroup>                          \
                    : (KernelFn)k_neighbors<DD, false, kGroup>;                        \
    }

#define PCMS_DEFINE_DIM_BVH(DD)                                                        \
    template <>                                                                        \
    KernelFn transfer_kernel_bvh<DD>(int degree, int precision, bool unit)             \
    {                                                                                  \
        if (unit)                                                                      \
            return degree == 0 ? pick_prec<DD, 0, true, true>(precision)               \
                 : degree == 1 ? pick_prec<DD, 1, true, true>(precision)               \
                               : pick_prec<DD, 2, true, true>(precision);              \
        return degree == 0 ? pick_prec<DD, 0, false, true>(precision)                  \
             : degree == 1 ? pick_prec<DD, 1, false, true>(precision)                  \
                           : pick_prec<DD, 2, false, true>(precision);                 \
    }                                                                                  \
    template <>                                                                        \
    KernelFn nbr_kernel_bvh<DD>(bool unit)                                             \
    {                                                                                  \
        return unit ? (KernelFn)k_neighbors<DD, true, kGroup, true>                    \
                    : (KernelFn)k_neighbors<DD, false, kGroup, true>;                  \
    }

#define PCMS_DEFINE_DIM_OPERATOR_BVH(DD)                                               \
    template <>                                                                        \
    KernelFn operator_kernel_bvh<DD>(int degree, int precision, bool unit)             \
    {                                                                                  \
        if (unit)                                                                      \
            return degree == 0 ? pick_prec_op<DD, 0, true, true>(precision)            \
                 : degree == 1 ? pick_prec_op<DD, 1, true, true>(precision)            \
                               : pick_prec_op<DD, 2, true, true>(precision);           \
        return degree == 0 ? pick_prec_op<DD, 0, false, true>(precision)               \
             : degree == 1 ? pick_prec_op<DD, 1, false, true>(precision)               \
                           : pick_prec_op<DD, 2, false, true>(precision);              \
    }

#define PCMS_DEFINE_DIM_OPERATOR(DD)                                                   \
    template <>                                                                        \
    KernelFn operator_kernel<DD>(int degree, int precision, bool unit)                 \
    {                                                                                  \
        if (unit)                                                                      \
            return degree == 0 ? pick_prec_op<DD, 0, true>(precision)                  \
                 : degree == 1 ? pick_prec_op<DD, 1, true>(precision)                  \
                               : pick_prec_op<DD, 2, true>(precision);                 \
        return degree == 0 ? pick_prec_op<DD, 0, false>(precision)                     \
             : degree == 1 ? pick_prec_op<DD, 1, false>(precision)                     \
                           : pick_prec_op<DD, 2, false>(precision);                    \
    }

}  // namespace pcms
