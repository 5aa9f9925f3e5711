// The kernels of the batched transfer (batch.hip), one per class of
// problems, instantiated per precision in batch_fp64.hip,
// batch_mixed.hip and batch_refine.hip so that the variants compile in
// parallel.
#pragma once

#include <hip/hip_runtime.h>

#include "fit.h"
#include "internal.h"
#include "launch_common.h"

namespace pcms {

// Classes of the batched problems handled by the class kernels:
// dimension 1-3, degree 0-2, unit or scaled metric.
constexpr int kBatchClasses = 18;
PCMS_HD inline int batch_class(int dim, int degree, int unit) { return ((dim - 1) * 3 + degree) * 2 + unit; }

// Arguments of a class kernel: the batch's global arrays and its class's
// slice [item_begin, item_end) of the work queue.
struct BArgs {
    const BatchProb *probs;
    const GridParams *params;
    const int *cs;
    const double *spts;
    const float *spts32;
    const uint32_t *sq;
    const int *perm;
    const int *tperm;
    const double *svals;
    const int4 *items;
    int item_begin, item_end;
    int32_t *summary;
    int weight;
    double lambda;
};

// Launch of the kernel of class `cls` and precision PREC, one block per work
// item of its slice; defined per precision.
template <int PREC>
pcms_status batch_launch(int cls, const BArgs &b, int block, size_t shm, hipStream_t s);

#ifndef PCMS_BATCH_WAVES
#define PCMS_BATCH_WAVES(PREC) ((PREC) == PCMS_MIXED_REFINE ? 2 : 3)
#endif

namespace {

// Transfer of one class of problems (dimension D, degree P, metric UNIT):
// block j takes work item item_begin + j (problem, first sorted target,
// count), and its threads run one target each with the one-problem code.
// The items of a slice are in decreasing order of estimated cost and the
// hardware dispatches blocks in order as slots free up, so the schedule is
// the greedy largest-first one.  One instantiation per class, so that each
// gets its own register allocation.  (A persistent block looping over items
// kept the per-target state of one item live across the loop and spilled
// 200-290 bytes per lane.)
template <int PREC, int D, int P, bool UNIT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PCMS_BATCH_WAVES(PREC))))
k_batch_transfer(BArgs b)
{
    extern __shared__ int lds[];
    {
        const int it = b.item_begin + (int)blockIdx.x;   // < item_end by the launch
        const int4 w = b.items[it];
        const int q = w.x;
        const BatchProb &P_ = b.probs[q];
        KArgs a{};
        a.gp = b.params + q;
        a.cs = b.cs + P_.cs_off;
        a.spts = b.spts + P_.spts_off;
        a.spts32 = b.spts32 + P_.s32_off;
        a.sq = b.sq + P_.s32_off;
        a.perm = b.perm + P_.src_off;
        a.tgt = P_.tgt;
        a.tperm = b.tperm + P_.tgt_off;
        a.n_tgt = P_.n_tgt;
        a.mode = P_.mode;
        a.k = P_.k;
        a.n_min = P_.n_min;
        a.max_iter = P_.max_iter;
        a.r = P_.r;
        a.k_cap = P_.k_cap;
        a.words = P_.words;
        a.stride = P_.stride;
        a.svals = b.svals + P_.sval_off;
        a.nf = P_.nf;
        a.nfs = P_.nfs;
        a.weight = b.weight;
        a.lambda = b.lambda;
        a.out = P_.out;
        a.status = P_.status;
        a.summary = b.summary;
        const int slot = (int)threadIdx.x;
        const bool active = slot < w.z;
        int st = 0;
        if (active) {
            const GridParams gp = b.params[q];
            st = xfer_target<D, P, PREC, UNIT, 1>(a, gp, w.y + slot, lds + slot * P_.stride,
                                                  Grp<1>{0});
        }
        add_summary(b.summary, st, active);
    }
}

template <int PREC, int D, int P, bool UNIT>
pcms_status launch_class(const BArgs &b, int block, size_t shm, hipStream_t s)
{
    const int blocks = b.item_end - b.item_begin;
    if (blocks <= 0) return PCMS_OK;
    hipLaunchKernelGGL((k_batch_transfer<PREC, D, P, UNIT>), dim3(blocks), dim3(block), shm, s, b);
    PCMS_HIP(hipGetLastError());
    return PCMS_OK;
}

}  // namespace

#define PCMS_BATCH_CLASSES(X, PR)                                                          \
    X(PR, 1, 0, 0) X(PR, 1, 0, 1) X(PR, 1, 1, 0) X(PR, 1, 1, 1) X(PR, 1, 2, 0) X(PR, 1, 2, 1) \
    X(PR, 2, 0, 0) X(PR, 2, 0, 1) X(PR, 2, 1, 0) X(PR, 2, 1, 1) X(PR, 2, 2, 0) X(PR, 2, 2, 1) \
    X(PR, 3, 0, 0) X(PR, 3, 0, 1) X(PR, 3, 1, 0) X(PR, 3, 1, 1) X(PR, 3, 2, 0) X(PR, 3, 2, 1)
#define PCMS_BATCH_LAUNCH_CASE(PR, DD, PP, UU)                                             \
    case ((DD - 1) * 3 + PP) * 2 + UU: return launch_class<PR, DD, PP, (bool)UU>(b, block, shm, s);

#define PCMS_DEFINE_BATCH_KERNEL(PR)                                                       \
    template <>                                                                           \
    pcms_status batch_launch<PR>(int cls, const BArgs &b, int block, size_t shm,          \
                                 hipStream_t s)                                           \
    {                                                                                     \
        switch (cls) {                                                                    \
            PCMS_BATCH_CLASSES(PCMS_BATCH_LAUNCH_CASE, PR)                                \
        }                                                                                 \
        return PCMS_ERR_ARG;                                                              \
    }

}  // namespace pcms
