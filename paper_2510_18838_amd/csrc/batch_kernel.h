// The persistent kernel of the batched transfer (batch.hip), instantiated
// per precision in batch_fp64.hip, batch_mixed.hip and batch_refine.hip so
// that the variants compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include "fit.h"
#include "internal.h"
#include "launch_common.h"

namespace pcms {

// Arguments of the persistent kernel: the batch's global arrays and queue.
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
    int n_items;
    int *counter;
    int32_t *summary;
    int weight;
    double lambda;
};

// Launch of the persistent kernel of precision PREC on `blocks` blocks, and
// its resident blocks per CU; defined per precision.
template <int PREC>
pcms_status batch_launch(const BArgs &b, int blocks, int block, size_t shm, hipStream_t s);
template <int PREC>
int batch_occupancy(int block, size_t shm);

namespace {


// Persistent transfer: each block takes work items (problem, first sorted
// target, count) from the counter until the queue is empty; its threads run
// one target each with the problem's (dimension, degree, metric) variant of
// the one-problem code.  Problems of dimension 1-3 only.
template <int PREC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_batch_transfer(BArgs b)
{
    extern __shared__ int lds[];
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(b.counter, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();   // every thread has read s_item before it is rewritten
        if (it >= b.n_items) break;
        const int4 w = b.items[it];
        const int q = w.x;
        const BatchProb &P = b.probs[q];
        KArgs a{};
        a.gp = b.params + q;
        a.cs = b.cs + P.cs_off;
        a.spts = b.spts + P.spts_off;
        a.spts32 = b.spts32 + P.s32_off;
        a.sq = b.sq + P.s32_off;
        a.perm = b.perm + P.src_off;
        a.tgt = P.tgt;
        a.tperm = b.tperm + P.tgt_off;
        a.n_tgt = P.n_tgt;
        a.mode = P.mode;
        a.k = P.k;
        a.n_min = P.n_min;
        a.max_iter = P.max_iter;
        a.r = P.r;
        a.k_cap = P.k_cap;
        a.words = P.words;
        a.stride = P.stride;
        a.svals = b.svals + P.sval_off;
        a.nf = P.nf;
        a.nfs = P.nfs;
        a.weight = b.weight;
        a.lambda = b.lambda;
        a.out = P.out;
        a.status = P.status;
        a.summary = b.summary;
        const int slot = (int)threadIdx.x;
        const bool active = slot < w.z;
        int st = 0;
        if (active) {
            const GridParams gp = b.params[q];
            const int i = w.y + slot;
            int *L = lds + slot * P.stride;
            const Grp<1> g{0};
            const int cls = (P.dim * 3 + P.degree) * 2 + P.unit;
#define PCMS_BCASE(DD, PP, UU)                                                   \
    case (DD * 3 + PP) * 2 + UU:                                                 \
        st = xfer_target<DD, PP, PREC, (bool)UU, 1>(a, gp, i, L, g);             \
        break;
            switch (cls) {
                PCMS_BCASE(1, 0, 1) PCMS_BCASE(1, 1, 1) PCMS_BCASE(1, 2, 1)
                PCMS_BCASE(2, 0, 1) PCMS_BCASE(2, 1, 1) PCMS_BCASE(2, 2, 1)
                PCMS_BCASE(3, 0, 1) PCMS_BCASE(3, 1, 1) PCMS_BCASE(3, 2, 1)
                PCMS_BCASE(1, 0, 0) PCMS_BCASE(1, 1, 0) PCMS_BCASE(1, 2, 0)
                PCMS_BCASE(2, 0, 0) PCMS_BCASE(2, 1, 0) PCMS_BCASE(2, 2, 0)
                PCMS_BCASE(3, 0, 0) PCMS_BCASE(3, 1, 0) PCMS_BCASE(3, 2, 0)
            default: break;
            }
#undef PCMS_BCASE
        }
        add_summary(b.summary, st, active);
    }
}

}  // namespace

#define PCMS_DEFINE_BATCH_KERNEL(PR)                                                      \
    template <>                                                                          \
    pcms_status batch_launch<PR>(const BArgs &b, int blocks, int block, size_t shm,      \
                                 hipStream_t s)                                          \
    {                                                                                    \
        hipLaunchKernelGGL(k_batch_transfer<PR>, dim3(blocks), dim3(block), shm, s, b);  \
        PCMS_HIP(hipGetLastError());                                                     \
        return PCMS_OK;                                                                  \
    }                                                                                    \
    template <>                                                                          \
    int batch_occupancy<PR>(int block, size_t shm)                                       \
    {                                                                                    \
        int n = 0;                                                                       \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_transfer<PR>, block, \
                                                         shm) != hipSuccess)             \
            return 1;                                                                    \
        return n;                                                                        \
    }

}  // namespace pcms
