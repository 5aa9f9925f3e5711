// Device helpers shared by the kernels of the one-problem and batched
// transfer launches.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"

namespace pcms {

// Writes a source's FP64 record (padded_dim(D) doubles, the padding zero,
// with 16-byte stores), FP32 record (D floats, fl32(x_k - lo_k)) and 32-bit
// fixed-point record (D words, quantize()) from its D coordinates.
template <int D>
__device__ __forceinline__ void write_records(const double *__restrict__ x, const GridParams &gp,
                                              double *__restrict__ r64, float *__restrict__ r32,
                                              uint32_t *__restrict__ rq)
{
    constexpr int DP = padded_dim(D);
    double v[DP];
#pragma unroll
    for (int k = 0; k < DP; ++k) v[k] = k < D ? x[k] : 0.0;
#pragma unroll
    for (int k = 0; k < DP; k += 2) *reinterpret_cast<double2 *>(r64 + k) = make_double2(v[k], v[k + 1]);
#pragma unroll
    for (int k = 0; k < D; ++k) r32[k] = (float)(v[k] - gp.lo[k]);
#pragma unroll
    for (int k = 0; k < D; ++k) rq[k] = quantize(v[k], gp.lo[k], gp.iqs[k]);
}

// The same for a dimension known at run time.
__device__ __forceinline__ void write_records_dim(const double *__restrict__ x, int dim,
                                                  const GridParams &gp, double *__restrict__ r64,
                                                  float *__restrict__ r32, uint32_t *__restrict__ rq)
{
    switch (dim) {
    case 1: write_records<1>(x, gp, r64, r32, rq); break;
    case 2: write_records<2>(x, gp, r64, r32, rq); break;
    case 3: write_records<3>(x, gp, r64, r32, rq); break;
    case 4: write_records<4>(x, gp, r64, r32, rq); break;
    default: write_records<5>(x, gp, r64, r32, rq); break;
    }
}

// Blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// range of (spatially sorted) target blocks so its L2 sees neighbouring work.
__device__ __forceinline__ int logical_block(int n_blocks)
{
    const int per = (n_blocks + 7) >> 3;
    return (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
}

// Adds the wave's counts of statuses 1, 2, 3 and CAPPED to summary[0..3]
// (one atomic per wave and count).
__device__ __forceinline__ void add_summary(int32_t *summary, int st, bool active)
{
    if (!summary) return;
    unsigned long long b1 = __ballot(active && (st & 0xF) == PCMS_TGT_UNDERDETERMINED);
    unsigned long long b2 = __ballot(active && (st & 0xF) == PCMS_TGT_SINGULAR);
    unsigned long long b3 = __ballot(active && (st & 0xF) == PCMS_TGT_RADIUS_EXHAUSTED);
    unsigned long long b4 = __ballot(active && (st & PCMS_TGT_CAPPED));
    if ((threadIdx.x & 63) == 0) {
        if (b1) atomicAdd(&summary[0], (int)__popcll(b1));
        if (b2) atomicAdd(&summary[1], (int)__popcll(b2));
        if (b3) atomicAdd(&summary[2], (int)__popcll(b3));
        if (b4) atomicAdd(&summary[3], (int)__popcll(b4));
    }
}

}  // namespace pcms
