// Application and export of a precomputed transfer operator (the fit of the
// PCMS paper, Section 3.2.1, Eq. 1, reduced to its shape functions for fixed
// source and target clouds: fhat_i = sum_j N_ij f_j for every field).
//
// The weights are stored by slot, [slot][sorted target], so a wave's lanes
// (64 consecutive targets of the processing order) read each slot with one
// coalesced load.  Each application first copies the caller's field-major
// values into bucket order (one record of padded_dim(n_fields) doubles per
// source), then gathers records by sorted position: the kept sources of
// neighbouring targets are neighbouring records, which the caches exploit.
// The operator's 12 bytes per kept source, the field values and the outputs
// are the HBM traffic; the record gathers are served mostly by the caches.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "fit.h"
#include "internal.h"
#include "launch_common.h"

namespace pcms {

namespace {

constexpr int kBatch = 4;    // slots whose loads are issued together
constexpr int kPairs = 2;    // field pairs per lane and pass over a target's slots

// L lanes per target: lane q of a target sums the field pairs q, q + L, ...
// (fields 2p, 2p + 1 are one 16-byte word of the record), so the L lanes of a
// target read one record's consecutive words in the same instruction and a
// wave's gather touches 64 / L records' lines instead of 64.
template <int L>
__global__ void __launch_bounds__(256) k_op_apply(const int32_t *__restrict__ opn,
                                                  const int32_t *__restrict__ opc,
                                                  const double *__restrict__ opw,
                                                  const int *__restrict__ tperm, int n_tgt,
                                                  const double *__restrict__ svals, int nf, int nfs,
                                                  double *__restrict__ out, int n_blocks)
{
    // XCD-aware: each XCD takes a contiguous range of (spatially sorted)
    // targets, so its L2 holds the records their neighbours share
    const int lb = logical_block(n_blocks);
    const int gi = lb * blockDim.x + threadIdx.x;
    const int i = gi / L, q = gi % L;
    if (lb >= n_blocks || i >= n_tgt) return;
    const int n = opn[i];
    const int64_t ti = tperm[i];
    const int np = nfs / 2;   // field pairs per record
    if (n < 0) {
        for (int l = 2 * q; l < nf; l += 2 * L) {
            out[(int64_t)l * n_tgt + ti] = NAN;
            if (l + 1 < nf) out[(int64_t)(l + 1) * n_tgt + ti] = NAN;
        }
        return;
    }
    for (int p0 = q; p0 < np; p0 += L * kPairs) {
        double acc[kPairs][2];
#pragma unroll
        for (int h = 0; h < kPairs; ++h) acc[h][0] = acc[h][1] = 0.0;
        for (int e0 = 0; e0 < n; e0 += kBatch) {
            int c[kBatch];
            double w[kBatch];
#pragma unroll
            for (int j = 0; j < kBatch; ++j) {
                const int e = e0 + j;
                const bool ok = e < n;
                const int64_t at = (int64_t)(ok ? e : 0) * n_tgt + i;   // slot 0 exists (n >= 1)
                c[j] = opc[at];
                w[j] = ok ? opw[at] : 0.0;
            }
            double fv[kBatch][kPairs][2];
#pragma unroll
            for (int j = 0; j < kBatch; ++j) {
                const double *row = svals + (int64_t)c[j] * nfs;
#pragma unroll
                for (int h = 0; h < kPairs; ++h) {
                    const int p = p0 + h * L;
                    fv[j][h][0] = fv[j][h][1] = 0.0;
                    if (p < np) load_pair(row + 2 * p, fv[j][h][0], fv[j][h][1]);
                }
            }
#pragma unroll
            for (int j = 0; j < kBatch; ++j)
#pragma unroll
                for (int h = 0; h < kPairs; ++h) {
                    acc[h][0] = __builtin_fma(w[j], fv[j][h][0], acc[h][0]);
                    acc[h][1] = __builtin_fma(w[j], fv[j][h][1], acc[h][1]);
                }
        }
#pragma unroll
        for (int h = 0; h < kPairs; ++h) {
            const int l = 2 * (p0 + h * L);
            if (l < nf) out[(int64_t)l * n_tgt + ti] = acc[h][0];
            if (l + 1 < nf) out[(int64_t)(l + 1) * n_tgt + ti] = acc[h][1];
        }
    }
}

__global__ void k_op_export(const int32_t *__restrict__ opn, const int32_t *__restrict__ opc,
                            const double *__restrict__ opw, const int *__restrict__ tperm,
                            const int *__restrict__ perm, int n_tgt, int width, int stride,
                            int32_t *n_kept, int32_t *cols, double *weights)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_tgt) return;
    const int n = opn[i];
    const int64_t ti = tperm[i];
    n_kept[ti] = n;
    // n <= width <= stride (checked on the host): the whole row is written,
    // kept entries first, then -1 / 0
    for (int e = 0; e < stride; ++e) {
        const bool ok = e < n && e < width;
        if (cols) cols[ti * stride + e] = ok ? perm[opc[(int64_t)e * n_tgt + i]] : -1;
        if (weights) weights[ti * stride + e] = ok ? opw[(int64_t)e * n_tgt + i] : 0.0;
    }
}

}  // namespace

pcms_status operator_apply(const Operator &op, const double *vals, int n_fields, double *out,
                           hipStream_t s)
{
    if (op.n_tgt == 0) return PCMS_OK;
    const int nfs = padded_dim(n_fields);
    void *raw = nullptr;
    pcms_status st = scratch_alloc(&raw, sizeof(double) * (size_t)op.n_src * nfs, s);
    if (st != PCMS_OK) return st;
    double *svals = (double *)raw;
    Grid view{};
    view.n_src = op.n_src;
    view.iperm = op.iperm;
    if ((st = gather_values(&view, vals, n_fields, svals, s)) != PCMS_OK) return st;
    // lanes per target: one per 16-byte word of a record, at most 4
    const int lanes = nfs >= 8 ? 4 : nfs >= 4 ? 2 : 1;
    const int blocks = (int)((op.n_tgt * lanes + 255) / 256);
    const int padded = ((blocks + 7) / 8) * 8;
    if (lanes == 4)
        k_op_apply<4><<<padded, 256, 0, s>>>(op.op_n, op.op_c, op.op_w, op.tperm, (int)op.n_tgt,
                                             svals, n_fields, nfs, out, blocks);
    else if (lanes == 2)
        k_op_apply<2><<<padded, 256, 0, s>>>(op.op_n, op.op_c, op.op_w, op.tperm, (int)op.n_tgt,
                                             svals, n_fields, nfs, out, blocks);
    else
        k_op_apply<1><<<padded, 256, 0, s>>>(op.op_n, op.op_c, op.op_w, op.tperm, (int)op.n_tgt,
                                             svals, n_fields, nfs, out, blocks);
    PCMS_HIP(hipGetLastError());
    scratch_free(raw, s);
    return PCMS_OK;
}

pcms_status operator_export(const Operator &op, int stride, int32_t *n_kept, int32_t *cols,
                            double *weights, hipStream_t s)
{
    if (op.n_tgt == 0) return PCMS_OK;
    const int blocks = (int)((op.n_tgt + 255) / 256);
    k_op_export<<<blocks, 256, 0, s>>>(op.op_n, op.op_c, op.op_w, op.tperm, op.perm,
                                       (int)op.n_tgt, op.width, stride, n_kept, cols, weights);
    PCMS_HIP(hipGetLastError());
    return PCMS_OK;
}

}  // namespace pcms
