// Allocation-free variant of the transfer on a prebuilt grid, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).  Its workspace -- status counts,
// target order, sort buffers and bucket-ordered field records -- lives in a
// fixed device array of this translation unit instead of stream-ordered
// scratch; the kernels are those of pcms_mls_transfer_grid.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"

namespace pcms {

namespace {

constexpr size_t kScratchBytes = PCMS_NOALLOC_SCRATCH_BYTES;

// One copy per device, held until the process ends.  In host code this name
// stands for the symbol, not a device address: only the address returned by
// hipGetSymbolAddress may be handed to kernels or copies.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once per
// device (with that device current) on its first call.
pcms_status scratch_address(void **out)
{
    int dev = 0;
    PCMS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device ordinal " + std::to_string(dev) + " beyond the supported 64");
        return PCMS_ERR_ARG;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        void *p = nullptr;
        PCMS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_addr[dev] = p;
    }
    *out = g_addr[dev];
    return PCMS_OK;
}

}  // namespace

}  // namespace pcms

using namespace pcms;

extern "C" {

size_t pcms_noalloc_scratch_bytes(void) { return kScratchBytes; }

pcms_status pcms_mls_transfer_grid_noalloc(const pcms_grid *grid, const double *src_vals,
                                           int32_t n_fields, const double *tgt, int64_t n_tgt,
                                           int32_t basis_degree, const pcms_radius *radius,
                                           int32_t k_cap, const pcms_mls_opts *opts,
                                           pcms_stream_t stream, double *tgt_vals,
                                           uint8_t *status)
{
    if (!grid) {
        set_error("grid is NULL");
        return PCMS_ERR_ARG;
    }
    const Grid *g = reinterpret_cast<const Grid *>(grid);
    pcms_status st = check_transfer_args(g->n_src, g->dim, src_vals, n_fields, tgt, n_tgt,
                                         basis_degree, radius, k_cap, opts, tgt_vals);
    if (st != PCMS_OK) return st;
    if (opts && (opts->flags & PCMS_PROFILE)) {
        set_error("PCMS_PROFILE is not available without allocation (it creates HIP events)");
        return PCMS_ERR_ARG;
    }
    const size_t need = transfer_ws_bytes(g->n_src, n_fields, n_tgt);
    if (need > kScratchBytes) {
        set_error("the transfer needs " + std::to_string(need) + " bytes of workspace, more than "
                  "the " + std::to_string(kScratchBytes) + " of the allocation-free entry point "
                  "(about 8 * (n_src + n_tgt) * (n_fields rounded up to even) + 28 * n_tgt bytes)");
        return PCMS_ERR_ARG;
    }
    if (n_tgt == 0) return PCMS_OK;
    void *ws = nullptr;
    if ((st = scratch_address(&ws)) != PCMS_OK) return st;
    profile_off();
    return transfer_on_grid(g, src_vals, n_fields, tgt, n_tgt, basis_degree, radius, k_cap, opts,
                            (hipStream_t)stream, tgt_vals, status, ws);
}

}  // extern "C"
