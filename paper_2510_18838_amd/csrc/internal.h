// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "device_common.h"
#include "pcms_mls.h"

namespace pcms {

// Library-owned grid handle.
struct Grid {
    int dim;
    int64_t n_src;
    int n_cells_cap;
    double g[kMaxDim];
    GridParams *params;   // device
    int *cell_start;      // device [n_cells_cap + 1]
    int *perm;            // device [n_src]: sorted position -> source index
    int *iperm;           // device [n_src]: source index -> sorted position
    double *spts;         // device [n_src * padded_dim(dim)]: sorted coordinates
    int device;
};

// error plumbing ------------------------------------------------------------
void set_error(const std::string &msg);
pcms_status hip_fail(hipError_t e, const char *what);

#define PCMS_HIP(call)                                              \
    do {                                                            \
        hipError_t e_ = (call);                                     \
        if (e_ != hipSuccess) return ::pcms::hip_fail(e_, #call);   \
    } while (0)

// stream-ordered scratch allocation ------------------------------------------
pcms_status scratch_alloc(void **p, size_t bytes, hipStream_t s);
void scratch_free(void *p, hipStream_t s);

// grid construction (sort.hip) ----------------------------------------------
int cells_cap_for(int64_t n_src);
// Builds `grid` (allocated by the caller with the right capacity) from src.
// cell_width > 0: metric bucket width; else buckets sized for pts_per_cell.
pcms_status build_grid_device(Grid *grid, const double *src, double cell_width,
                              double pts_per_cell, hipStream_t s);
// Target ordering: tperm[i] = index of the target at sorted position i.
pcms_status sort_targets(const Grid *grid, const double *tgt, int64_t n_tgt, int *tperm,
                         hipStream_t s);
// Sorted field copy: svals[p * n_fields + l] = vals[l * n_src + perm[p]].
pcms_status gather_values(const Grid *grid, const double *vals, int n_fields, double *svals,
                          hipStream_t s);

// search and fit (mls.hip) ----------------------------------------------------
struct LaunchSpec {
    const Grid *grid;
    const double *tgt;
    const int *tperm;
    int64_t n_tgt;
    pcms_radius radius;
    int k_cap;
    int block;
    int32_t *summary;   // device [4]
};

pcms_status launch_neighbors(const LaunchSpec &ls, int32_t *nbr, int32_t *n_kept,
                             int32_t *n_found, double *r2, uint8_t *status, hipStream_t s);

pcms_status launch_transfer(const LaunchSpec &ls, const double *svals, int n_fields, int degree,
                            int weight, int precision, double lambda, double *out,
                            uint8_t *status, hipStream_t s);

pcms_status zero_ints(int32_t *p, int n, hipStream_t s);

}  // namespace pcms
