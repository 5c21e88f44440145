// sm_internal.h -- launch entry points shared between the API layer and the
// kernel translation units (host side only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sm_common.h"

namespace smk {

// Launch shapes chosen at plan creation.
struct LaunchCfg {
    int fwd_threads;   // 64 * ceil(nv / 64)
    int back_threads;  // 64 * ceil(nz / 64)
    int back_tile_x[4], back_tile_y[4];  // adjoint pixel tile per batch width 1, 2, 4, 8
    int back_pcols[4];                   // detector columns a tile can meet (max over views)
    int back_rmax;                       // strip records staged per round
    int lds_budget;                      // dynamic LDS bytes a workgroup may use
};

// x[B][nz][ny][nx] -> xt[ny][nx][B][nz] and back
hipError_t launch_to_columns(const void *x, void *xt, int elem, int B, int nz, int ny, int nx,
                             hipStream_t st);
hipError_t launch_from_columns(const void *xt, void *x, int elem, int B, int nz, int ny, int nx,
                               hipStream_t st);

hipError_t launch_fwd3d(const DevGeom &G, const LaunchCfg &L, bool fp64, const void *xt, void *y,
                        int B, hipStream_t st);
hipError_t launch_back3d(const DevGeom &G, const LaunchCfg &L, bool fp64, const void *y, void *xt,
                         int B, hipStream_t st);
hipError_t launch_fwd2d(const DevGeom &G, bool fp64, const void *x, void *y, int B,
                        hipStream_t st);
hipError_t launch_back2d(const DevGeom &G, bool fp64, const void *y, void *x, int B,
                         hipStream_t st);

// exact footprint boxes of one view (documented FP64 order), device output
hipError_t launch_footprints(const DevGeom &G, int view, int32_t *boxes, hipStream_t st);

// CSR passes over all (view, voxel) pairs
hipError_t launch_csr_count(const DevGeom &G, double tau_keep, int32_t *row_cnt, hipStream_t st);
hipError_t launch_csr_fill(const DevGeom &G, bool fp64_vals, double tau_keep,
                           const int64_t *row_ptr, int32_t *cursor, int32_t *cols, void *vals,
                           hipStream_t st);
hipError_t launch_csr_sort(const int64_t *row_ptr, int64_t n_rows, int32_t *cols, void *vals,
                           bool fp64_vals, hipStream_t st);
hipError_t launch_scan_counts(const int32_t *cnt, int64_t n, int64_t *row_ptr, hipStream_t st);

}  // namespace smk
