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
    int back_pcols[4]; // detector columns an adjoint tile can meet (max over views)
    int rspan;         // detector columns a single pixel can meet (max over views)
    int back_groups;   // view runs per chunk in the adjoint (partial volumes)
    int lds_budget;    // dynamic LDS bytes a workgroup may use
};

// Workspace of one call: strip records of a chunk of views, followed by the
// per-call volume buffer (prefix sums for the forward, sums for the adjoint).
struct RecLayout {
    int cap;           // records per strip
    int n_major_max;   // max(nx, ny)
    int views;         // views per chunk
    int pad;
    int64_t recs_off, sj0_off, soff_off, pixk_off, data_off;  // byte offsets
};

struct RecPtrs {
    void *recs;
    int *sj0;
    int *soff;
    int2 *pixk;
    char *data;
};

inline int64_t align256(int64_t v) { return (v + 255) & ~(int64_t)255; }

inline RecLayout make_layout(int cap, int n_major_max, int views, int nu, int nx, int ny,
                             size_t rec_size)
{
    RecLayout L;
    L.cap = cap;
    L.n_major_max = n_major_max;
    L.views = views;
    L.pad = 0;
    const int64_t strips = (int64_t)views * nu;
    L.recs_off = 0;
    L.sj0_off = align256(L.recs_off + strips * cap * (int64_t)rec_size);
    L.soff_off = align256(L.sj0_off + strips * n_major_max * (int64_t)sizeof(int));
    L.pixk_off = align256(L.soff_off + strips * (n_major_max + 1) * (int64_t)sizeof(int));
    L.data_off = align256(L.pixk_off + (int64_t)views * nx * ny * (int64_t)sizeof(int2));
    return L;
}

inline RecPtrs rec_ptrs(const RecLayout &L, void *ws, size_t)
{
    char *b = (char *)ws;
    RecPtrs P;
    P.recs = b + L.recs_off;
    P.sj0 = (int *)(b + L.sj0_off);
    P.soff = (int *)(b + L.soff_off);
    P.pixk = (int2 *)(b + L.pixk_off);
    P.data = b + L.data_off;
    return P;
}

// strip records for views [v0, v0 + nvc)
hipError_t launch_records(const DevGeom &G, const RecLayout &RL, bool fp64, int v0, int nvc,
                          void *ws, hipStream_t st);
hipError_t launch_strip_count(const DevGeom &G, int *max_count, hipStream_t st);

// x[B][nz][ny][nx] -> voxel columns X[ny*nx][B][nz] (same element type); for
// FP32 volumes also xmax[B] = bits of max |x| per batch element
hipError_t launch_to_columns(const void *x, void *X, unsigned *xmax, bool fp64, int B, int nz, int ny,
                            int nx, hipStream_t st);
// sum over g of xt[g][ny*nx][B][nz] -> x[B][nz][ny][nx] (partials added in order)
hipError_t launch_from_columns(const void *xt, void *x, int elem, int B, int nz, int ny, int nx,
                               int groups, hipStream_t st);

hipError_t launch_fwd3d(const DevGeom &G, const LaunchCfg &L, const RecLayout &RL, bool fp64,
                        int v0, int nvc, void *ws, const void *X, const unsigned *xmax, void *y,
                        int B, hipStream_t st);
hipError_t launch_back3d(const DevGeom &G, const LaunchCfg &L, const RecLayout &RL, bool fp64,
                         int v0, int nvc, void *ws, const void *y, void *xt, int B, bool first,
                         hipStream_t st);
// Pixel rows of the single-volume adjoint's tile (4 pixels wide): 2 when its
// workgroups have two waves or fewer (nz <= 128), or in FP64 (256-byte
// records, 8-byte detector values), whose occupancy the 4 x 4 tile's staged
// records and detector patch would bound, else 4.
inline int back_tile_rows(const DevGeom &G, bool fp64) { return G.nz <= 128 || fp64 ? 2 : 4; }

// Whether the smallest forward configuration (single batch element) fits LDS.
bool fwd3d_fits(const LaunchCfg &L, bool fp64);
// LDS bytes of the smallest adjoint configuration (single batch element).
size_t back3d_lds_min(const DevGeom &G, const LaunchCfg &L, bool fp64);
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
// rows of W^T (one per voxel), filled in no particular order within a row
hipError_t launch_csr_count_vox(const DevGeom &G, double tau_keep, int32_t *vox_cnt, hipStream_t st);
hipError_t launch_csr_fill_vox(const DevGeom &G, bool fp64_vals, double tau_keep,
                               const int64_t *row_ptr, int32_t *cursor, int32_t *cols, void *vals,
                               hipStream_t st);

}  // namespace smk
