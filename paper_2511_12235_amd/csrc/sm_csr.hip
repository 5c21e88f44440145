// sm_csr.hip -- explicit system matrix for small problems and the exact
// footprint boxes (Sec. I: W in R^{M x N}; eq. "relevant detectors 2d" and
// the row bounds of Sec. III-C).
//
// CSR: a count pass (one thread per (view, voxel), integer atomics on the row
// counts), a scan, a fill pass (per-row cursors) and a per-row sort by column,
// so the result does not depend on scheduling.  The pattern W > tau_keep is
// decided with FP64 weights; values come in the requested precision.
#include "sm_internal.h"

namespace smk {

// ---------------------------------------------------------------------------
// exact footprint box (fixed FP64 operation order, no contraction)
// ---------------------------------------------------------------------------
__device__ void cell_range_exact(double lo, double hi, double o, double p, int n, int &first,
                                 int &last)
{
#pragma clang fp contract(off)
    double e = floor((lo - o) / p);
    int m = e < 0.0 ? 0 : (e > (double)n ? n : (int)e);
    while (m > 0 && o + (double)m * p > lo) --m;
    while (m < n && !(o + (double)(m + 1) * p > lo)) ++m;
    first = m;
    e = floor((hi - o) / p);
    m = e < -1.0 ? -1 : (e > (double)(n - 1) ? n - 1 : (int)e);
    while (m < n - 1 && o + (double)(m + 1) * p < hi) ++m;
    while (m >= 0 && !(o + (double)m * p < hi)) --m;
    last = m;
}

__device__ void footprint_box(const DevGeom &G, double cp, double sp, int ix, int iy, int iz,
                              int box[4])
{
#pragma clang fp contract(off)
    const double D = G.D;
    double umin = 1e308, umax = -1e308, lmin = 1e308, lmax = -1e308;
    for (int q = 0; q < 4; ++q) {
        const double x = G.x0 + (double)(ix + (q >> 1)) * G.a;
        const double y = G.y0 + (double)(iy + (q & 1)) * G.b;
        const double l = G.s - (x * cp + y * sp);
        const double t = y * cp - x * sp;
        const double u = (D * t) / l;
        umin = u < umin ? u : umin;
        umax = u > umax ? u : umax;
        lmin = l < lmin ? l : lmin;
        lmax = l > lmax ? l : lmax;
    }
    cell_range_exact(umin, umax, G.u0, G.du, G.nu, box[0], box[1]);
    if (G.dim == 2) {
        box[2] = 0;
        box[3] = 0;
        return;
    }
    const double za = G.z0 + (double)iz * G.c;
    const double zb = G.z0 + (double)(iz + 1) * G.c;
    const double v1 = (D * za) / lmin, v2 = (D * za) / lmax;
    const double v3 = (D * zb) / lmin, v4 = (D * zb) / lmax;
    const double vmin = v1 < v2 ? v1 : v2;
    const double vmax = v3 > v4 ? v3 : v4;
    cell_range_exact(vmin, vmax, G.v0, G.dv, G.nv, box[2], box[3]);
}

__global__ void footprints_kernel(DevGeom G, int view, int32_t *boxes)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nvox = (int64_t)G.nx * G.ny * G.nz;
    if (j >= nvox) return;
    const int ix = (int)(j % G.nx);
    const int iy = (int)((j / G.nx) % G.ny);
    const int iz = (int)(j / ((int64_t)G.nx * G.ny));
    const double2 cs = G.trig[view];
    int box[4];
    footprint_box(G, cs.x, cs.y, ix, iy, iz, box);
    for (int q = 0; q < 4; ++q) boxes[4 * j + q] = box[q];
}

hipError_t launch_footprints(const DevGeom &G, int view, int32_t *boxes, hipStream_t st)
{
    const int64_t nvox = (int64_t)G.nx * G.ny * G.nz;
    hipLaunchKernelGGL(footprints_kernel, dim3((unsigned)((nvox + 255) / 256)), dim3(256), 0, st, G,
                       view, boxes);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-voxel weights of one view
// ---------------------------------------------------------------------------
// Calls fn(ray, w64, w32) for every detector element with w64 > tau_keep.
template <typename F>
__device__ void voxel_view_weights(const DevGeom &G, int view, int ix, int iy, int iz,
                                   double tau_keep, bool want32, F fn)
{
    const double2 cs = G.trig[view];
    const double cp = cs.x, sp = cs.y;
    int k0, k1;
    pixel_columns(G, cp, sp, ix, iy, k0, k1);
    if (G.dim == 2) {
        const double xc = G.x0 + ((double)ix + 0.5) * G.a;
        const double yc = G.y0 + ((double)iy + 0.5) * G.b;
        const double lc = G.s - (xc * cp + yc * sp);
        const double tc = yc * cp - xc * sp;
        for (int k = k0; k <= k1; ++k) {
            const double mu0 = (G.u0 + (double)k * G.du) / G.D, mu1 = (G.u0 + (double)(k + 1) * G.du) / G.D;
            const double w = sweep_area<double>(cp, sp, lc, tc, mu1, G.a, G.b) -
                             sweep_area<double>(cp, sp, lc, tc, mu0, G.a, G.b);
            if (w > tau_keep) {
                float w32 = 0.f;
                if (want32)
                    w32 = sweep_area<float>(cp, sp, lc, tc, mu1, (float)G.a, (float)G.b) -
                          sweep_area<float>(cp, sp, lc, tc, mu0, (float)G.a, (float)G.b);
                fn((int64_t)view * G.nu + k, w, w32);
            }
        }
        return;
    }
    const double za = G.z0 + (double)iz * G.c, zb = za + G.c;
    double2 ws[8];
    for (int k = k0; k <= k1; ++k) {
        Rec<double> R;
        build_record<double>(G, cp, sp, ix, iy, k, R, ws);
        const int n = R.n;
        if (n == 0) continue;
        Rec<float> Rf;
        if (want32) build_record<float>(G, cp, sp, ix, iy, k, Rf, ws);
        const double lmin = R.lc + R.tab[0][0], lmax = R.lc + R.tab[n - 1][0];
        // planes cutting the voxel inside the strip: [pf, pl]; estimated from
        // the slope where the plane's highest (lowest) point meets za (zb),
        // then settled with exact comparisons
        const double tst = za / (za >= 0.0 ? lmax : lmin);
        int pf = (int)fmin(fmax(floor((tst * G.D - G.v0) / G.dv) + 1.0, 0.0), (double)(G.nv + 1));
        while (pf > 0) {
            const double t = G.tau[pf - 1];
            if (t * (t >= 0.0 ? lmax : lmin) > za) --pf; else break;
        }
        while (pf <= G.nv) {
            const double t = G.tau[pf];
            if (!(t * (t >= 0.0 ? lmax : lmin) > za)) ++pf; else break;
        }
        const double tss = zb / (zb >= 0.0 ? lmin : lmax);
        int pl = (int)fmin(fmax(ceil((tss * G.D - G.v0) / G.dv) - 1.0, -1.0), (double)G.nv);
        while (pl < G.nv) {
            const double t = G.tau[pl + 1];
            if (t * (t >= 0.0 ? lmin : lmax) < zb) ++pl; else break;
        }
        while (pl >= 0) {
            const double t = G.tau[pl];
            if (!(t * (t >= 0.0 ? lmin : lmax) < zb)) --pl; else break;
        }
        const int r0 = max(pf - 1, 0), r1 = min(pl, G.nv - 1);
        const double cA = G.c * R.tab[0][2];
        const float cA32 = want32 ? (float)G.c * Rf.tab[0][2] : 0.f;
        double Hlo = 0.0;
        float Hlo32 = 0.f;
        for (int r = r0; r <= r1 + 1 && r <= G.nv; ++r) {
            // volume of the voxel below plane r: K(za) - K(zb)
            double H;
            float H32 = 0.f;
            if (r < pf) {
                H = 0.0;
            } else if (r > pl) {
                H = cA;
                H32 = cA32;
            } else {
                const double t = G.tau[r];
                const double it = t != 0.0 ? 1.0 / t : 0.0;
                const double ea = t * R.lc - za;
                H = eval_K<double>(R.tab, n, t, it, ea) - eval_K<double>(R.tab, n, t, it, ea - G.c);
                if (want32) {
                    const float tf = (float)t, itf = tf != 0.f ? 1.f / tf : 0.f;
                    H32 = eval_K<float>(Rf.tab, Rf.n, tf, itf, (float)ea) -
                          eval_K<float>(Rf.tab, Rf.n, tf, itf, (float)(ea - G.c));
                }
            }
            if (r > r0) {
                const double w = H - Hlo;
                if (w > tau_keep) fn(((int64_t)view * G.nv + (r - 1)) * G.nu + k, w, H32 - Hlo32);
            }
            Hlo = H;
            Hlo32 = H32;
        }
    }
}

// Grid-stride loops: an AMD dispatch holds at most 2^32 work-items per
// dimension, and n_p * n_vox exceeds that for the larger scans.
__global__ void csr_count_kernel(DevGeom G, double tau_keep, int32_t *row_cnt)
{
    const int64_t nvox = (int64_t)G.nx * G.ny * G.nz;
    const int64_t n = nvox * G.n_p;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int view = (int)(q / nvox);
        const int64_t j = q - (int64_t)view * nvox;
        const int ix = (int)(j % G.nx), iy = (int)((j / G.nx) % G.ny), iz = (int)(j / ((int64_t)G.nx * G.ny));
        voxel_view_weights(G, view, ix, iy, iz, tau_keep, false,
                           [&](int64_t i, double, float) { atomicAdd(&row_cnt[i], 1); });
    }
}

template <typename V>
__global__ void csr_fill_kernel(DevGeom G, double tau_keep, const int64_t *row_ptr,
                                int32_t *cursor, int32_t *cols, V *vals)
{
    const int64_t nvox = (int64_t)G.nx * G.ny * G.nz;
    const int64_t n = nvox * G.n_p;
    const bool want32 = sizeof(V) == 4;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int view = (int)(q / nvox);
        const int64_t j = q - (int64_t)view * nvox;
        const int ix = (int)(j % G.nx), iy = (int)((j / G.nx) % G.ny), iz = (int)(j / ((int64_t)G.nx * G.ny));
        voxel_view_weights(G, view, ix, iy, iz, tau_keep, want32, [&](int64_t i, double w, float w32) {
            const int64_t pos = row_ptr[i] + atomicAdd(&cursor[i], 1);
            cols[pos] = (int32_t)j;
            vals[pos] = want32 ? (V)w32 : (V)w;
        });
    }
}

// Rows of W^T (one per voxel): entry counts per voxel, one atomic per
// (view, voxel) work-item.
__global__ void csr_count_vox_kernel(DevGeom G, double tau_keep, int32_t *vox_cnt)
{
    const int64_t nvox = (int64_t)G.nx * G.ny * G.nz;
    const int64_t n = nvox * G.n_p;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int view = (int)(q / nvox);
        const int64_t j = q - (int64_t)view * nvox;
        const int ix = (int)(j % G.nx), iy = (int)((j / G.nx) % G.ny), iz = (int)(j / ((int64_t)G.nx * G.ny));
        int c = 0;
        voxel_view_weights(G, view, ix, iy, iz, tau_keep, false, [&](int64_t, double, float) { ++c; });
        if (c > 0) atomicAdd(&vox_cnt[j], c);
    }
}

// Fill the rows of W^T (column = detector element); the order within a row
// is settled by the segmented sort that follows.
template <typename V>
__global__ void csr_fill_vox_kernel(DevGeom G, double tau_keep, const int64_t *row_ptr,
                                    int32_t *cursor, int32_t *cols, V *vals)
{
    const int64_t nvox = (int64_t)G.nx * G.ny * G.nz;
    const int64_t n = nvox * G.n_p;
    const bool want32 = sizeof(V) == 4;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int view = (int)(q / nvox);
        const int64_t j = q - (int64_t)view * nvox;
        const int ix = (int)(j % G.nx), iy = (int)((j / G.nx) % G.ny), iz = (int)(j / ((int64_t)G.nx * G.ny));
        voxel_view_weights(G, view, ix, iy, iz, tau_keep, want32, [&](int64_t i, double w, float w32) {
            const int64_t pos = row_ptr[j] + atomicAdd(&cursor[j], 1);
            cols[pos] = (int32_t)i;
            vals[pos] = want32 ? (V)w32 : (V)w;
        });
    }
}

template <typename V>
__global__ void csr_sort_kernel(const int64_t *row_ptr, int64_t n_rows, int32_t *cols, V *vals)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_rows;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = row_ptr[i], e = row_ptr[i + 1];
        for (int64_t p = a + 1; p < e; ++p) {
            const int32_t c = cols[p];
            const V v = vals[p];
            int64_t q = p - 1;
            while (q >= a && cols[q] > c) {
                cols[q + 1] = cols[q];
                vals[q + 1] = vals[q];
                --q;
            }
            cols[q + 1] = c;
            vals[q + 1] = v;
        }
    }
}

// row_ptr[0] = 0, row_ptr[i + 1] = cnt[0] + ... + cnt[i]; one workgroup.
__global__ void __launch_bounds__(1024) scan_kernel(const int32_t *cnt, int64_t n, int64_t *row_ptr)
{
    __shared__ int64_t part[1024];
    __shared__ int64_t carry;
    const int tid = threadIdx.x;
    if (tid == 0) {
        carry = 0;
        row_ptr[0] = 0;
    }
    __syncthreads();
    for (int64_t base = 0; base < n; base += 1024) {
        const int64_t i = base + tid;
        part[tid] = i < n ? (int64_t)cnt[i] : 0;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int64_t t = tid >= o ? part[tid - o] : 0;
            __syncthreads();
            part[tid] += t;
            __syncthreads();
        }
        if (i < n) row_ptr[i + 1] = carry + part[tid];
        __syncthreads();
        if (tid == 1023) carry += part[1023];
        __syncthreads();
    }
}

static dim3 stride_grid(int64_t n, int threads)
{
    const int64_t want = (n + threads - 1) / threads;
    return dim3((unsigned)(want < (1 << 20) ? (want > 0 ? want : 1) : (1 << 20)));
}

hipError_t launch_csr_count(const DevGeom &G, double tau_keep, int32_t *row_cnt, hipStream_t st)
{
    const int64_t n = (int64_t)G.nx * G.ny * G.nz * G.n_p;
    hipLaunchKernelGGL(csr_count_kernel, stride_grid(n, 128), dim3(128), 0, st, G, tau_keep,
                       row_cnt);
    return hipGetLastError();
}

hipError_t launch_csr_fill(const DevGeom &G, bool fp64_vals, double tau_keep,
                           const int64_t *row_ptr, int32_t *cursor, int32_t *cols, void *vals,
                           hipStream_t st)
{
    const int64_t n = (int64_t)G.nx * G.ny * G.nz * G.n_p;
    const dim3 grid = stride_grid(n, 128);
    if (fp64_vals)
        hipLaunchKernelGGL(csr_fill_kernel<double>, grid, dim3(128), 0, st, G, tau_keep, row_ptr,
                           cursor, cols, (double *)vals);
    else
        hipLaunchKernelGGL(csr_fill_kernel<float>, grid, dim3(128), 0, st, G, tau_keep, row_ptr,
                           cursor, cols, (float *)vals);
    return hipGetLastError();
}

hipError_t launch_csr_count_vox(const DevGeom &G, double tau_keep, int32_t *vox_cnt, hipStream_t st)
{
    const int64_t n = (int64_t)G.nx * G.ny * G.nz * G.n_p;
    hipLaunchKernelGGL(csr_count_vox_kernel, stride_grid(n, 128), dim3(128), 0, st, G, tau_keep,
                       vox_cnt);
    return hipGetLastError();
}

hipError_t launch_csr_fill_vox(const DevGeom &G, bool fp64_vals, double tau_keep,
                               const int64_t *row_ptr, int32_t *cursor, int32_t *cols, void *vals,
                               hipStream_t st)
{
    const int64_t n = (int64_t)G.nx * G.ny * G.nz * G.n_p;
    const dim3 grid = stride_grid(n, 128);
    if (fp64_vals)
        hipLaunchKernelGGL(csr_fill_vox_kernel<double>, grid, dim3(128), 0, st, G, tau_keep,
                           row_ptr, cursor, cols, (double *)vals);
    else
        hipLaunchKernelGGL(csr_fill_vox_kernel<float>, grid, dim3(128), 0, st, G, tau_keep,
                           row_ptr, cursor, cols, (float *)vals);
    return hipGetLastError();
}

hipError_t launch_csr_sort(const int64_t *row_ptr, int64_t n_rows, int32_t *cols, void *vals,
                           bool fp64_vals, hipStream_t st)
{
    const dim3 grid = stride_grid(n_rows, 128);
    if (fp64_vals)
        hipLaunchKernelGGL(csr_sort_kernel<double>, grid, dim3(128), 0, st, row_ptr, n_rows, cols,
                           (double *)vals);
    else
        hipLaunchKernelGGL(csr_sort_kernel<float>, grid, dim3(128), 0, st, row_ptr, n_rows, cols,
                           (float *)vals);
    return hipGetLastError();
}

hipError_t launch_scan_counts(const int32_t *cnt, int64_t n, int64_t *row_ptr, hipStream_t st)
{
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, cnt, n, row_ptr);
    return hipGetLastError();
}

}  // namespace smk
