// sm_fwd3d.hip -- cone-beam forward projection y = W x (Sec. III-C).
//
// The paper's Algorithm 1 scatters each voxel into the detector elements it
// meets.  On the GPU that would need atomics, so the loop is turned inside
// out: one workgroup owns one (view, detector column k) and accumulates every
// row of that column in registers, one lane per detector row.
//
//   1. The pixels (top-view columns of voxels) that the wedge of column k can
//      meet are enumerated along the major axis; each workgroup pass takes up
//      to NB of them and builds their strip records (sm_common.h) in FP64,
//      one thread per pixel, into LDS.
//   2. The voxel columns of those pixels (z-contiguous copies, see
//      sm_transpose.hip) are staged in LDS.
//   3. Lane r owns row r and its lower plane r.  For a pixel with strip area
//      A and voxel height c, the contribution to row r is
//          c A * sum_{iz in [f_r, f_{r+1})} x_iz  +  G_{r+1} - G_r,
//      G_p = sum over voxels cut by plane p of x_iz * H_iz(p), where f_p is
//      the first voxel not entirely below plane p and H the cumulative
//      sub-volume below the plane.  Lane r accumulates  c A R - G_r  and G_r
//      separately; the G of the plane above is added once at the end through
//      LDS.  The top detector edge (plane nv) has no lane; its G is computed
//      by the thread that built each pixel's record.
//
// Every weight is evaluated once per call and applied to NBAT batch elements.
#include "sm_internal.h"

namespace smk {

// Block-wide exclusive scan of one int per thread (blockDim.x <= 1024).
__device__ int block_exclusive_scan(int v, int *tmp, int &total)
{
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = (blockDim.x + 63) >> 6;
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) tmp[wid] = incl;
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int w = 0; w < nw; ++w) {
            int t = tmp[w];
            tmp[w] = run;
            run += t;
        }
        tmp[nw] = run;
    }
    __syncthreads();
    const int excl = tmp[wid] + incl - v;
    total = tmp[nw];
    __syncthreads();
    return excl;
}

template <typename T, int NBAT>
__device__ __forceinline__ void plane_range(const DevGeom &G, double tau, const Rec<T> &R,
                                            double inv_c, int &f, int &l)
{
    const double llo = tau < 0.0 ? R.lmax : R.lmin;
    const double lhi = tau < 0.0 ? R.lmin : R.lmax;
    const double lo_abs = tau * llo, hi_abs = tau * lhi;
    f = (int)fmin(fmax(floor((lo_abs - G.z0) * inv_c), 0.0), (double)G.nz);
    l = (int)fmin(fmax(floor((hi_abs - G.z0) * inv_c), -1.0), (double)(G.nz - 1));
}

template <typename T, int NBAT>
__global__ void __launch_bounds__(1024)
fwd3d_kernel(DevGeom G, const T *__restrict__ xt, T *__restrict__ y, int B, int b0, int NB)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int nthr = blockDim.x, tid = threadIdx.x;
    const int nz = G.nz, nv = G.nv;

    // LDS layout
    Rec<T> *rec = reinterpret_cast<Rec<T> *>(smem);
    T *xs = reinterpret_cast<T *>(smem + sizeof(Rec<T>) * NB);
    int *jstart = reinterpret_cast<int *>(smem + sizeof(Rec<T>) * NB + sizeof(T) * NB * NBAT * nz);
    int *offs = jstart + nthr;
    int *scan_tmp = offs + nthr + 1;

    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int view = lb / G.nu, k = lb - view * G.nu;
    const double2 cs = view_trig(G, view);
    const double cp = cs.x, sp = cs.y;
    const double ulo = G.u0 + (double)k * G.du, uhi = G.u0 + (double)(k + 1) * G.du;
    const double inv_c = 1.0 / G.c;
    const T cT = T(G.c);

    // per-lane plane constants (lane r: plane r is the lower edge of row r)
    const int r = tid;
    const bool active = r < nv;
    const double tau0 = active ? G.tau[r] : 0.0;
    const double tau1 = active ? G.tau[r + 1] : 0.0;
    const int sg0 = tau0 < 0.0;
    const T at0 = T(fabs(tau0));
    const T inv0 = at0 > T(0) ? T(1) / at0 : T(0);
    // top detector edge (plane nv), evaluated per pixel by the record builder
    const double tauT = G.tau[nv];
    const int sgT = tauT < 0.0;
    const T atT = T(fabs(tauT));
    const T invT = atT > T(0) ? T(1) / atT : T(0);

    T acc1[NBAT], acc2[NBAT], accT[NBAT];
#pragma unroll
    for (int b = 0; b < NBAT; ++b) acc1[b] = acc2[b] = accT[b] = T(0);

    const StripAxis ax = strip_axis(G, cp, sp);
    for (int base = 0; base < ax.n_major; base += nthr) {
        // --- enumerate the pixels of this chunk of major cells
        const int im = base + tid;
        int cnt = 0, j0 = 0, j1 = -1;
        if (im < ax.n_major) {
            strip_minor_range(G, ax, cp, sp, ulo, uhi, im, j0, j1);
            cnt = j1 >= j0 ? j1 - j0 + 1 : 0;
        }
        jstart[tid] = j0;
        int total;
        const int ex = block_exclusive_scan(cnt, scan_tmp, total);
        offs[tid] = ex;
        if (tid == 0) offs[nthr] = total;
        __syncthreads();

        for (int g0 = 0; g0 < total; g0 += NB) {
            const int ne = min(NB, total - g0);
            // --- strip records, one thread per pixel
            if (tid < ne) {
                const int e = g0 + tid;
                int lo = 0, hi = nthr;  // largest m with offs[m] <= e
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (offs[mid] <= e) lo = mid; else hi = mid;
                }
                const int mj = base + lo;
                const int mn = jstart[lo] + (e - offs[lo]);
                const int ix = ax.major_x ? mj : mn;
                const int iy = ax.major_x ? mn : mj;
                build_record<T>(G, cp, sp, ix, iy, k, rec[tid]);
                rec[tid].pix = iy * G.nx + ix;
            }
            __syncthreads();
            // --- stage the voxel columns of these pixels
            for (int tb = 0; tb < ne * NBAT; ++tb) {
                const int t = tb / NBAT, bb = tb - t * NBAT;
                const T *src = xt + ((size_t)rec[t].pix * B + b0 + bb) * nz;
                T *dst = xs + (size_t)tb * nz;
                for (int iz = tid; iz < nz; iz += nthr) dst[iz] = src[iz];
            }
            __syncthreads();
            // --- top detector edge: G of plane nv for this thread's pixel
            if (tid < ne && rec[tid].n > 0) {
                const Rec<T> &R = rec[tid];
                int f, l;
                plane_range<T, NBAT>(G, tauT, R, inv_c, f, l);
                const double hz = tauT * R.lc - G.z0;
                const T *xp = xs + (size_t)tid * NBAT * nz;
                for (int iz = f; iz <= l; ++iz) {
                    const T e = T(hz - (double)iz * G.c);
                    const T Hv = eval_H<T>(R, sgT, atT, invT, e, cT);
#pragma unroll
                    for (int b = 0; b < NBAT; ++b) accT[b] += xp[b * nz + iz] * Hv;
                }
            }
            // --- rows: lane r, every pixel of the pass
            if (active) {
                for (int t = 0; t < ne; ++t) {
                    const Rec<T> &R = rec[t];
                    if (R.n == 0) continue;
                    int f, l, f1, l1;
                    plane_range<T, NBAT>(G, tau0, R, inv_c, f, l);
                    plane_range<T, NBAT>(G, tau1, R, inv_c, f1, l1);
                    const int iend = max(l, f1 - 1);
                    const double hz = tau0 * R.lc - G.z0;
                    const T cA = cT * R.area;
                    const T *xp = xs + (size_t)t * NBAT * nz;
                    T rs[NBAT], gs[NBAT];
#pragma unroll
                    for (int b = 0; b < NBAT; ++b) rs[b] = gs[b] = T(0);
                    for (int iz = f; iz <= iend; ++iz) {
                        T xv[NBAT];
#pragma unroll
                        for (int b = 0; b < NBAT; ++b) xv[b] = xp[b * nz + iz];
                        if (iz < f1) {
#pragma unroll
                            for (int b = 0; b < NBAT; ++b) rs[b] += xv[b];
                        }
                        if (iz <= l) {
                            const T e = T(hz - (double)iz * G.c);
                            const T Hv = eval_H<T>(R, sg0, at0, inv0, e, cT);
#pragma unroll
                            for (int b = 0; b < NBAT; ++b) gs[b] += xv[b] * Hv;
                        }
                    }
#pragma unroll
                    for (int b = 0; b < NBAT; ++b) {
                        acc1[b] += cA * rs[b] - gs[b];
                        acc2[b] += gs[b];
                    }
                }
            }
            __syncthreads();
        }
    }

    // --- y_r = acc1_r + acc2_{r+1}; acc2_nv is the sum of accT over threads
    T *ex = reinterpret_cast<T *>(smem);  // (nthr + 1) * NBAT, reuses the record area
    T *red = ex + (size_t)(nthr + 1) * NBAT;
#pragma unroll
    for (int b = 0; b < NBAT; ++b) {
        ex[tid * NBAT + b] = acc2[b];
        red[tid * NBAT + b] = accT[b];
    }
    __syncthreads();
    for (int w = 1; w < nthr; w <<= 1) {  // fixed-order tree reduction of accT
        if ((tid & (2 * w - 1)) == 0 && tid + w < nthr) {
#pragma unroll
            for (int b = 0; b < NBAT; ++b) red[tid * NBAT + b] += red[(tid + w) * NBAT + b];
        }
        __syncthreads();
    }
    if (tid == 0) {
#pragma unroll
        for (int b = 0; b < NBAT; ++b) ex[nv * NBAT + b] = red[b];
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int b = 0; b < NBAT; ++b) {
            const size_t o = (((size_t)(b0 + b) * G.n_p + view) * nv + r) * G.nu + k;
            y[o] = acc1[b] + ex[(r + 1) * NBAT + b];
        }
    }
}

template <typename T, int NBAT>
static size_t fwd3d_lds(const DevGeom &G, const LaunchCfg &L, int &NB)
{
    const int nthr = L.fwd_threads;
    // pixels per pass: staged columns near 32 KiB, records + columns within budget
    const size_t fixed = sizeof(int) * (2 * (size_t)nthr + 1 + 20);
    const size_t per_pix = sizeof(Rec<T>) + sizeof(T) * (size_t)NBAT * G.nz;
    NB = (int)(32768 / ((size_t)sizeof(T) * NBAT * G.nz));
    const int nb_fit = L.lds_budget > (int)fixed ? (int)(((size_t)L.lds_budget - fixed) / per_pix) : 0;
    NB = NB > nb_fit ? nb_fit : NB;
    NB = NB < 1 ? 1 : (NB > 64 ? 64 : NB);
    if (NB > nthr) NB = nthr;
    size_t lds = per_pix * NB + fixed;
    const size_t lds_end = sizeof(T) * (size_t)(2 * nthr + 2) * NBAT;  // exchange + reduction
    return lds_end > lds ? lds_end : lds;
}

template <typename T, int NBAT>
static hipError_t launch_fwd3d_t(const DevGeom &G, const LaunchCfg &L, const T *xt, T *y, int B,
                                 int b0, hipStream_t st)
{
    int NB;
    const size_t lds = fwd3d_lds<T, NBAT>(G, L, NB);
    if (lds > (size_t)L.lds_budget) return hipErrorInvalidValue;
    const int nblk = G.n_p * G.nu;
    hipLaunchKernelGGL((fwd3d_kernel<T, NBAT>), dim3(nblk), dim3(L.fwd_threads), lds, st, G, xt, y,
                       B, b0, NB);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_fwd3d_all(const DevGeom &G, const LaunchCfg &L, const T *xt, T *y, int B,
                                   hipStream_t st)
{
    int nb;
    const size_t bud = (size_t)L.lds_budget;
    const bool fit8 = fwd3d_lds<T, 8>(G, L, nb) <= bud;
    const bool fit4 = fwd3d_lds<T, 4>(G, L, nb) <= bud;
    const bool fit2 = fwd3d_lds<T, 2>(G, L, nb) <= bud;
    hipError_t e = hipSuccess;
    for (int b0 = 0; b0 < B && e == hipSuccess;) {
        const int rem = B - b0;
        if (rem >= 8 && fit8) { e = launch_fwd3d_t<T, 8>(G, L, xt, y, B, b0, st); b0 += 8; }
        else if (rem >= 4 && fit4) { e = launch_fwd3d_t<T, 4>(G, L, xt, y, B, b0, st); b0 += 4; }
        else if (rem >= 2 && fit2) { e = launch_fwd3d_t<T, 2>(G, L, xt, y, B, b0, st); b0 += 2; }
        else { e = launch_fwd3d_t<T, 1>(G, L, xt, y, B, b0, st); b0 += 1; }
    }
    return e;
}

hipError_t launch_fwd3d(const DevGeom &G, const LaunchCfg &L, bool fp64, const void *xt, void *y,
                        int B, hipStream_t st)
{
    if (fp64) return launch_fwd3d_all<double>(G, L, (const double *)xt, (double *)y, B, st);
    return launch_fwd3d_all<float>(G, L, (const float *)xt, (float *)y, B, st);
}

}  // namespace smk
