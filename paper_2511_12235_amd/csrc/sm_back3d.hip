// sm_back3d.hip -- cone-beam adjoint x = W^T y with the forward's weights.
//
// Voxel-stationary gather, no atomics: a workgroup owns a TX x TY tile of
// pixels and every voxel above them (one lane per z index), loops over all
// views and keeps the tile's sums in registers.  Per view:
//   1. the detector columns each pixel can meet are found, and the union of
//      those columns (all rows, zero-padded above and below) is staged in LDS;
//   2. the strip records of every (pixel, column) pair are built in FP64, one
//      thread each, into LDS;
//   3. lane iz finds the row planes p_first..p_last that cut its voxel inside
//      the strip and adds, with the cumulative sub-volume H_p below plane p,
//          c A y[p_last] + sum_p H_p (y[p-1] - y[p])
//      which is  sum_r (H_{r+1} - H_r) y[r]  summed by parts over the rows.
// The tile's sums are written once to the z-contiguous workspace and
// transposed to the caller's layout afterwards.
#include "sm_internal.h"

namespace smk {

template <typename T, int NBAT, int TX, int TY>
__global__ void __launch_bounds__(1024)
back3d_kernel(DevGeom G, const T *__restrict__ y, T *__restrict__ xt, int B, int b0, int pcols,
              int rmax)
{
    constexpr int TP = TX * TY;
    extern __shared__ __align__(16) unsigned char smem[];
    const int nthr = blockDim.x, tid = threadIdx.x;
    const int nz = G.nz, nv = G.nv;

    // LDS layout
    Rec<T> *rec = reinterpret_cast<Rec<T> *>(smem);
    size_t off = sizeof(Rec<T>) * rmax;
    double *ptau = reinterpret_cast<double *>(smem + off);
    off += sizeof(double) * (nv + 1);
    T *pat = reinterpret_cast<T *>(smem + off);
    off += sizeof(T) * (nv + 1);
    T *pinv = reinterpret_cast<T *>(smem + off);
    off += sizeof(T) * (nv + 1);
    off = (off + 15) & ~(size_t)15;
    T *patch = reinterpret_cast<T *>(smem + off);
    off += sizeof(T) * (size_t)NBAT * pcols * (nv + 2);
    off = (off + 15) & ~(size_t)15;
    int *pk0 = reinterpret_cast<int *>(smem + off);
    int *poffs = pk0 + TP;       // TP + 1
    int *pspan = poffs + TP + 1; // kmin, kmax

    for (int p = tid; p <= nv; p += nthr) {
        const double t = G.tau[p];
        ptau[p] = t;
        pat[p] = T(fabs(t));
        pinv[p] = fabs(t) > 0.0 ? T(1) / T(fabs(t)) : T(0);
    }

    const int ntx = (G.nx + TX - 1) / TX;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int tyi = lb / ntx, txi = lb - tyi * ntx;
    const int ix0 = txi * TX, iy0 = tyi * TY;

    const int iz = tid;
    const bool active = iz < nz;
    const double za = G.z0 + (double)iz * G.c;
    const double zb = za + G.c;
    const T cT = T(G.c);
    const double inv_dv = 1.0 / G.dv;
    const int rowstride = nv + 2;

    T acc[TP][NBAT];
#pragma unroll
    for (int p = 0; p < TP; ++p)
#pragma unroll
        for (int b = 0; b < NBAT; ++b) acc[p][b] = T(0);

    for (int view = 0; view < G.n_p; ++view) {
        const double2 cs = view_trig(G, view);
        const double cp = cs.x, sp = cs.y;
        __syncthreads();  // previous view's records and patch are consumed
        // --- detector columns per pixel
        if (tid < TP) {
            const int ix = ix0 + tid % TX, iy = iy0 + tid / TX;
            int k0 = 0, k1 = -1;
            if (ix < G.nx && iy < G.ny) pixel_columns(G, cp, sp, ix, iy, k0, k1);
            pk0[tid] = k0;
            poffs[tid + 1] = k1 >= k0 ? k1 - k0 + 1 : 0;
        }
        __syncthreads();
        if (tid == 0) {
            int run = 0, kmin = 1 << 30, kmax = -1;
            poffs[0] = 0;
            for (int p = 0; p < TP; ++p) {
                const int c = poffs[p + 1];
                if (c > 0) {
                    kmin = min(kmin, pk0[p]);
                    kmax = max(kmax, pk0[p] + c - 1);
                }
                run += c;
                poffs[p + 1] = run;
            }
            if (kmax >= 0 && kmax - kmin + 1 > pcols) kmax = kmin + pcols - 1;  // bound from the plan
            pspan[0] = kmin;
            pspan[1] = kmax;
        }
        __syncthreads();
        const int total = poffs[TP];
        if (total == 0) continue;
        const int kmin = pspan[0], kmax = pspan[1];
        const int pc = kmax - kmin + 1;
        // --- stage y[view][:, kmin..kmax] with zero rows at -1 and nv
        {
            const float inv_pc = 1.0f / (float)pc;
            const int per_b = pc * nv;
            for (int bb = 0; bb < NBAT; ++bb) {
                const T *src = y + ((size_t)(b0 + bb) * G.n_p + view) * nv * G.nu;
                T *dst = patch + (size_t)bb * pcols * rowstride;
                for (int q = tid; q < per_b; q += nthr) {
                    const int row = (int)(((float)q + 0.5f) * inv_pc);
                    const int col = q - row * pc;
                    dst[col * rowstride + row + 1] = src[(size_t)row * G.nu + kmin + col];
                }
                for (int col = tid; col < pc; col += nthr) {
                    dst[col * rowstride] = T(0);
                    dst[col * rowstride + nv + 1] = T(0);
                }
            }
        }
        // --- strip records, in rounds of rmax
        for (int rr = 0; rr < total; rr += rmax) {
            const int ne = min(rmax, total - rr);
            if (tid < ne) {
                const int e = rr + tid;
                int p = 0;
                while (p + 1 < TP && poffs[p + 1] <= e) ++p;
                const int ix = ix0 + p % TX, iy = iy0 + p / TX;
                build_record<T>(G, cp, sp, ix, iy, pk0[p] + (e - poffs[p]), rec[tid]);
                rec[tid].pix = p;
            }
            __syncthreads();
            if (active) {
#pragma unroll
                for (int p = 0; p < TP; ++p) {
                    const int e0 = max(poffs[p], rr), e1 = min(poffs[p + 1], rr + ne);
                    for (int e = e0; e < e1; ++e) {
                        const Rec<T> &R = rec[e - rr];
                        if (R.n == 0) continue;
                        const int col = R.k - kmin;
                        if (col < 0 || col >= pc) continue;
                        // row planes cutting the voxel inside the strip
                        const double tst = za >= 0.0 ? za * R.ilmax : za * R.ilmin;
                        int pf = (int)fmin(fmax(floor((tst * G.D - G.v0) * inv_dv) + 1.0, 0.0),
                                           (double)(nv + 1));
                        while (pf > 0) {
                            const double t = ptau[pf - 1];
                            if (t * (t >= 0.0 ? R.lmax : R.lmin) > za) --pf; else break;
                        }
                        while (pf <= nv) {
                            const double t = ptau[pf];
                            if (!(t * (t >= 0.0 ? R.lmax : R.lmin) > za)) ++pf; else break;
                        }
                        const double tss = zb >= 0.0 ? zb * R.ilmin : zb * R.ilmax;
                        int pl = (int)fmin(fmax(ceil((tss * G.D - G.v0) * inv_dv) - 1.0, -1.0),
                                           (double)nv);
                        while (pl < nv) {
                            const double t = ptau[pl + 1];
                            if (t * (t >= 0.0 ? R.lmin : R.lmax) < zb) ++pl; else break;
                        }
                        while (pl >= 0) {
                            const double t = ptau[pl];
                            if (!(t * (t >= 0.0 ? R.lmin : R.lmax) < zb)) --pl; else break;
                        }
                        const T cA = cT * R.area;
                        const T *Y = patch + (size_t)col * rowstride + 1;  // Y[-1] .. Y[nv]
                        T sum[NBAT];
#pragma unroll
                        for (int b = 0; b < NBAT; ++b)
                            sum[b] = (pl >= 0 && pl < nv) ? cA * Y[(size_t)b * pcols * rowstride + pl]
                                                          : T(0);
                        for (int q = pf; q <= pl; ++q) {
                            const double t = ptau[q];
                            const T e = T(t * R.lc - za);
                            const T Hv = eval_H<T>(R, t < 0.0, pat[q], pinv[q], e, cT);
#pragma unroll
                            for (int b = 0; b < NBAT; ++b) {
                                const T *Yb = Y + (size_t)b * pcols * rowstride;
                                sum[b] += Hv * (Yb[q - 1] - Yb[q]);
                            }
                        }
#pragma unroll
                        for (int b = 0; b < NBAT; ++b) acc[p][b] += sum[b];
                    }
                }
            }
            __syncthreads();
        }
    }

    if (active) {
#pragma unroll
        for (int p = 0; p < TP; ++p) {
            const int ix = ix0 + p % TX, iy = iy0 + p / TX;
            if (ix < G.nx && iy < G.ny) {
                const size_t pix = (size_t)iy * G.nx + ix;
#pragma unroll
                for (int b = 0; b < NBAT; ++b) xt[(pix * B + b0 + b) * nz + iz] = acc[p][b];
            }
        }
    }
}

template <typename T, int NBAT, int TX, int TY>
static size_t back3d_lds(const DevGeom &G, const LaunchCfg &L, int slot)
{
    size_t lds = sizeof(Rec<T>) * L.back_rmax + sizeof(double) * (G.nv + 1) + 2 * sizeof(T) * (G.nv + 1);
    lds = (lds + 15) & ~(size_t)15;
    lds += sizeof(T) * (size_t)NBAT * L.back_pcols[slot] * (G.nv + 2);
    lds = (lds + 15) & ~(size_t)15;
    lds += sizeof(int) * (2 * TX * TY + 3);
    return lds;
}

template <typename T, int NBAT, int TX, int TY>
static hipError_t launch_back3d_t(const DevGeom &G, const LaunchCfg &L, int slot, const T *y,
                                  T *xt, int B, int b0, hipStream_t st)
{
    const size_t lds = back3d_lds<T, NBAT, TX, TY>(G, L, slot);
    if (lds > (size_t)L.lds_budget) return hipErrorInvalidValue;
    const int ntx = (G.nx + TX - 1) / TX, nty = (G.ny + TY - 1) / TY;
    hipLaunchKernelGGL((back3d_kernel<T, NBAT, TX, TY>), dim3(ntx * nty), dim3(L.back_threads), lds,
                       st, G, y, xt, B, b0, L.back_pcols[slot], L.back_rmax);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_back3d_all(const DevGeom &G, const LaunchCfg &L, const T *y, T *xt, int B,
                                    hipStream_t st)
{
    const size_t bud = (size_t)L.lds_budget;
    const bool fit8 = back3d_lds<T, 8, 2, 1>(G, L, 3) <= bud;
    const bool fit4 = back3d_lds<T, 4, 2, 2>(G, L, 2) <= bud;
    const bool fit2 = back3d_lds<T, 2, 4, 2>(G, L, 1) <= bud;
    hipError_t e = hipSuccess;
    for (int b0 = 0; b0 < B && e == hipSuccess;) {
        const int rem = B - b0;
        if (rem >= 8 && fit8) { e = launch_back3d_t<T, 8, 2, 1>(G, L, 3, y, xt, B, b0, st); b0 += 8; }
        else if (rem >= 4 && fit4) { e = launch_back3d_t<T, 4, 2, 2>(G, L, 2, y, xt, B, b0, st); b0 += 4; }
        else if (rem >= 2 && fit2) { e = launch_back3d_t<T, 2, 4, 2>(G, L, 1, y, xt, B, b0, st); b0 += 2; }
        else { e = launch_back3d_t<T, 1, 4, 4>(G, L, 0, y, xt, B, b0, st); b0 += 1; }
    }
    return e;
}

hipError_t launch_back3d(const DevGeom &G, const LaunchCfg &L, bool fp64, const void *y, void *xt,
                         int B, hipStream_t st)
{
    if (fp64) return launch_back3d_all<double>(G, L, (const double *)y, (double *)xt, B, st);
    return launch_back3d_all<float>(G, L, (const float *)y, (float *)xt, B, st);
}

}  // namespace smk
