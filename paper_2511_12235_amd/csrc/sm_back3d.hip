// sm_back3d.hip -- cone-beam adjoint x = W^T y with the forward's weights.
//
// Voxel-stationary gather, no atomics: a workgroup owns a TX x TY tile of
// pixels and every voxel above them (one lane per z index) and keeps the
// tile's sums in registers while it loops over the views of a chunk.  Per
// view it stages the detector columns the tile can meet (all rows, with a zero
// row above and below) in LDS, then for every (pixel, column) strip record
// (built by sm_rec.hip, found through the strip's per-major table and read
// with scalar loads) lane iz finds the row planes p_first..p_last that cut its
// voxel inside the strip and adds
//     c A y[p_last] + sum_p H_p (y[p-1] - y[p]),   H_p = K_p(za) - K_p(zb),
// which is  sum_r (H_{r+1} - H_r) y[r]  summed by parts over the rows; H_p is
// the volume of the voxel below plane p (sm_common.h).  Chunks of views add
// into the z-contiguous workspace in a fixed order, which is transposed to the
// caller's layout afterwards.
#include "sm_internal.h"

namespace smk {

template <typename T, int NBAT, int TX, int TY>
__global__ void __launch_bounds__(1024)
back3d_kernel(DevGeom G, RecLayout RL, int v0, int nvc, const Rec<T> *__restrict__ recs,
              const int *__restrict__ sj0, const int *__restrict__ soff,
              const int2 *__restrict__ pixk, const T *__restrict__ y, T *__restrict__ xt, int B,
              int b0, int pcols, int first)
{
    constexpr int TP = TX * TY;
    extern __shared__ __align__(16) unsigned char smem[];
    const int nthr = blockDim.x, tid = threadIdx.x;
    const int nz = G.nz, nv = G.nv;
    const int rowstride = nv + 2;

    double *ptau = reinterpret_cast<double *>(smem);
    T *ptf = reinterpret_cast<T *>(smem + sizeof(double) * (nv + 1));
    T *pinv = ptf + (nv + 1);
    size_t off = sizeof(double) * (nv + 1) + 2 * sizeof(T) * (nv + 1);
    off = (off + 15) & ~(size_t)15;
    T *patch = reinterpret_cast<T *>(smem + off);

    for (int p = tid; p <= nv; p += nthr) {
        const double t = G.tau[p];
        ptau[p] = t;
        ptf[p] = T(t);
        pinv[p] = t != 0.0 ? T(1) / T(t) : T(0);
    }

    const int ntx = (G.nx + TX - 1) / TX;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int tyi = lb / ntx, txi = lb - tyi * ntx;
    const int ix0 = txi * TX, iy0 = tyi * TY;
    const int npix = G.nx * G.ny;

    const int iz = tid;
    const bool active = iz < nz;
    const double za = G.z0 + (double)iz * G.c;
    const double zb = za + G.c;
    const float fza = (float)za, fzb = (float)zb;
    const T cT = T(G.c);
    const float inv_dv = (float)(1.0 / G.dv);
    const float fD = (float)G.D, fv0 = (float)G.v0;

    T acc[TP][NBAT];
#pragma unroll
    for (int p = 0; p < TP; ++p)
#pragma unroll
        for (int b = 0; b < NBAT; ++b) acc[p][b] = T(0);

    for (int vl = 0; vl < nvc; ++vl) {
        const int view = v0 + vl;
        const double2 cs = G.trig[view];
        const StripAxis ax = strip_axis(G, cs.x, cs.y);
        // detector columns of the tile's pixels (from the record pass)
        int kk0[TP], kk1[TP];
        int kmin = 1 << 30, kmax = -1;
#pragma unroll
        for (int p = 0; p < TP; ++p) {
            const int ix = ix0 + p % TX, iy = iy0 + p / TX;
            kk0[p] = 0;
            kk1[p] = -1;
            if (ix < G.nx && iy < G.ny) {
                const int2 q = pixk[(size_t)vl * npix + (size_t)iy * G.nx + ix];
                kk0[p] = q.x;
                kk1[p] = q.y;
                if (q.y >= q.x) {
                    kmin = min(kmin, q.x);
                    kmax = max(kmax, q.y);
                }
            }
        }
        if (kmax < kmin) continue;
        if (kmax - kmin + 1 > pcols) kmax = kmin + pcols - 1;  // bound from the plan
        const int pc = kmax - kmin + 1;
        __syncthreads();  // previous view's patch is consumed
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
        __syncthreads();
        if (!active) continue;
#pragma unroll
        for (int p = 0; p < TP; ++p) {
            const int ix = ix0 + p % TX, iy = iy0 + p / TX;
            for (int k = max(kk0[p], kmin); k <= min(kk1[p], kmax); ++k) {
                const int64_t strip = (int64_t)vl * G.nu + k;
                const int pos = strip_position(ax.major_x, ix, iy, sj0 + strip * RL.n_major_max,
                                               soff + strip * (RL.n_major_max + 1));
                if (pos < 0) continue;
                const Rec<T> &R = recs[strip * RL.cap + pos];
                const int n = R.n;
                if (n == 0) continue;
                const double lmin = R.lc + (double)R.tab[0][0];
                const double lmax = R.lc + (double)R.tab[n - 1][0];
                // row planes cutting the voxel inside the strip: estimate the
                // index where a plane's highest point reaches za (lowest point
                // reaches zb), then settle it with exact FP64 comparisons
                const float tst = fza / (float)(za >= 0.0 ? lmax : lmin);
                int pf = (int)fminf(fmaxf(floorf((tst * fD - fv0) * inv_dv) + 1.0f, 0.0f), (float)(nv + 1));
                while (pf > 0) {
                    const double t = ptau[pf - 1];
                    if (t * (t >= 0.0 ? lmax : lmin) > za) --pf; else break;
                }
                while (pf <= nv) {
                    const double t = ptau[pf];
                    if (!(t * (t >= 0.0 ? lmax : lmin) > za)) ++pf; else break;
                }
                const float tss = fzb / (float)(zb >= 0.0 ? lmin : lmax);
                int pl = (int)fminf(fmaxf(ceilf((tss * fD - fv0) * inv_dv) - 1.0f, -1.0f), (float)nv);
                while (pl < nv) {
                    const double t = ptau[pl + 1];
                    if (t * (t >= 0.0 ? lmin : lmax) < zb) ++pl; else break;
                }
                while (pl >= 0) {
                    const double t = ptau[pl];
                    if (!(t * (t >= 0.0 ? lmin : lmax) < zb)) --pl; else break;
                }
                const T cA = cT * R.tab[0][2];
                const T *Y = patch + (size_t)(k - kmin) * rowstride + 1;  // Y[-1] .. Y[nv]
                T sum[NBAT];
#pragma unroll
                for (int b = 0; b < NBAT; ++b)
                    sum[b] = (pl >= 0 && pl < nv) ? cA * Y[(size_t)b * pcols * rowstride + pl] : T(0);
                for (int q = pf; q <= pl; ++q) {
                    const double ea = ptau[q] * R.lc - za;
                    const T Ha = eval_K<T>(R.tab, n, ptf[q], pinv[q], T(ea));
                    const T Hb = eval_K<T>(R.tab, n, ptf[q], pinv[q], T(ea - G.c));
                    const T Hv = Ha - Hb;
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

    if (active) {
#pragma unroll
        for (int p = 0; p < TP; ++p) {
            const int ix = ix0 + p % TX, iy = iy0 + p / TX;
            if (ix < G.nx && iy < G.ny) {
                const size_t pix = (size_t)iy * G.nx + ix;
#pragma unroll
                for (int b = 0; b < NBAT; ++b) {
                    const size_t o = (pix * B + b0 + b) * nz + iz;
                    xt[o] = first ? acc[p][b] : xt[o] + acc[p][b];
                }
            }
        }
    }
}

template <typename T, int NBAT, int TX, int TY>
static size_t back3d_lds(const DevGeom &G, const LaunchCfg &L, int slot)
{
    size_t lds = sizeof(double) * (G.nv + 1) + 2 * sizeof(T) * (G.nv + 1);
    lds = (lds + 15) & ~(size_t)15;
    lds += sizeof(T) * (size_t)NBAT * L.back_pcols[slot] * (G.nv + 2);
    return lds;
}

template <typename T, int NBAT, int TX, int TY>
static hipError_t launch_back3d_t(const DevGeom &G, const LaunchCfg &L, const RecLayout &RL,
                                  int slot, int v0, int nvc, const RecPtrs &RP, const T *y, T *xt,
                                  int B, int b0, bool first, hipStream_t st)
{
    const size_t lds = back3d_lds<T, NBAT, TX, TY>(G, L, slot);
    if (lds > (size_t)L.lds_budget) return hipErrorInvalidValue;
    const int ntx = (G.nx + TX - 1) / TX, nty = (G.ny + TY - 1) / TY;
    hipLaunchKernelGGL((back3d_kernel<T, NBAT, TX, TY>), dim3(ntx * nty), dim3(L.back_threads), lds,
                       st, G, RL, v0, nvc, (const Rec<T> *)RP.recs, RP.sj0, RP.soff, RP.pixk, y, xt,
                       B, b0, L.back_pcols[slot], first ? 1 : 0);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_back3d_all(const DevGeom &G, const LaunchCfg &L, const RecLayout &RL,
                                    int v0, int nvc, void *ws, const T *y, T *xt, int B, bool first,
                                    hipStream_t st)
{
    const RecPtrs RP = rec_ptrs(RL, ws, sizeof(Rec<T>));
    const size_t bud = (size_t)L.lds_budget;
    const bool fit8 = back3d_lds<T, 8, 2, 1>(G, L, 3) <= bud;
    const bool fit4 = back3d_lds<T, 4, 2, 2>(G, L, 2) <= bud;
    const bool fit2 = back3d_lds<T, 2, 4, 2>(G, L, 1) <= bud;
    hipError_t e = hipSuccess;
    for (int b0 = 0; b0 < B && e == hipSuccess;) {
        const int rem = B - b0;
        if (rem >= 8 && fit8) { e = launch_back3d_t<T, 8, 2, 1>(G, L, RL, 3, v0, nvc, RP, y, xt, B, b0, first, st); b0 += 8; }
        else if (rem >= 4 && fit4) { e = launch_back3d_t<T, 4, 2, 2>(G, L, RL, 2, v0, nvc, RP, y, xt, B, b0, first, st); b0 += 4; }
        else if (rem >= 2 && fit2) { e = launch_back3d_t<T, 2, 4, 2>(G, L, RL, 1, v0, nvc, RP, y, xt, B, b0, first, st); b0 += 2; }
        else { e = launch_back3d_t<T, 1, 4, 4>(G, L, RL, 0, v0, nvc, RP, y, xt, B, b0, first, st); b0 += 1; }
    }
    return e;
}

hipError_t launch_back3d(const DevGeom &G, const LaunchCfg &L, const RecLayout &RL, bool fp64,
                         int v0, int nvc, void *ws, const void *y, void *xt, int B, bool first,
                         hipStream_t st)
{
    if (fp64) return launch_back3d_all<double>(G, L, RL, v0, nvc, ws, (const double *)y, (double *)xt, B, first, st);
    return launch_back3d_all<float>(G, L, RL, v0, nvc, ws, (const float *)y, (float *)xt, B, first, st);
}

}  // namespace smk
