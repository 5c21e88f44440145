// sm_fwd3d.hip -- cone-beam forward projection y = W x (Sec. III-C).
//
// The paper's Algorithm 1 scatters each voxel into the detector elements it
// meets; on the GPU that would need atomics, so the loop is turned inside out.
// One workgroup owns one (view, detector column k) and one lane owns detector
// row r and its lower row plane r.  The workgroup walks the strip records of
// column k (built by sm_rec.hip; uniform, so they are read with scalar loads)
// and, for each pixel, lane r adds
//     c A * sum_{iz in [f_r, f_{r+1})} x_iz  +  G_{r+1} - G_r,
// where A is the strip area, f_p the first voxel of the column not entirely
// below plane p, and G_p the x-weighted volume below plane p of the voxels
// plane p cuts.  By parts over the voxel faces z_j,
//     G_p = sum_j (x_j - x_{j-1}) K_p(z_j),
// K_p(z) being the volume of the strip column above z and below plane p
// (sm_common.h); only faces the plane crosses inside the strip need the
// piecewise evaluation, the others are linear or zero.  Voxel sums come from
// FP64 prefix sums along z, so the range sum is a single difference.  Lane r
// keeps  c A R - G_r  and  G_r  apart; the G of the plane above is added once
// at the end through LDS.  The top detector edge (plane nv) has no lane: its G
// is summed lane-parallel over the strip's pixels and reduced in a fixed order.
#include "sm_internal.h"

namespace smk {

template <typename T, int NBAT>
__device__ __forceinline__ void plane_terms(const DevGeom &G, const Rec<T> &R, int n, double tau,
                                            T tauf, T invt, double inv_c, double zoff,
                                            const double *const (&Pc)[NBAT], bool want_range,
                                            double tau_next, T (&rs)[NBAT], T (&gs)[NBAT])
{
    const T d0 = R.tab[0][0], dn = R.tab[n - 1][0];
    const double lmin = R.lc + (double)d0, lmax = R.lc + (double)dn;
    const bool neg = tau < 0.0;
    const double lo_abs = tau * (neg ? lmax : lmin), hi_abs = tau * (neg ? lmin : lmax);
    const int f = (int)dmin_(dmax_(floor(lo_abs * inv_c - zoff), 0.0), (double)G.nz);
    const int l = (int)dmin_(dmax_(floor(hi_abs * inv_c - zoff), -1.0), (double)(G.nz - 1));
    double Pprev[NBAT];
#pragma unroll
    for (int b = 0; b < NBAT; ++b) Pprev[b] = Pc[b][f];
    if (want_range) {
        const double lo1 = tau_next * (tau_next < 0.0 ? lmax : lmin);
        const int f1 = (int)dmin_(dmax_(floor(lo1 * inv_c - zoff), 0.0), (double)G.nz);
#pragma unroll
        for (int b = 0; b < NBAT; ++b) rs[b] = T(Pc[b][f1] - Pprev[b]);
    }
    const double hz = tau * R.lc - G.z0;  // plane height above z0 at the pixel centre
    T xprev[NBAT];
#pragma unroll
    for (int b = 0; b < NBAT; ++b) {
        xprev[b] = T(0);
        gs[b] = T(0);
    }
    for (int j = f; j <= l + 1; ++j) {
        T xcur[NBAT];
#pragma unroll
        for (int b = 0; b < NBAT; ++b) xcur[b] = T(0);
        if (j <= l) {
#pragma unroll
            for (int b = 0; b < NBAT; ++b) {
                const double pn = Pc[b][j + 1];
                xcur[b] = T(pn - Pprev[b]);
                Pprev[b] = pn;
            }
        }
        const T e = T(hz - (double)j * G.c);
        const T Kv = eval_K<T>(R.tab, n, tauf, invt, e);
#pragma unroll
        for (int b = 0; b < NBAT; ++b) {
            gs[b] += (xcur[b] - xprev[b]) * Kv;
            xprev[b] = xcur[b];
        }
    }
}

template <typename T, int NBAT>
__global__ void __launch_bounds__(1024)
fwd3d_kernel(DevGeom G, RecLayout RL, int v0, const Rec<T> *__restrict__ recs,
             const int *__restrict__ soff, const double *__restrict__ P, T *__restrict__ y, int B,
             int b0)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int nthr = blockDim.x, tid = threadIdx.x;
    T *ex = reinterpret_cast<T *>(smem);          // (nthr + 1) * NBAT
    T *red = ex + (size_t)(nthr + 1) * NBAT;      // nthr * NBAT
    const int nz = G.nz, nv = G.nv;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int vl = lb / G.nu, k = lb - vl * G.nu;
    const int view = v0 + vl;
    const double2 cs = G.trig[view];
    const StripAxis ax = strip_axis(G, cs.x, cs.y);
    const int64_t strip = (int64_t)vl * G.nu + k;
    const int n_ent = soff[strip * (RL.n_major_max + 1) + ax.n_major];
    const Rec<T> *Rs = recs + strip * RL.cap;
    const double inv_c = 1.0 / G.c, zoff = G.z0 * inv_c;
    const T cT = T(G.c);
    const size_t colstride = (size_t)(nz + 1);

    // lane r: plane r is the lower edge of row r
    const int r = tid;
    const bool active = r < nv;
    const double tau0 = active ? G.tau[r] : 0.0;
    const double tau1 = active ? G.tau[r + 1] : 0.0;
    const T tf0 = T(tau0);
    const T inv0 = tf0 != T(0) ? T(1) / tf0 : T(0);

    T acc1[NBAT], acc2[NBAT];
#pragma unroll
    for (int b = 0; b < NBAT; ++b) acc1[b] = acc2[b] = T(0);

    for (int e = 0; e < n_ent; ++e) {
        const Rec<T> &R = Rs[e];
        const int n = R.n;
        if (n == 0) continue;
        if (active) {
            const double *Pc[NBAT];
#pragma unroll
            for (int b = 0; b < NBAT; ++b) Pc[b] = P + ((size_t)R.pix * B + b0 + b) * colstride;
            T rs[NBAT], gs[NBAT];
            plane_terms<T, NBAT>(G, R, n, tau0, tf0, inv0, inv_c, zoff, Pc, true, tau1, rs, gs);
            const T cA = cT * R.tab[0][2];
#pragma unroll
            for (int b = 0; b < NBAT; ++b) {
                acc1[b] += cA * rs[b] - gs[b];
                acc2[b] += gs[b];
            }
        }
    }

    // top detector edge (plane nv): lane-parallel over the strip's pixels
    T accT[NBAT];
#pragma unroll
    for (int b = 0; b < NBAT; ++b) accT[b] = T(0);
    {
        const double tauT = G.tau[nv];
        const T tfT = T(tauT);
        const T invT = tfT != T(0) ? T(1) / tfT : T(0);
        for (int e = tid; e < n_ent; e += nthr) {
            const Rec<T> &R = Rs[e];
            const int n = R.n;
            if (n == 0) continue;
            const double *Pc[NBAT];
#pragma unroll
            for (int b = 0; b < NBAT; ++b) Pc[b] = P + ((size_t)R.pix * B + b0 + b) * colstride;
            T rs[NBAT], gs[NBAT];
            plane_terms<T, NBAT>(G, R, n, tauT, tfT, invT, inv_c, zoff, Pc, false, 0.0, rs, gs);
#pragma unroll
            for (int b = 0; b < NBAT; ++b) accT[b] += gs[b];
        }
    }

    // y_r = acc1_r + acc2_{r+1}; acc2_nv is the fixed-order sum of accT
#pragma unroll
    for (int b = 0; b < NBAT; ++b) {
        ex[tid * NBAT + b] = acc2[b];
        red[tid * NBAT + b] = accT[b];
    }
    __syncthreads();
    for (int w = 1; w < nthr; w <<= 1) {
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
static hipError_t launch_fwd3d_t(const DevGeom &G, const LaunchCfg &L, const RecLayout &RL, int v0,
                                 int nvc, const Rec<T> *recs, const int *soff, const double *P,
                                 T *y, int B, int b0, hipStream_t st)
{
    const size_t lds = sizeof(T) * (size_t)(2 * L.fwd_threads + 1) * NBAT;
    hipLaunchKernelGGL((fwd3d_kernel<T, NBAT>), dim3(nvc * G.nu), dim3(L.fwd_threads), lds, st, G,
                       RL, v0, recs, soff, P, y, B, b0);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_fwd3d_all(const DevGeom &G, const LaunchCfg &L, const RecLayout &RL,
                                   int v0, int nvc, void *ws, const double *P, T *y, int B,
                                   hipStream_t st)
{
    RecPtrs RP = rec_ptrs(RL, ws, sizeof(Rec<T>));
    const Rec<T> *recs = (const Rec<T> *)RP.recs;
    hipError_t e = hipSuccess;
    for (int b0 = 0; b0 < B && e == hipSuccess;) {
        const int rem = B - b0;
        if (rem >= 8) { e = launch_fwd3d_t<T, 8>(G, L, RL, v0, nvc, recs, RP.soff, P, y, B, b0, st); b0 += 8; }
        else if (rem >= 4) { e = launch_fwd3d_t<T, 4>(G, L, RL, v0, nvc, recs, RP.soff, P, y, B, b0, st); b0 += 4; }
        else if (rem >= 2) { e = launch_fwd3d_t<T, 2>(G, L, RL, v0, nvc, recs, RP.soff, P, y, B, b0, st); b0 += 2; }
        else { e = launch_fwd3d_t<T, 1>(G, L, RL, v0, nvc, recs, RP.soff, P, y, B, b0, st); b0 += 1; }
    }
    return e;
}

hipError_t launch_fwd3d(const DevGeom &G, const LaunchCfg &L, const RecLayout &RL, bool fp64,
                        int v0, int nvc, void *ws, const double *P, void *y, int B, hipStream_t st)
{
    if (fp64) return launch_fwd3d_all<double>(G, L, RL, v0, nvc, ws, P, (double *)y, B, st);
    return launch_fwd3d_all<float>(G, L, RL, v0, nvc, ws, P, (float *)y, B, st);
}

}  // namespace smk
