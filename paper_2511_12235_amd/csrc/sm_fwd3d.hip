// sm_fwd3d.hip -- cone-beam forward projection y = W x (Sec. III-C).
//
// The paper's Algorithm 1 scatters each voxel into the detector elements it
// meets; on the GPU that would need atomics, so the loop is turned inside out.
// One workgroup owns one (view, detector column k) and one lane owns detector
// row r and its lower row plane r.  The workgroup walks the strip records of
// column k (built by sm_rec.hip; staged in LDS in chunks) and, for each pixel,
// lane r adds V_{r+1} - V_r, where V_p is the x-weighted volume of the pixel's
// voxel column below plane p:
//     V_p = c A sum_{iz < f} x_iz  +  G_p,
// f being the first voxel not wholly below the plane.  By parts over the
// voxel faces z_j, G_p = sum_j K_p(z_j) (x_j - x_{j-1}) over the faces from
// z_f up, K_p(z) the volume of the strip column above z and below plane p
// (sm_common.h).  Face z_f lies wholly below the plane, so K_p(z_f) is the
// linear volume A (tau lbar - z_f); faces the plane straddles need the chord
// table; faces wholly above it add nothing.  Voxel sums come from FP64 prefix
// sums along z, so c A (V_{r+1} - V_r) needs one difference.  Lane r keeps
// c A (range sum) - G_r and G_r apart; the G of the plane above is added once
// at the end through LDS.  The top detector edge (plane nv) has no lane: its
// G is summed lane-parallel over the strip's pixels in a fixed order.
#include "sm_internal.h"

namespace smk {

constexpr int kFwdChunk = 64;  // strip records staged in LDS at a time

template <typename T, int NBAT>
__global__ void __launch_bounds__(1024)
fwd3d_kernel(DevGeom G, RecLayout RL, int v0, const Rec<T> *__restrict__ recs,
             const int *__restrict__ soff, const double *__restrict__ P, T *__restrict__ y, int B,
             int b0)
{
    constexpr int RCH = (int)(sizeof(Rec<T>) / 16);
    extern __shared__ __align__(16) unsigned char smem[];
    const int nthr = blockDim.x, tid = threadIdx.x;
    Rec<T> *rbuf = reinterpret_cast<Rec<T> *>(smem);                                // kFwdChunk
    T *ex = reinterpret_cast<T *>(smem + sizeof(Rec<T>) * kFwdChunk);               // (nthr + 1) * NBAT
    T *red = ex + (size_t)(nthr + 1) * NBAT;                                        // nthr * NBAT
    const int nz = G.nz, nv = G.nv;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int vl = lb / G.nu, k = lb - vl * G.nu;
    const int view = v0 + vl;
    const double2 cs = G.trig[view];
    const StripAxis ax = strip_axis(G, cs.x, cs.y);
    const int64_t strip = (int64_t)vl * G.nu + k;
    const int n_ent = soff[strip * (RL.n_major_max + 1) + ax.n_major];
    const Rec<T> *Rs = recs + strip * RL.cap;
    const T inv_c = T(1.0 / G.c), z0c = T(G.z0 / G.c);
    const T cT = T(G.c);
    const size_t colstride = (size_t)(nz + 1);

    // lane r: plane r is the lower edge of row r
    const int r = tid;
    const bool active = r < nv;
    const double tau0 = active ? G.tau[r] : 0.0;
    const T tf0 = T(tau0), tf1 = T(active ? G.tau[r + 1] : 0.0);
    const T inv0 = tf0 != T(0) ? T(1) / tf0 : T(0);
    const double tauT = G.tau[nv];
    const T tfT = T(tauT);
    const T invT = tfT != T(0) ? T(1) / tfT : T(0);

    T acc1[NBAT], acc2[NBAT], accT[NBAT];
#pragma unroll
    for (int b = 0; b < NBAT; ++b) acc1[b] = acc2[b] = accT[b] = T(0);

    for (int c0 = 0; c0 < n_ent; c0 += kFwdChunk) {
        const int cnt = n_ent - c0 < kFwdChunk ? n_ent - c0 : kFwdChunk;
        __syncthreads();  // previous chunk consumed
        {
            const uint4 *src = reinterpret_cast<const uint4 *>(Rs + c0);
            uint4 *dst = reinterpret_cast<uint4 *>(rbuf);
            for (int q = tid; q < cnt * RCH; q += nthr) dst[q] = src[q];
        }
        __syncthreads();
        if (active) {
            for (int e = 0; e < cnt; ++e) {
                const Rec<T> &R = Rs[c0 + e];  // uniform fields through the scalar cache
                const int n = R.n;
                if (n == 0) continue;
                const StripTab<T> S = strip_tab<T>(R.tab, rbuf[e].tab);
                const double lc = R.lc;
                const T Llo = T(lc + (double)S.d0), Lhi = T(lc + (double)R.tab[n - 1][0]);
                const double lbar = lc + (double)R.lbo;
                const double *Pc[NBAT];
#pragma unroll
                for (int b = 0; b < NBAT; ++b) Pc[b] = P + ((size_t)R.pix * B + b0 + b) * colstride;
                int f;
                T gs[NBAT];
                plane_G<T, NBAT>(G, S, lc, lbar, Llo, Lhi, tau0, tf0, inv0, inv_c, z0c, Pc, f, gs);
                // first voxel not wholly below plane r + 1, as its own lane finds it
                T lo1, hi1;
                plane_extent<T>(tf1, Llo, Lhi, lo1, hi1);
                int fa1, fb1;
                face_split<T>(lo1, hi1, inv_c, z0c, nz, fa1, fb1);
                const int f1 = fa1 - 1 < 0 ? 0 : (fa1 - 1 > nz ? nz : fa1 - 1);
                const T cA = cT * S.A;
#pragma unroll
                for (int b = 0; b < NBAT; ++b) {
                    acc1[b] += cA * T(Pc[b][f1] - Pc[b][f]) - gs[b];
                    acc2[b] += gs[b];
                }
            }
        }
        // top detector edge: lane e takes record c0 + e (fields from LDS)
        if (tid < cnt) {
            const Rec<T> &R = rbuf[tid];
            const int n = R.n;
            if (n > 0) {
                const StripTab<T> S = strip_tab<T>(R.tab, R.tab);
                const double lc = R.lc;
                const T Llo = T(lc + (double)S.d0), Lhi = T(lc + (double)R.tab[n - 1][0]);
                const double lbar = lc + (double)R.lbo;
                const double *Pc[NBAT];
#pragma unroll
                for (int b = 0; b < NBAT; ++b) Pc[b] = P + ((size_t)R.pix * B + b0 + b) * colstride;
                int f;
                T gs[NBAT];
                plane_G<T, NBAT>(G, S, lc, lbar, Llo, Lhi, tauT, tfT, invT, inv_c, z0c, Pc, f, gs);
#pragma unroll
                for (int b = 0; b < NBAT; ++b) accT[b] += gs[b];
            }
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
static size_t fwd3d_lds(const LaunchCfg &L)
{
    return sizeof(Rec<T>) * kFwdChunk + sizeof(T) * (size_t)(2 * L.fwd_threads + 1) * NBAT;
}

template <typename T, int NBAT>
static hipError_t launch_fwd3d_t(const DevGeom &G, const LaunchCfg &L, const RecLayout &RL, int v0,
                                 int nvc, const Rec<T> *recs, const int *soff, const double *P,
                                 T *y, int B, int b0, hipStream_t st)
{
    const size_t lds = fwd3d_lds<T, NBAT>(L);
    if (lds > (size_t)L.lds_budget) return hipErrorInvalidValue;
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
