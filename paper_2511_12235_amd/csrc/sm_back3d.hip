// sm_back3d.hip -- cone-beam adjoint x = W^T y with the forward's weights.
//
// Voxel-stationary gather, no atomics: a workgroup owns a TX x TY tile of
// pixels and every voxel above them (one lane per z index) and keeps the
// tile's sums in registers while it loops over a run of views of a chunk
// (small volumes split the chunk's views into several runs, each with its
// own partial volume, so that the grid fills the device).  Per
// view it stages in LDS the detector columns the tile can meet (all rows, with
// a zero row above and below) and the strip records of the tile's pixels
// (built by sm_rec.hip).  For every (pixel, column) record lane iz then adds
//     sum_q (K_q(za) - K_q(zb)) (y[q-1] - y[q]),
// the by-parts form of sum_r W_r y[r] over the rows, where K_q(z) is the
// volume of the strip column above height z and below row plane q
// (sm_common.h) and za / zb are the voxel's bottom and top faces.  Planes
// wholly below the voxel add nothing; planes wholly above it add c A each,
// which telescopes to c A y[first such plane - 1].  Of the planes reaching
// into the voxel, those wholly above za contribute the linear volume
// A (tau lc - za) at za (lc the strip's centroid depth); only planes
// straddling a face need the chord table.  Chunks of views add into the
// z-contiguous workspace in a fixed order, which is transposed to the
// caller's layout afterwards.

#include "sm_internal.h"

namespace smk {

static_assert(sizeof(AdjRec<float>) == 160 && sizeof(AdjRec<double>) == 288, "staged record");

// Stage view `view`'s detector columns kmin .. kmax (pc of them, all rows,
// zero rows at -1 and nv) and the strip records of the tile's pixels, slot
// (p, k - k0(p)) at rtab + slot * RS bytes; a slot without a record gets
// n = 0.
template <typename T, int NBAT, int TX, int TY, size_t RS>
__device__ __forceinline__ void stage_view(const DevGeom &G, const RecLayout &RL, const StripAxis &ax,
                                           int vl, int view, int ix0, int iy0, int kmin, int kmax,
                                           const Rec<T> *__restrict__ recs, const int *__restrict__ sj0,
                                           const int *__restrict__ soff, const int2 *__restrict__ pixk,
                                           const T *__restrict__ y, int b0, int pcols, int rspan,
                                           unsigned char *rtab, T *patch)
{
    constexpr int TP = TX * TY;
    const int nthr = blockDim.x, tid = threadIdx.x;
    const int nv = G.nv, rowstride = nv + 2, npix = G.nx * G.ny;
    const int pc = kmax - kmin + 1;
    // y[view][:, kmin..kmax] (a single volume: one thread per detector row, its
    // pc values side by side; batches: consecutive threads on consecutive columns)
    for (int bb = 0; bb < NBAT; ++bb) {
        const T *src = y + ((size_t)(b0 + bb) * G.n_p + view) * nv * G.nu + kmin;
        T *dst = patch + (size_t)bb * pcols * rowstride + 1;
        if constexpr (NBAT == 1) {
            for (int row = tid; row < nv; row += nthr) {
                const T *s = src + (size_t)row * G.nu;
                T *d = dst + row;
                for (int col = 0; col < pc; ++col) d[col * rowstride] = s[col];
            }
        } else {
            const float inv_pc = 1.0f / (float)pc;
            for (int q = tid; q < pc * nv; q += nthr) {
                const int row = (int)(((float)q + 0.5f) * inv_pc);
                const int col = q - row * pc;
                dst[col * rowstride + row] = src[(size_t)row * G.nu + col];
            }
        }
        for (int col = tid; col < pc; col += nthr) {
            dst[col * rowstride - 1] = T(0);
            dst[col * rowstride + nv] = T(0);
        }
    }
    // strip records into AdjRec slots, several threads per slot: part 0
    // copies the fields, the others table rows 1 .. MAXV - 1 (all five per
    // thread for an FP32 single volume, else one; a whole record per thread
    // set the kernel's register peak) with the coefficient of the segment
    // ending at each
    constexpr int RPT = NBAT == 1 && sizeof(T) == 4 ? MAXV - 1 : 1;  // table rows per thread
    constexpr int TPS = 1 + (MAXV - 1) / RPT;                        // threads per slot
    constexpr int RC = (int)(sizeof(T) * 4 / 16);                    // 16-byte chunks per row
    static_assert((MAXV - 1) % RPT == 0, "table rows per thread");
    const float inv_rspan = 1.0f / (float)rspan;
    for (int q = tid; q < TP * rspan * TPS; q += nthr) {
        const int pk = q / TPS, part = q - pk * TPS;          // TPS is a constant
        const int p = (int)(((float)pk + 0.5f) * inv_rspan);  // exact for pk < 16 rspan, rspan <= 2048
        const int kk = pk - p * rspan;
        const int ix = ix0 + p % TX, iy = iy0 + p / TX;
        AdjRec<T> *dst = reinterpret_cast<AdjRec<T> *>(rtab + (size_t)(p * rspan + kk) * RS);
        int pos = -1;
        int64_t strip = 0;
        if (ix < G.nx && iy < G.ny) {
            const int2 kr = pixk[(size_t)vl * npix + (size_t)iy * G.nx + ix];
            const int k = kr.x + kk;
            if (k <= kr.y && k >= kmin && k <= kmax) {
                strip = (int64_t)vl * G.nu + k;
                pos = strip_position(ax.major_x, ix, iy, sj0 + strip * RL.n_major_max,
                                     soff + strip * (RL.n_major_max + 1));
            }
        }
        // FP32 single volumes: a slot without a record, or with an empty
        // polygon, gets a zero header.  Index scales 0 make both plane splits
        // independent of the face, so that the record adds exactly zero (no
        // linear volumes, no straddled planes whose table would be read,
        // c A = A = 0) and the adjoint evaluates it without a test.  The
        // other instances mark it n = 0 and skip it (the zero header cost
        // them a wave per SIMD in registers).
        constexpr bool kZeroEmpty = NBAT == 1 && sizeof(T) == 4;
        if (kZeroEmpty && part == 0 && (pos < 0 || recs[strip * RL.cap + pos].n == 0)) {
            dst->lc = 0.0;
            dst->n = 0;
            dst->k4[0] = dst->k4[1] = dst->k4[2] = dst->k4[3] = T(0);
            dst->cA = dst->bA = dst->d0 = dst->A = T(0);
        } else if (pos >= 0) {
            const Rec<T> &src = recs[strip * RL.cap + pos];
            if (part == 0) {
                dst->lc = src.lc;
                dst->n = src.n;
                dst->k4[0] = src.kLo;
                dst->k4[1] = src.kHi;
                dst->k4[2] = src.kHi;
                dst->k4[3] = src.kLo;
                dst->cA = src.cA;
                dst->bA = src.bA;
                dst->d0 = src.tab[0][0];
                dst->A = src.tab[0][2];
            } else {
                const int r0 = 1 + (part - 1) * RPT;
                T dp = src.tab[r0 - 1][0], wp = src.tab[r0 - 1][1];
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const int r = r0 + i;
                    uint4 ch[RC];
#pragma unroll
                    for (int c = 0; c < RC; ++c) ch[c] = reinterpret_cast<const uint4 *>(src.tab[r])[c];
#pragma unroll
                    for (int c = 0; c < RC; ++c) reinterpret_cast<uint4 *>(dst->seg[r - 1])[c] = ch[c];
                    const T *row = reinterpret_cast<const T *>(ch);
                    // g / 6 on segment r - 1: (w_r-1 / 2 - w_r / 2) / (3 L) from
                    // the table's half widths; the guard keeps it finite on a
                    // zero-length segment, where h = 0
                    const T L = row[0] - dp;
                    dst->g6[r - 1] = (wp - row[1]) * rcp_(L > T(1e-30) ? L : T(1e-30)) * T(1.0 / 3.0);
                    dp = row[0];
                    wp = row[1];
                }
            }
        } else if (part == 0) {
            dst->n = 0;  // an empty slot
        }
    }
}

// Detector columns the tile's pixels meet in view vl (from the record pass):
// false when none; kmax is clipped so that kmax - kmin < pcols.
template <int TX, int TY>
__device__ __forceinline__ bool tile_columns(const DevGeom &G, const int2 *__restrict__ pixk, int vl,
                                             int ix0, int iy0, int pcols, int &kmin, int &kmax)
{
    constexpr int TP = TX * TY;
    const int npix = G.nx * G.ny;
    kmin = 1 << 30;
    kmax = -1;
#pragma unroll
    for (int p = 0; p < TP; ++p) {
        const int ix = ix0 + p % TX, iy = iy0 + p / TX;
        if (ix < G.nx && iy < G.ny) {
            const int2 q = pixk[(size_t)vl * npix + (size_t)iy * G.nx + ix];
            if (q.y >= q.x) {
                kmin = min(kmin, q.x);
                kmax = max(kmax, q.y);
            }
        }
    }
    if (kmax < kmin) return false;
    if (kmax - kmin + 1 > pcols) kmax = kmin + pcols - 1;  // pcols bounds every tile's span
    return true;
}

template <typename T, int NBAT, int TX, int TY>
__global__ void __launch_bounds__(1024)
back3d_kernel(DevGeom G, RecLayout RL, int v0, int nvc, const Rec<T> *__restrict__ recs,
              const int *__restrict__ sj0, const int *__restrict__ soff,
              const int2 *__restrict__ pixk, const T *__restrict__ y, T *__restrict__ xt, int B,
              int b0, int pcols, int rspan, int first, int groups)
{
    constexpr int TP = TX * TY;
    extern __shared__ __align__(16) unsigned char smem[];
    const int nthr = blockDim.x, tid = threadIdx.x;
    const int nz = G.nz, nv = G.nv;
    const int rowstride = nv + 2;

    // LDS: staged records | plane table | detector patch
    AdjRec<T> *rtab = reinterpret_cast<AdjRec<T> *>(smem);
    size_t off = sizeof(AdjRec<T>) * (size_t)TP * rspan;  // a multiple of 16
    PlaneRow<T> *prow = reinterpret_cast<PlaneRow<T> *>(smem + off);
    off += sizeof(PlaneRow<T>) * (nv + 1);
    T *patch = reinterpret_cast<T *>(smem + off);

    for (int p = tid; p <= nv; p += nthr) {
        const double t = G.tau[p];
        PlaneRow<T> row;
        row.tau = t;
        row.tf = T(t);
        row.inv = t != 0.0 ? T(1) / T(t) : T(0);
        prow[p] = row;
    }

    const int ntx = (G.nx + TX - 1) / TX, nty = (G.ny + TY - 1) / TY;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    // view group: the chunk's views are split into `groups` contiguous runs,
    // each summed into its own partial volume
    const int grp = lb / (ntx * nty);
    const int tile = lb - grp * ntx * nty;
    const int vbeg = (int)((int64_t)nvc * grp / groups), vend = (int)((int64_t)nvc * (grp + 1) / groups);
    xt += (size_t)grp * G.nx * G.ny * B * G.nz;
    const int tyi = tile / ntx, txi = tile - tyi * ntx;
    const int ix0 = txi * TX, iy0 = tyi * TY;
    const int npix = G.nx * G.ny;

    const int iz = tid;
    const bool active = iz < nz;
    const double za = G.z0 + (double)iz * G.c;
    const double zb = G.z0 + (double)(iz + 1) * G.c;
    const T v0dv = T(G.v0 / G.dv);
    // each face's index-scale pair in a staged record (see plane_split)
    const int ka_off = T(za) >= T(0) ? 2 : 0, kb_off = T(zb) >= T(0) ? 2 : 0;

    T acc[TP][NBAT];
#pragma unroll
    for (int p = 0; p < TP; ++p)
#pragma unroll
        for (int b = 0; b < NBAT; ++b) acc[p][b] = T(0);

    for (int vl = vbeg; vl < vend; ++vl) {
        const int view = v0 + vl;
        const double2 cs = G.trig[view];
        const StripAxis ax = strip_axis(G, cs.x, cs.y);
        int kmin, kmax;
        if (!tile_columns<TX, TY>(G, pixk, vl, ix0, iy0, pcols, kmin, kmax)) continue;
        kmin = __builtin_amdgcn_readfirstlane(kmin);  // uniform: keep the column
        kmax = __builtin_amdgcn_readfirstlane(kmax);  // bounds in scalar registers
        __syncthreads();  // the previous view's patch and records are consumed
        stage_view<T, NBAT, TX, TY, sizeof(AdjRec<T>)>(G, RL, ax, vl, view, ix0, iy0, kmin, kmax, recs, sj0,
                                                    soff, pixk, y, b0, pcols, rspan,
                                                    reinterpret_cast<unsigned char *>(rtab), patch);
        __syncthreads();
        if (!active) continue;
        // Pixels in a loop unrolled by 8: the current pixel's sums are acc[0];
        // the array rotates by one slot per pixel, so after TP pixels every
        // sum is back in its own slot (keeps the sums in registers; the
        // unrolled copies merge eight rotations into one, while a full
        // unroll measured slower).
#pragma unroll 8
        for (int p = 0; p < TP; ++p) {
            const int ix = ix0 + p % TX, iy = iy0 + p / TX;
            // the column range is the same for every lane: scalar registers
            // and scalar loop control (pixels past the volume's edge read
            // their clamped neighbour's range and then take an empty one)
            const bool inside = ix < G.nx && iy < G.ny;
            const int2 q = pixk[(size_t)vl * npix + (size_t)min(iy, G.ny - 1) * G.nx + min(ix, G.nx - 1)];
            const int qx = __builtin_amdgcn_readfirstlane(q.x), qy = __builtin_amdgcn_readfirstlane(q.y);
            const int k0 = inside ? qx : 0;
            const int k1 = __builtin_amdgcn_readfirstlane(
                inside ? min(min(qy, qx + rspan - 1), kmax) : -1);  // rspan bounds every span
            T cur[NBAT];
#pragma unroll
            for (int b = 0; b < NBAT; ++b) cur[b] = acc[0][b];
            for (int k = max(k0, kmin); k <= k1; ++k) {
                const AdjRec<T> &R = rtab[p * rspan + (k - k0)];  // LDS copy (zeros when empty)
                // FP32 single volumes evaluate an empty record (its zero
                // header adds exactly zero), the others skip it
                if constexpr (NBAT > 1 || sizeof(T) == 8) {
                    if (__builtin_amdgcn_readfirstlane(R.n) == 0) continue;
                }
                const AdjTab<T> S = adj_tab<T>(R);
                const T *Y = patch + (size_t)(k - kmin) * rowstride + 1;  // Y[-1] .. Y[nv]
                T sum[NBAT];
                adj_terms<T, NBAT>(S, R.lc, R.cA, R.bA, R.k4 + ka_off, R.k4 + kb_off, prow, za, zb, v0dv,
                                   nv, Y, (size_t)pcols * rowstride, sum);
#pragma unroll
                for (int b = 0; b < NBAT; ++b) cur[b] += sum[b];
            }
#pragma unroll
            for (int i = 0; i + 1 < TP; ++i)
#pragma unroll
                for (int b = 0; b < NBAT; ++b) acc[i][b] = acc[i + 1][b];
#pragma unroll
            for (int b = 0; b < NBAT; ++b) acc[TP - 1][b] = cur[b];
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
    size_t lds = sizeof(AdjRec<T>) * (size_t)TX * TY * L.rspan;
    lds += sizeof(PlaneRow<T>) * (G.nv + 1);
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
    hipLaunchKernelGGL((back3d_kernel<T, NBAT, TX, TY>), dim3(ntx * nty * L.back_groups),
                       dim3(L.back_threads), lds, st, G, RL, v0, nvc, (const Rec<T> *)RP.recs, RP.sj0,
                       RP.soff, RP.pixk, y, xt, B, b0, L.back_pcols[slot], L.rspan, first ? 1 : 0,
                       L.back_groups);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_back3d_all(const DevGeom &G, const LaunchCfg &L, const RecLayout &RL,
                                    int v0, int nvc, void *ws, const T *y, T *xt, int B, bool first,
                                    hipStream_t st)
{
    const RecPtrs RP = rec_ptrs(RL, ws, sizeof(Rec<T>));
    const size_t bud = (size_t)L.lds_budget;
    const bool fit4 = back3d_lds<T, 4, 2, 2>(G, L, 2) <= bud;
    const bool fit2 = back3d_lds<T, 2, 4, 2>(G, L, 1) <= bud;
    // single volumes with two waves per workgroup (nz <= 128) take 4 x 2
    // tiles: a 4 x 4 tile's staged records and detector patch would hold
    // such workgroups to about 4.5 waves per SIMD
    const bool half = back_tile_rows(G, sizeof(T) == 8) == 2 && back3d_lds<T, 1, 4, 2>(G, L, 1) <= bud;
    hipError_t e = hipSuccess;
    // at most four volumes per launch: eight (2 x 1 tiles) measured slower per
    // volume than two launches of four at 256^3
    for (int b0 = 0; b0 < B && e == hipSuccess;) {
        const int rem = B - b0;
        if (rem >= 4 && fit4) { e = launch_back3d_t<T, 4, 2, 2>(G, L, RL, 2, v0, nvc, RP, y, xt, B, b0, first, st); b0 += 4; }
        else if (rem >= 2 && fit2) { e = launch_back3d_t<T, 2, 4, 2>(G, L, RL, 1, v0, nvc, RP, y, xt, B, b0, first, st); b0 += 2; }
        else if (half) { e = launch_back3d_t<T, 1, 4, 2>(G, L, RL, 1, v0, nvc, RP, y, xt, B, b0, first, st); b0 += 1; }
        else { e = launch_back3d_t<T, 1, 4, 4>(G, L, RL, 0, v0, nvc, RP, y, xt, B, b0, first, st); b0 += 1; }
    }
    return e;
}

size_t back3d_lds_min(const DevGeom &G, const LaunchCfg &L, bool fp64)
{
    if (back_tile_rows(G, fp64) == 2)
        return fp64 ? back3d_lds<double, 1, 4, 2>(G, L, 1) : back3d_lds<float, 1, 4, 2>(G, L, 1);
    return fp64 ? back3d_lds<double, 1, 4, 4>(G, L, 0) : back3d_lds<float, 1, 4, 4>(G, L, 0);
}

hipError_t launch_back3d(const DevGeom &G, const LaunchCfg &L, const RecLayout &RL, bool fp64,
                         int v0, int nvc, void *ws, const void *y, void *xt, int B, bool first,
                         hipStream_t st)
{
    if (fp64) return launch_back3d_all<double>(G, L, RL, v0, nvc, ws, (const double *)y, (double *)xt, B, first, st);
    return launch_back3d_all<float>(G, L, RL, v0, nvc, ws, (const float *)y, (float *)xt, B, first, st);
}

}  // namespace smk
