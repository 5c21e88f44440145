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
// linear volume A (tau lc - z_f), lc the strip's centroid depth; faces the
// plane straddles need the chord table; faces wholly above it add nothing.
// So c A (V_{r+1} - V_r) needs the sum of the voxels between the two planes'
// first voxels f and f' (one or two at the scanned geometries: a detector
// row's height at the pixel is about a voxel height), gathered from
// z-contiguous voxel columns.  Lane r keeps
// c A (range sum) - G_r and G_r apart; the G of the plane above is added once
// at the end through LDS.  The top detector edge (plane nv) has no lane: its
// G is summed lane-parallel over the strip's pixels in a fixed order.
//
// Straddled faces are rare and fall on the same lanes record after record, so
// each wave queues them (ballot positions) and evaluates the queue with all 64
// lanes.  For FP32 plans the evaluating lane rounds each term to a fixed-point
// grid and adds it to its owner's 64-bit integer sum in LDS: integer sums do
// not depend on the order of the atomic adds, so results stay deterministic,
// and the owner converts its sum once at the end.  The grid is a power of two
// chosen per workgroup from a bound on the sum of |terms| (records x straddled
// faces x their volume x 2 max|x|, max|x| per volume from the column pass), so
// the sum stays below 2^62 and each term keeps about 40 more bits than FP32
// carries.  FP64 plans keep FP64 sums and read their results back round by
// round.
#include "sm_internal.h"
#include "sm_wave.h"

namespace smk {

// Strip records staged in LDS at a time: 16 per wave of the workgroup, at
// most 64, so that the LDS of a workgroup stays near 5 KiB per wave and small
// workgroups (few detector rows) still reach 8 waves per SIMD.  FP64 records
// (272 bytes in LDS) stage half as many, so that LDS does not bound the FP64
// kernel below the waves its registers allow.
constexpr int kFwdChunkMax = 64;
template <typename T>
__host__ __device__ inline int fwd_chunk(int threads)
{
    return sizeof(T) == 4 ? min(kFwdChunkMax, 16 * (threads / 64)) : min(kFwdChunkMax / 2, 8 * (threads / 64));
}

// Straddle jobs a wave can hold: 128 (evaluated once 64 are pending) or, when
// LDS is short (many rows), 64 (evaluated before every ballot round); at most
// kRounds ballot rounds are kept between evaluations.  A job is one word:
// staged record (bits 0-5), plane r (bits 6-16) and face j (bits 17-27); the
// evaluating lane gathers the face height and the voxel difference itself.
constexpr int kQueueMax = 128;
constexpr int kRounds = 32;

// Evaluate the queued straddle jobs of this wave, K_r(z_j) (x_j - x_{j-1}),
// and add every lane's own results (in queue order) to its accumulators.
template <typename T, int NBAT>
__device__ __forceinline__ void fwd_flush(const DevGeom &G, const unsigned char *rbuf,
                                          const double *ptau, const T *ptf, const T *pinv,
                                          const T *__restrict__ X, int B, int b0,
                                          const unsigned *jobs, T *res, const JobRound *rounds,
                                          int &pending, int &nrounds, int lane, T (&acc1)[NBAT],
                                          T (&acc2)[NBAT])
{
    wave_sync();
    const int nz = G.nz;
    for (int s = lane; s < pending; s += 64) {
        const unsigned jb = jobs[s];
        const int e = (int)(jb & 63u), q = (int)((jb >> 6) & 2047u), j = (int)((jb >> 17) & 2047u);
        const Rec<T> &R = lds_rec<T>(rbuf, e);
        const T ev = T(ptau[q] * R.lc - (G.z0 + (double)j * G.c));
        const T K = K_cut<T>(strip_tab<T>(R.tab, R.tab), ptf[q], pinv[q], ev);
#pragma unroll
        for (int b = 0; b < NBAT; ++b) {
            const T *Xc = X + ((size_t)R.pix * B + b0 + b) * nz;
            const T xj = j < nz ? Xc[j] : T(0);  // x_j and x_{j-1}, zero outside
            const T xm = j >= 1 ? Xc[j - 1] : T(0);
            res[s * NBAT + b] = K * (xj - xm);
        }
    }
    wave_sync();
    T g[NBAT];
#pragma unroll
    for (int b = 0; b < NBAT; ++b) g[b] = T(0);
    for (int i = 0; i < nrounds; ++i) {
        const JobRound jr = rounds[i];
        const unsigned long long bal = ((unsigned long long)jr.hi << 32) | jr.lo;
        if ((bal >> lane) & 1ull) {
            const int slot = jr.base + lane_rank(bal);
#pragma unroll
            for (int b = 0; b < NBAT; ++b) g[b] += res[slot * NBAT + b];
        }
    }
#pragma unroll
    for (int b = 0; b < NBAT; ++b) {
        acc1[b] -= g[b];
        acc2[b] += g[b];
    }
    pending = 0;
    nrounds = 0;
    wave_sync();
}

// FP32 plans: evaluate the queued jobs and add each term, on the fixed-point
// grid of its volume, to the owner lane's integer sum gacc[b * nthr + r].
template <typename T, int NBAT>
__device__ __forceinline__ void fwd_flush_fixed(const DevGeom &G, const unsigned char *rbuf,
                                                const double *ptau, const T *ptf, const T *pinv,
                                                const T *__restrict__ X, int B, int b0,
                                                const unsigned *jobs, unsigned long long *gacc,
                                                int nthr, const int (&esh)[NBAT], int &pending, int lane)
{
    wave_sync();
    const int nz = G.nz;
    for (int s = lane; s < pending; s += 64) {
        const unsigned jb = jobs[s];
        const int e = (int)(jb & 63u), q = (int)((jb >> 6) & 2047u), j = (int)((jb >> 17) & 2047u);
        const Rec<T> &R = lds_rec<T>(rbuf, e);
        const T ev = T(ptau[q] * R.lc - (G.z0 + (double)j * G.c));
        const T K = K_cut<T>(strip_tab<T>(R.tab, R.tab), ptf[q], pinv[q], ev);
#pragma unroll
        for (int b = 0; b < NBAT; ++b) {
            const T *Xc = X + ((size_t)R.pix * B + b0 + b) * nz;
            const T xj = j < nz ? Xc[j] : T(0);  // x_j and x_{j-1}, zero outside
            const T xm = j >= 1 ? Xc[j - 1] : T(0);
            const T v = K * (xj - xm);
            const long long fx = __double2ll_rn(ldexp((double)v, esh[b]));
            atomicAdd(&gacc[(size_t)b * nthr + q], (unsigned long long)fx);
        }
    }
    pending = 0;
    wave_sync();
}

// The single-volume FP32 instance is held to 64 VGPRs (8 waves per SIMD): the
// extra waves hide the latency of the voxel gathers; the other instances keep
// their registers.
template <typename T, int NBAT>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(NBAT == 1 && sizeof(T) == 4 ? 8 : 1)))
fwd3d_kernel(DevGeom G, RecLayout RL, int v0, const Rec<T> *__restrict__ recs,
             const int *__restrict__ soff, const T *__restrict__ X,
             const unsigned *__restrict__ xmax, T *__restrict__ y, int B, int b0, int qcap)
{
    constexpr bool fixed = sizeof(T) == 4;  // fixed-point straddle sums (FP32 plans)
    constexpr int RCH = (int)(sizeof(Rec<T>) / 16);
    extern __shared__ __align__(16) unsigned char smem[];
    const int nthr = blockDim.x, tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    // LDS: staged records | per-wave job queues | exchange and reduction arrays
    const int chunk = fwd_chunk<T>(nthr);
    unsigned char *rbuf = smem;  // chunk records at lds_rec_stride<T>()
    size_t off = lds_rec_stride<T>() * chunk;
    const size_t qbytes = fixed ? (size_t)qcap * sizeof(unsigned)
                                : kRounds * sizeof(JobRound) + (size_t)qcap * (sizeof(unsigned) + sizeof(T) * NBAT);
    unsigned char *qw = smem + off + (size_t)wave * qbytes;
    JobRound *rounds = reinterpret_cast<JobRound *>(qw);
    unsigned *jobs = reinterpret_cast<unsigned *>(fixed ? qw : qw + kRounds * sizeof(JobRound));
    T *res = reinterpret_cast<T *>(qw + kRounds * sizeof(JobRound) + qcap * sizeof(unsigned));
    off += qbytes * (size_t)(nthr / 64);
    double *ptau = reinterpret_cast<double *>(smem + off);  // nv + 1 plane slopes (FP64)
    off += sizeof(double) * (size_t)(G.nv + 1);
    T *ptf = reinterpret_cast<T *>(smem + off);  // the slopes in T and their inverses
    T *pinv = ptf + (G.nv + 1);
    off += 2 * sizeof(T) * (size_t)(G.nv + 1);
    off = (off + 15) & ~(size_t)15;
    T *ex = reinterpret_cast<T *>(smem + off);  // (nthr + 1) * NBAT
    T *red = ex + (size_t)(nthr + 1) * NBAT;    // nthr * NBAT
    off += sizeof(T) * (size_t)(2 * nthr + 1) * NBAT;
    off = (off + 15) & ~(size_t)15;
    // fixed-point straddle sums of every lane (FP32 plans)
    unsigned long long *gacc = reinterpret_cast<unsigned long long *>(smem + off);
    const int nz = G.nz, nv = G.nv;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int vl = lb / G.nu, k = lb - vl * G.nu;
    const int view = v0 + vl;
    const double2 cs = G.trig[view];
    const StripAxis ax = strip_axis(G, cs.x, cs.y);
    const int64_t strip = (int64_t)vl * G.nu + k;
    const int n_ent = soff[strip * (RL.n_major_max + 1) + ax.n_major];
    const Rec<T> *Rs = recs + strip * RL.cap;
    const T z0c = T(G.z0 / G.c);

    // lane r: plane r is the lower edge of row r (lanes past nv carry tau = 0
    // and queue nothing)
    const int r = tid;
    const bool active = r < nv;
    const double tau0 = active ? G.tau[r] : 0.0;
    const T tf0 = T(tau0), tf1 = T(active ? G.tau[r + 1] : 0.0);
    const double tauT = G.tau[nv];
    const T tfT = T(tauT);
    const T invT = tfT != T(0) ? T(1) / tfT : T(0);

    for (int q = tid; q <= nv; q += nthr) {
        const double td = G.tau[q];
        const T t = T(td);
        ptau[q] = td;
        ptf[q] = t;
        pinv[q] = t != T(0) ? T(1) / t : T(0);
    }

    T acc1[NBAT], acc2[NBAT], accT[NBAT];
#pragma unroll
    for (int b = 0; b < NBAT; ++b) acc1[b] = acc2[b] = accT[b] = T(0);
    int pending = 0, nrounds = 0;

    // fixed-point grid 1 / scale[b]: |straddle sum| <= n_ent * faces * K * 2 max|x|,
    // H = max|tau| * pixel diagonal being the plane's rise over a pixel, a
    // straddled face lying within one voxel height of it (faces <= H / c + 3)
    // and K <= a b (H + c)
    int esh[NBAT];  // scale = 2^esh (uniform, kept in scalar registers)
    if (fixed) {
        const double tmx = fmax(fabs(G.tau[0]), fabs(G.tau[nv]));
        const double H = tmx * sqrt(G.a * G.a + G.b * G.b);
        const double bound = (double)n_ent * (H / G.c + 3.0) * (G.a * G.b * (H + G.c)) * 2.0 * (1.0 + 1e-6);
#pragma unroll
        for (int b = 0; b < NBAT; ++b) {
            const float xm = __uint_as_float(xmax[b0 + b]);
            int E = 62;
            const double m = isfinite(xm) && xm > 0.0f ? bound * (double)xm : 0.0;
            if (m > 0.0) frexp(m, &E);  // m < 2^E
            esh[b] = __builtin_amdgcn_readfirstlane(62 - E);
        }
        for (int i = tid; i < nthr * NBAT; i += nthr) gacc[i] = 0ull;
    }

    for (int c0 = 0; c0 < n_ent; c0 += chunk) {
        const int cnt = n_ent - c0 < chunk ? n_ent - c0 : chunk;
        __syncthreads();  // previous chunk consumed
        {
            const uint4 *src = reinterpret_cast<const uint4 *>(Rs + c0);
            for (int q = tid; q < cnt * RCH; q += nthr) {
                const int e = q / RCH, ch = q - e * RCH;
                reinterpret_cast<uint4 *>(rbuf + (size_t)e * lds_rec_stride<T>())[ch] = src[q];
            }
        }
        __syncthreads();
        // software pipeline: the voxel gathers of record e + 1 are issued before
        // record e is used (indices are clamped into the column, so the loads of
        // an empty record stay in range and are not used)
        auto faces = [&](int e, int &fa, int &je, int &f, int &f1) {
            const Rec<T> &R = Rs[c0 + e];
            int fb;
            plane_faces<T>(tf0, R.hLo, R.hHi, z0c, nz, fa, fb);
            f = max(fa - 1, 0);
            je = fb - 1 < nz ? fb - 1 : nz;
            int fa1, fb1;
            plane_faces<T>(tf1, R.hLo, R.hHi, z0c, nz, fa1, fb1);
            f1 = max(fa1 - 1, 0);
        };
        // x_f and x_{f+1} of the next record (f <= nz, so f + 1 is clamped)
        // (32-bit byte offsets from the column's uniform base: one shift
        // per gather instead of a 64-bit address)
        auto gather = [&](int e, int f, T (&xa)[NBAT], T (&xb)[NBAT]) {
            const int pix = Rs[c0 + e].pix;
            const unsigned oa = (unsigned)(f < nz ? f : nz - 1) * (unsigned)sizeof(T);
            const unsigned ob = (unsigned)(f + 1 < nz ? f + 1 : nz - 1) * (unsigned)sizeof(T);
#pragma unroll
            for (int b = 0; b < NBAT; ++b) {
                const char *Xn = reinterpret_cast<const char *>(X + ((size_t)pix * B + b0 + b) * nz);
                xa[b] = *reinterpret_cast<const T *>(Xn + oa);
                xb[b] = *reinterpret_cast<const T *>(Xn + ob);
            }
        };
        int nfa = 0, nje = 0, nf = 0, nf1 = 0;
        T nxa[NBAT], nxb[NBAT];
        if (cnt > 0) {
            faces(0, nfa, nje, nf, nf1);
            gather(0, nf, nxa, nxb);
        }
        for (int e = 0; e < cnt; ++e) {
            const int fa = nfa, je = nje, f = nf, f1 = nf1;
            T xa[NBAT], xb[NBAT];
#pragma unroll
            for (int b = 0; b < NBAT; ++b) {
                xa[b] = nxa[b];
                xb[b] = nxb[b];
            }
            if (e + 1 < cnt) {
                faces(e + 1, nfa, nje, nf, nf1);
                gather(e + 1, nf, nxa, nxb);
            }
            const Rec<T> &R = Rs[c0 + e];  // uniform fields through the scalar cache
            const int n = R.n;
            if (n == 0) continue;
            const StripTab<T> S = strip_tab<T>(R.tab, lds_rec<T>(rbuf, e).tab);
            const double lc = R.lc;
            const T cA = R.cA;
            const T Klin = S.A * T(tau0 * lc - (G.z0 + (double)f * G.c));
            const bool lin = fa >= 1 && fa <= nz;  // then f = fa - 1 < nz
            // voxels f .. f1 - 1 lie between the two planes' first voxels
            T rs[NBAT];
#pragma unroll
            for (int b = 0; b < NBAT; ++b)
                rs[b] = (f1 > f ? xa[b] : T(0)) + (f1 > f + 1 ? xb[b] : T(0));
            for (int j = f + 2; j < f1; ++j) {  // taller spans: rare, loaded in place
#pragma unroll
                for (int b = 0; b < NBAT; ++b) rs[b] += X[((size_t)R.pix * B + b0 + b) * nz + j];
            }
#pragma unroll
            for (int b = 0; b < NBAT; ++b) {
                const T gs = lin ? Klin * xa[b] : T(0);
                acc1[b] += cA * rs[b] - gs;
                acc2[b] += gs;
            }
            // queue the straddled faces fa .. je, one ballot round per face
            const int ns = active && je >= fa ? je - fa + 1 : 0;
            for (int t = 0;; ++t) {
                const bool want = t < ns;
                const unsigned long long bal = __ballot(want);
                if (bal == 0ull) break;
                if (fixed) {
                    if (pending > qcap - 64)
                        fwd_flush_fixed<T, NBAT>(G, rbuf, ptau, ptf, pinv, X, B, b0, jobs, gacc, nthr,
                                                 esh, pending, lane);
                } else if (pending > qcap - 64 || nrounds == kRounds) {
                    fwd_flush<T, NBAT>(G, rbuf, ptau, ptf, pinv, X, B, b0, jobs, res, rounds, pending,
                                       nrounds, lane, acc1, acc2);
                }
                if (want) {
                    const unsigned j = fa + t;
                    const int slot = pending + lane_rank(bal);
                    jobs[slot] = (unsigned)e | ((unsigned)r << 6) | (j << 17);
                }
                if (!fixed) {
                    if (lane == 0)
                        rounds[nrounds] = JobRound{(unsigned)bal, (unsigned)(bal >> 32), pending, 0};
                    ++nrounds;
                }
                pending += __popcll(bal);
            }
            if (pending >= 64) {
                if (fixed)
                    fwd_flush_fixed<T, NBAT>(G, rbuf, ptau, ptf, pinv, X, B, b0, jobs, gacc, nthr, esh,
                                             pending, lane);
                else
                    fwd_flush<T, NBAT>(G, rbuf, ptau, ptf, pinv, X, B, b0, jobs, res, rounds, pending,
                                       nrounds, lane, acc1, acc2);
            }
        }
        // jobs refer to this chunk's records: evaluate them before restaging
        if (pending > 0) {
            if (fixed)
                fwd_flush_fixed<T, NBAT>(G, rbuf, ptau, ptf, pinv, X, B, b0, jobs, gacc, nthr, esh,
                                         pending, lane);
            else
                fwd_flush<T, NBAT>(G, rbuf, ptau, ptf, pinv, X, B, b0, jobs, res, rounds, pending,
                                   nrounds, lane, acc1, acc2);
        }
        // top detector edge: lane e takes record c0 + e (fields from LDS)
        if (tid < cnt) {
            const Rec<T> &R = lds_rec<T>(rbuf, tid);
            const int n = R.n;
            if (n > 0) {
                const StripTab<T> S = strip_tab<T>(R.tab, R.tab);
                const double lc = R.lc;
                const T *Xc[NBAT];
#pragma unroll
                for (int b = 0; b < NBAT; ++b) Xc[b] = X + ((size_t)R.pix * B + b0 + b) * nz;
                int f;
                T gs[NBAT];
                plane_G<T, NBAT>(G, S, lc, R.hLo, R.hHi, tauT, tfT, invT, z0c, Xc, f, gs);
#pragma unroll
                for (int b = 0; b < NBAT; ++b) accT[b] += gs[b];
            }
        }
    }

    if (fixed) {  // every wave's adds to this lane's sums are done
        __syncthreads();
#pragma unroll
        for (int b = 0; b < NBAT; ++b) {
            // a non-finite value in the volume makes the sum NaN (0 * inf)
            const float xm = __uint_as_float(xmax[b0 + b]);
            const T g = T(ldexp((double)(long long)gacc[(size_t)b * nthr + tid], -esh[b])) + T(0.0f * xm);
            acc1[b] -= g;
            acc2[b] += g;
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
static size_t fwd3d_lds(const LaunchCfg &L, int qcap)
{
    constexpr bool fixed = sizeof(T) == 4;
    const size_t qbytes = fixed ? (size_t)qcap * sizeof(unsigned)
                                : kRounds * sizeof(JobRound) + (size_t)qcap * (sizeof(unsigned) + sizeof(T) * NBAT);
    size_t lds = lds_rec_stride<T>() * fwd_chunk<T>(L.fwd_threads) + qbytes * (size_t)(L.fwd_threads / 64);
    // plane tables (nv + 1 <= fwd_threads + 1)
    lds += (sizeof(double) + 2 * sizeof(T)) * (size_t)(L.fwd_threads + 1);
    lds = (lds + 15) & ~(size_t)15;
    lds += sizeof(T) * (size_t)(2 * L.fwd_threads + 1) * NBAT;
    lds = (lds + 15) & ~(size_t)15;
    if (fixed) lds += sizeof(unsigned long long) * (size_t)L.fwd_threads * NBAT;
    return lds;
}

// Largest queue capacity whose LDS fits, 0 when none does.
template <typename T, int NBAT>
static int fwd3d_qcap(const LaunchCfg &L)
{
    for (int q = kQueueMax; q >= 64; q -= 64)
        if (fwd3d_lds<T, NBAT>(L, q) <= (size_t)L.lds_budget) return q;
    return 0;
}

template <typename T, int NBAT>
static hipError_t launch_fwd3d_t(const DevGeom &G, const LaunchCfg &L, const RecLayout &RL, int v0,
                                 int nvc, const Rec<T> *recs, const int *soff, const T *X,
                                 const unsigned *xmax, T *y, int B, int b0, hipStream_t st)
{
    const int qcap = fwd3d_qcap<T, NBAT>(L);
    if (qcap == 0) return hipErrorInvalidValue;
    const size_t lds = fwd3d_lds<T, NBAT>(L, qcap);
    hipLaunchKernelGGL((fwd3d_kernel<T, NBAT>), dim3(nvc * G.nu), dim3(L.fwd_threads), lds, st, G,
                       RL, v0, recs, soff, X, xmax, y, B, b0, qcap);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_fwd3d_all(const DevGeom &G, const LaunchCfg &L, const RecLayout &RL,
                                   int v0, int nvc, void *ws, const T *X, const unsigned *xmax,
                                   T *y, int B, hipStream_t st)
{
    RecPtrs RP = rec_ptrs(RL, ws, sizeof(Rec<T>));
    const Rec<T> *recs = (const Rec<T> *)RP.recs;
    const bool fit4 = fwd3d_qcap<T, 4>(L) > 0;
    const bool fit2 = fwd3d_qcap<T, 2>(L) > 0;
    hipError_t e = hipSuccess;
    // at most four volumes per launch: eight measured slower per volume than
    // two launches of four at 256^3 (register pressure of the eight sums)
    for (int b0 = 0; b0 < B && e == hipSuccess;) {
        const int rem = B - b0;
        if (rem >= 4 && fit4) { e = launch_fwd3d_t<T, 4>(G, L, RL, v0, nvc, recs, RP.soff, X, xmax, y, B, b0, st); b0 += 4; }
        else if (rem >= 2 && fit2) { e = launch_fwd3d_t<T, 2>(G, L, RL, v0, nvc, recs, RP.soff, X, xmax, y, B, b0, st); b0 += 2; }
        else { e = launch_fwd3d_t<T, 1>(G, L, RL, v0, nvc, recs, RP.soff, X, xmax, y, B, b0, st); b0 += 1; }
    }
    return e;
}

bool fwd3d_fits(const LaunchCfg &L, bool fp64)
{
    return fp64 ? fwd3d_qcap<double, 1>(L) > 0 : fwd3d_qcap<float, 1>(L) > 0;
}

hipError_t launch_fwd3d(const DevGeom &G, const LaunchCfg &L, const RecLayout &RL, bool fp64,
                        int v0, int nvc, void *ws, const void *X, const unsigned *xmax, void *y,
                        int B, hipStream_t st)
{
    if (fp64) return launch_fwd3d_all<double>(G, L, RL, v0, nvc, ws, (const double *)X, nullptr, (double *)y, B, st);
    return launch_fwd3d_all<float>(G, L, RL, v0, nvc, ws, (const float *)X, xmax, (float *)y, B, st);
}

}  // namespace smk
