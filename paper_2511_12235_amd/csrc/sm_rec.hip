// sm_rec.hip -- strip records for a chunk of views.
//
// One workgroup per (view, detector column k).  The pixels that the wedge of
// column k can meet are enumerated along the major axis (sm_common.h); their
// per-major start/offset table and one strip record per pixel (the top-view
// polygon of Sec. III-B with its chord-width table, built in FP64) are written
// to the workspace.  Every thread builds records, so the FP64 polygon work
// runs at full occupancy and never stalls the projection kernels.  The forward
// kernel walks a strip's records in order; the adjoint finds the record of
// (pixel, column) through the per-major table and the per-pixel column range.
#include "sm_internal.h"

namespace smk {

// Block-wide exclusive scan of one int per thread (blockDim.x <= 1024).
__device__ int block_scan_excl(int v, int *tmp, int &total)
{
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = (blockDim.x + 63) >> 6;
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) tmp[wid] = incl;
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int w = 0; w < nw; ++w) {
            const int t = tmp[w];
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

// Four waves per SIMD: the FP64 polygon work is written one edge at a time so
// that it fits 128 registers; with fewer waves the kernel idles on latency.
//
// Records leave through LDS: each lane puts its record's 16-byte chunks in
// its own column of `stage` (the vertex scratch, free again once the record
// is built), and the wave then stores its records' chunks in address order,
// 64 consecutive chunks per instruction, instead of every lane storing one
// chunk of its own record per instruction (64 partial lines each time).
// FP64 records (16 chunks) go out in two passes of 8.
constexpr int kStageRows = 9;
// Row stride of `stage` in 16-byte elements: one more than the threads, so
// that the chunks one store instruction gathers (several chunks of each of
// a few records) fall in different LDS banks.
constexpr int kStageStride = 257;

template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
rec_kernel(DevGeom G, RecLayout RL, int v0, Rec<T> *__restrict__ recs, int *__restrict__ sj0,
           int *__restrict__ soff, int2 *__restrict__ pixk)
{
    constexpr int RCH = (int)(sizeof(Rec<T>) / 16);           // chunks per record
    constexpr int NPASS = (RCH + kStageRows - 1) / kStageRows;  // staging passes
    constexpr int PCH = RCH / NPASS;                            // chunks per pass
    static_assert(PCH * NPASS == RCH && PCH <= kStageRows, "record chunks per pass");
    __shared__ int offs[257];
    __shared__ int jst[256];
    __shared__ int scan_tmp[8];
    // vertex i of thread t at [i][t] (no bank conflicts); later chunk c of
    // thread t's record at [c][t]
    __shared__ uint4 stage[kStageRows][kStageStride];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, wbase = tid - lane;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int vl = lb / G.nu, k = lb - vl * G.nu;
    const int view = v0 + vl;
    const double2 cs = G.trig[view];
    const double cp = cs.x, sp = cs.y;
    const double ulo = G.u0 + (double)k * G.du, uhi = G.u0 + (double)(k + 1) * G.du;
    const StripAxis ax = strip_axis(G, cp, sp);
    const int64_t strip = (int64_t)vl * G.nu + k;
    int *J0 = sj0 + strip * RL.n_major_max;
    int *OFF = soff + strip * (RL.n_major_max + 1);
    uint4 *out = reinterpret_cast<uint4 *>(recs + strip * RL.cap);
    int2 *pk = pixk + (int64_t)vl * G.nx * G.ny;

    int run = 0;  // entries written by earlier chunks of majors
    for (int base = 0; base < ax.n_major; base += nthr) {
        const int im = base + tid;
        int cnt = 0, j0 = 0, j1 = -1;
        if (im < ax.n_major) {
            strip_minor_range(G, ax, cp, sp, ulo, uhi, im, j0, j1);
            cnt = j1 >= j0 ? j1 - j0 + 1 : 0;
        }
        int total;
        const int ex = block_scan_excl(cnt, scan_tmp, total);
        jst[tid] = j0;
        offs[tid] = ex;
        if (tid == 0) offs[nthr] = total;
        if (im < ax.n_major) {
            J0[im] = j0;
            OFF[im] = run + ex;
        }
        __syncthreads();
        // entries that get a slot: e < total and run + e < cap
        const int nrec = min(total, RL.cap - run);
        for (int e0 = 0; e0 < nrec; e0 += nthr) {
            const int e = e0 + tid;
            Rec<T> R;
            if (e < nrec) {
                int lo = 0, hi = nthr;  // largest m with offs[m] <= e
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (offs[mid] <= e) lo = mid; else hi = mid;
                }
                const int mj = base + lo;
                const int mn = jst[lo] + (e - offs[lo]);
                const int ix = ax.major_x ? mj : mn;
                const int iy = ax.major_x ? mn : mj;
                build_record<T>(G, cp, sp, ix, iy, k, R,
                                LdsVerts{reinterpret_cast<double2 *>(&stage[0][tid]), kStageStride});
                R.pix = iy * G.nx + ix;
                if (R.n > 0) {
                    atomicMin(&pk[R.pix].x, k);
                    atomicMax(&pk[R.pix].y, k);
                }
            }
            // this wave's records: slots run + e0 + wbase + r, r < nw
            const int nw = min(max(nrec - e0 - wbase, 0), 64);
            uint4 *dst = out + (int64_t)(run + e0 + wbase) * RCH;
            const uint4 *rc = reinterpret_cast<const uint4 *>(&R);
#pragma unroll
            for (int ps = 0; ps < NPASS; ++ps) {
                // the vertex scratch (or the previous pass) of every lane of
                // the wave is consumed before it is overwritten
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (e < nrec) {
#pragma unroll
                    for (int c = 0; c < PCH; ++c) stage[c][tid] = rc[ps * PCH + c];
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                for (int q = lane; q < nw * PCH; q += 64) {
                    const int r = q / PCH, c = q - r * PCH;
                    dst[(int64_t)r * RCH + ps * PCH + c] = stage[c][wbase + r];
                }
            }
            // the next round's vertex scratch overwrites the staged chunks
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        run += total;
        __syncthreads();
    }
    if (tid == 0) OFF[ax.n_major] = run;
}

// Largest number of pixels any strip enumerates (the record capacity).
__global__ void strip_count_kernel(DevGeom G, int *max_count)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= G.n_p * G.nu) return;
    const int view = q / G.nu, k = q - view * G.nu;
    const double2 cs = G.trig[view];
    const StripAxis ax = strip_axis(G, cs.x, cs.y);
    const double ulo = G.u0 + (double)k * G.du, uhi = G.u0 + (double)(k + 1) * G.du;
    int tot = 0;
    for (int i = 0; i < ax.n_major; ++i) {
        int j0, j1;
        strip_minor_range(G, ax, cs.x, cs.y, ulo, uhi, i, j0, j1);
        tot += j1 >= j0 ? j1 - j0 + 1 : 0;
    }
    atomicMax(max_count, tot);
}

__global__ void fill_int2_kernel(int2 *p, int64_t n, int2 v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
static hipError_t launch_records_t(const DevGeom &G, const RecLayout &RL, int v0, int nvc,
                                   void *ws, hipStream_t st)
{
    RecPtrs P = rec_ptrs(RL, ws, sizeof(Rec<T>));
    const int64_t npix = (int64_t)nvc * G.nx * G.ny;
    const int64_t want = (npix + 255) / 256;
    hipLaunchKernelGGL(fill_int2_kernel, dim3((unsigned)(want < 65536 ? want : 65536)), dim3(256), 0,
                       st, P.pixk, npix, make_int2(0x7fffffff, -1));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rec_kernel<T>, dim3(nvc * G.nu), dim3(256), 0, st, G, RL, v0,
                       (Rec<T> *)P.recs, P.sj0, P.soff, P.pixk);
    return hipGetLastError();
}

hipError_t launch_records(const DevGeom &G, const RecLayout &RL, bool fp64, int v0, int nvc,
                          void *ws, hipStream_t st)
{
    if (fp64) return launch_records_t<double>(G, RL, v0, nvc, ws, st);
    return launch_records_t<float>(G, RL, v0, nvc, ws, st);
}

hipError_t launch_strip_count(const DevGeom &G, int *max_count, hipStream_t st)
{
    const int n = G.n_p * G.nu;
    hipLaunchKernelGGL(strip_count_kernel, dim3((n + 127) / 128), dim3(128), 0, st, G, max_count);
    return hipGetLastError();
}

}  // namespace smk
