// sm_transpose.hip -- layout changes between the caller's volume layout
// x[B][nz][ny][nx] and the column layouts the cone-beam kernels use:
//   forward input : voxel columns X[ny*nx][B][nz] (z contiguous, the plan's
//                   precision), which the forward gathers a few voxels at a
//                   time, and (FP32) the largest |x| of every batch element,
//                   which sets the fixed-point grid of the forward's straddle
//                   sums;
//   adjoint output: xt[g][ny*nx][B][nz] (z contiguous), one partial volume per
//                   view run g, summed in order and transposed back here.
// Both go through LDS so global reads and writes stay coalesced.
#include "sm_internal.h"

namespace smk {

__global__ void zero_u32_kernel(unsigned *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// One workgroup per (PW = 2^pwl consecutive pixels of one row, batch element):
// the PW columns pass through LDS (row stride nz + 1, so that the transposing
// writes hit distinct banks) and leave z-contiguous.  xmax (FP32 only, else
// NULL): bits of max |x| per batch element, raised with an integer max
// (non-negative floats order like their bit patterns).
template <typename T>
__global__ void __launch_bounds__(256) columns_kernel(const T *__restrict__ x, T *__restrict__ X,
                                                      unsigned *__restrict__ xmax, int B, int nz,
                                                      int ny, int nx, int pwl)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned wmax[4];
    T *col = reinterpret_cast<T *>(smem);  // [PW][nz + 1]
    const int tid = threadIdx.x;
    const int PW = 1 << pwl;
    const int nxb = (nx + PW - 1) / PW;
    const int bi = blockIdx.x;
    const int b = bi / (ny * nxb);
    const int rem = bi - b * ny * nxb;
    const int iy = rem / nxb, ix0 = (rem - iy * nxb) * PW;
    const int w = min(PW, nx - ix0);
    const int cs = nz + 1;
    unsigned m = 0u;
    for (int q = tid; q < PW * nz; q += blockDim.x) {  // PW consecutive x values per z slice
        const int iz = q >> pwl, i = q & (PW - 1);
        if (i < w) {
            const T v = x[(((size_t)b * nz + iz) * ny + iy) * nx + ix0 + i];
            col[i * cs + iz] = v;
            if (sizeof(T) == 4) m = max(m, __float_as_uint(fabsf((float)v)));
        }
    }
    if (xmax) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, o, 64));
        if ((tid & 63) == 0) wmax[tid >> 6] = m;
    }
    __syncthreads();
    if (xmax && tid == 0) {
        unsigned mb = wmax[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) mb = max(mb, wmax[i]);
        atomicMax(&xmax[b], mb);
    }
    for (int i = 0; i < w; ++i) {
        T *dst = X + (((size_t)iy * nx + ix0 + i) * B + b) * nz;
        for (int iz = tid; iz < nz; iz += blockDim.x) dst[iz] = col[i * cs + iz];
    }
}

template <typename T>
__global__ void __launch_bounds__(256) from_columns_kernel(const T *__restrict__ xt, T *__restrict__ x,
                                                            int B, int nz, int ny, int nx, int groups)
{
    __shared__ T tile[32][33];
    const int s = blockIdx.z;
    const int b = s / ny, iy = s - b * ny;
    const int ix0 = blockIdx.x * 32, iz0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int j = ty; j < 32; j += 8) {
        const int ix = ix0 + j, iz = iz0 + tx;
        if (iz < nz && ix < nx) {
            const size_t o = (((size_t)iy * nx + ix) * B + b) * nz + iz;
            const size_t gs = (size_t)nx * ny * B * nz;
            T v = xt[o];
            for (int g = 1; g < groups; ++g) v += xt[(size_t)g * gs + o];
            tile[j][tx] = v;
        }
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int iz = iz0 + j, ix = ix0 + tx;
        if (iz < nz && ix < nx) x[(((size_t)b * nz + iz) * ny + iy) * nx + ix] = tile[tx][j];
    }
}

hipError_t launch_to_columns(const void *x, void *X, unsigned *xmax, bool fp64, int B, int nz, int ny,
                            int nx, hipStream_t st)
{
    const size_t es = fp64 ? 8 : 4;
    int pwl = 4;  // 16 pixels per workgroup while the columns fit in 48 KiB of LDS
    while (pwl > 0 && es * ((size_t)1 << pwl) * (size_t)(nz + 1) > 49152) --pwl;
    const int PW = 1 << pwl;
    const int nxb = (nx + PW - 1) / PW;
    const dim3 grid((unsigned)B * ny * nxb);
    const size_t lds = es * PW * (size_t)(nz + 1);
    if (fp64) {
        hipLaunchKernelGGL(columns_kernel<double>, grid, dim3(256), lds, st, (const double *)x,
                           (double *)X, (unsigned *)nullptr, B, nz, ny, nx, pwl);
    } else {
        hipLaunchKernelGGL(zero_u32_kernel, dim3((B + 255) / 256), dim3(256), 0, st, xmax, B);
        hipLaunchKernelGGL(columns_kernel<float>, grid, dim3(256), lds, st, (const float *)x, (float *)X,
                           xmax, B, nz, ny, nx, pwl);
    }
    return hipGetLastError();
}

hipError_t launch_from_columns(const void *xt, void *x, int elem, int B, int nz, int ny, int nx,
                               int groups, hipStream_t st)
{
    dim3 grid((nx + 31) / 32, (nz + 31) / 32, B * ny);
    if (elem == 8)
        hipLaunchKernelGGL(from_columns_kernel<double>, grid, dim3(256), 0, st, (const double *)xt,
                           (double *)x, B, nz, ny, nx, groups);
    else
        hipLaunchKernelGGL(from_columns_kernel<float>, grid, dim3(256), 0, st, (const float *)xt,
                           (float *)x, B, nz, ny, nx, groups);
    return hipGetLastError();
}

}  // namespace smk
