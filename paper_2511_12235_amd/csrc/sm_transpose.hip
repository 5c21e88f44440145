// sm_transpose.hip -- layout changes between the caller's volume layout
// x[B][nz][ny][nx] and the z-contiguous working layout xt[ny][nx][B][nz]
// that the cone-beam kernels read and write (one voxel column of one batch
// element is nz consecutive values).  Tiled 32 x 32 through LDS so both the
// reads and the writes are coalesced.
#include "sm_internal.h"

namespace smk {

// For each slab s = (b, iy): in[iz][ix] -> out[ix][iz].
template <typename T>
__global__ void __launch_bounds__(256) to_columns_kernel(const T *__restrict__ x, T *__restrict__ xt,
                                                          int B, int nz, int ny, int nx)
{
    __shared__ T tile[32][33];
    const int s = blockIdx.z;
    const int b = s / ny, iy = s - b * ny;
    const int ix0 = blockIdx.x * 32, iz0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int j = ty; j < 32; j += 8) {
        const int iz = iz0 + j, ix = ix0 + tx;
        if (iz < nz && ix < nx) tile[j][tx] = x[(((size_t)b * nz + iz) * ny + iy) * nx + ix];
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int ix = ix0 + j, iz = iz0 + tx;
        if (iz < nz && ix < nx) xt[(((size_t)iy * nx + ix) * B + b) * nz + iz] = tile[tx][j];
    }
}

template <typename T>
__global__ void __launch_bounds__(256) from_columns_kernel(const T *__restrict__ xt, T *__restrict__ x,
                                                            int B, int nz, int ny, int nx)
{
    __shared__ T tile[32][33];
    const int s = blockIdx.z;
    const int b = s / ny, iy = s - b * ny;
    const int ix0 = blockIdx.x * 32, iz0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int j = ty; j < 32; j += 8) {
        const int ix = ix0 + j, iz = iz0 + tx;
        if (iz < nz && ix < nx) tile[j][tx] = xt[(((size_t)iy * nx + ix) * B + b) * nz + iz];
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int iz = iz0 + j, ix = ix0 + tx;
        if (iz < nz && ix < nx) x[(((size_t)b * nz + iz) * ny + iy) * nx + ix] = tile[tx][j];
    }
}

hipError_t launch_to_columns(const void *x, void *xt, int elem, int B, int nz, int ny, int nx,
                             hipStream_t st)
{
    dim3 grid((nx + 31) / 32, (nz + 31) / 32, B * ny);
    if (elem == 8)
        hipLaunchKernelGGL(to_columns_kernel<double>, grid, dim3(256), 0, st, (const double *)x,
                           (double *)xt, B, nz, ny, nx);
    else
        hipLaunchKernelGGL(to_columns_kernel<float>, grid, dim3(256), 0, st, (const float *)x,
                           (float *)xt, B, nz, ny, nx);
    return hipGetLastError();
}

hipError_t launch_from_columns(const void *xt, void *x, int elem, int B, int nz, int ny, int nx,
                               hipStream_t st)
{
    dim3 grid((nx + 31) / 32, (nz + 31) / 32, B * ny);
    if (elem == 8)
        hipLaunchKernelGGL(from_columns_kernel<double>, grid, dim3(256), 0, st, (const double *)xt,
                           (double *)x, B, nz, ny, nx);
    else
        hipLaunchKernelGGL(from_columns_kernel<float>, grid, dim3(256), 0, st, (const float *)xt,
                           (float *)x, B, nz, ny, nx);
    return hipGetLastError();
}

}  // namespace smk
