// sm_2d.hip -- fan-beam forward and adjoint (Sec. III-B, Algorithm 1).
//
// The 2D weight of pixel n for detector element m is the pixel area between
// the rays to the element's two edges.  With A(u*) the area on the u <= u*
// side of the ray through detector coordinate u* (the paper's sweep of the
// sorted vertex angles: triangle A_3, then trapezoid A_4, then the pixel minus
// a triangle; sweep_area() in sm_common.h), the weight is A(u_{m+1}) - A(u_m).
//
// Forward: one workgroup per (view, detector element) walks the pixels of the
// element's wedge and reduces in a fixed order (no atomics).  Adjoint: one
// wave per pixel; lane l takes views l, l + 64, ... and the elements each
// meets, and the wave adds its lanes' sums in a fixed butterfly order (one
// thread per pixel left a 64^2 image with 64 waves for 1024 SIMDs).
#include "sm_internal.h"

namespace smk {

template <typename T, int NBAT>
__global__ void __launch_bounds__(256) fwd2d_kernel(DevGeom G, const T *__restrict__ x,
                                                     T *__restrict__ y, int B, int b0)
{
    __shared__ T red[256 * NBAT];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int view = lb / G.nu, k = lb - view * G.nu;
    const double2 cs = G.trig[view];
    const double cp = cs.x, sp = cs.y;
    const double ulo = G.u0 + (double)k * G.du, uhi = G.u0 + (double)(k + 1) * G.du;
    const double mu0 = ulo / G.D, mu1 = uhi / G.D;
    const T a = T(G.a), b = T(G.b);
    const size_t npix = (size_t)G.nx * G.ny;

    T acc[NBAT];
#pragma unroll
    for (int q = 0; q < NBAT; ++q) acc[q] = T(0);

    const StripAxis ax = strip_axis(G, cp, sp);
    for (int im = tid; im < ax.n_major; im += nthr) {
        int j0, j1;
        strip_minor_range(G, ax, cp, sp, ulo, uhi, im, j0, j1);
        for (int jm = j0; jm <= j1; ++jm) {
            const int ix = ax.major_x ? im : jm, iy = ax.major_x ? jm : im;
            const double xc = G.x0 + ((double)ix + 0.5) * G.a;
            const double yc = G.y0 + ((double)iy + 0.5) * G.b;
            const double lc = G.s - (xc * cp + yc * sp);
            const double tc = yc * cp - xc * sp;
            const T w = sweep_area<T>(cp, sp, lc, tc, mu1, a, b) - sweep_area<T>(cp, sp, lc, tc, mu0, a, b);
            const size_t pix = (size_t)iy * G.nx + ix;
#pragma unroll
            for (int q = 0; q < NBAT; ++q) acc[q] += w * x[(size_t)(b0 + q) * npix + pix];
        }
    }
#pragma unroll
    for (int q = 0; q < NBAT; ++q) red[tid * NBAT + q] = acc[q];
    __syncthreads();
    for (int w = 1; w < nthr; w <<= 1) {
        if ((tid & (2 * w - 1)) == 0 && tid + w < nthr) {
#pragma unroll
            for (int q = 0; q < NBAT; ++q) red[tid * NBAT + q] += red[(tid + w) * NBAT + q];
        }
        __syncthreads();
    }
    if (tid == 0) {
#pragma unroll
        for (int q = 0; q < NBAT; ++q) y[((size_t)(b0 + q) * G.n_p + view) * G.nu + k] = red[q];
    }
}

template <typename T, int NBAT>
__global__ void __launch_bounds__(256) back2d_kernel(DevGeom G, const T *__restrict__ y,
                                                      T *__restrict__ x, int B, int b0)
{
    const int lane = threadIdx.x & 63;
    const int pix = xcd_remap(blockIdx.x, gridDim.x) * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6);
    const int npix = G.nx * G.ny;
    if (pix >= npix) return;  // uniform over the wave
    const int iy = pix / G.nx, ix = pix - iy * G.nx;
    const double xc = G.x0 + ((double)ix + 0.5) * G.a;
    const double yc = G.y0 + ((double)iy + 0.5) * G.b;
    const T a = T(G.a), b = T(G.b);
    T acc[NBAT];
#pragma unroll
    for (int q = 0; q < NBAT; ++q) acc[q] = T(0);
    for (int view = lane; view < G.n_p; view += 64) {
        const double2 cs = G.trig[view];
        const double cp = cs.x, sp = cs.y;
        int k0, k1;
        pixel_columns(G, cp, sp, ix, iy, k0, k1);
        if (k1 < k0) continue;
        const double lc = G.s - (xc * cp + yc * sp);
        const double tc = yc * cp - xc * sp;
        T Aprev = sweep_area<T>(cp, sp, lc, tc, (G.u0 + (double)k0 * G.du) / G.D, a, b);
        for (int k = k0; k <= k1; ++k) {
            const T Anext = sweep_area<T>(cp, sp, lc, tc, (G.u0 + (double)(k + 1) * G.du) / G.D, a, b);
            const T w = Anext - Aprev;
            Aprev = Anext;
#pragma unroll
            for (int q = 0; q < NBAT; ++q) acc[q] += w * y[((size_t)(b0 + q) * G.n_p + view) * G.nu + k];
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int q = 0; q < NBAT; ++q) acc[q] += __shfl_xor(acc[q], o, 64);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NBAT; ++q) x[(size_t)(b0 + q) * npix + pix] = acc[q];
    }
}

template <typename T>
static hipError_t fwd2d_all(const DevGeom &G, const T *x, T *y, int B, hipStream_t st)
{
    const int nblk = G.n_p * G.nu;
    for (int b0 = 0; b0 < B;) {
        const int rem = B - b0;
        if (rem >= 4) {
            hipLaunchKernelGGL((fwd2d_kernel<T, 4>), dim3(nblk), dim3(64), 0, st, G, x, y, B, b0);
            b0 += 4;
        } else {
            hipLaunchKernelGGL((fwd2d_kernel<T, 1>), dim3(nblk), dim3(64), 0, st, G, x, y, B, b0);
            b0 += 1;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
static hipError_t back2d_all(const DevGeom &G, const T *y, T *x, int B, hipStream_t st)
{
    const int npix = G.nx * G.ny;
    const int nblk = (npix + 3) / 4;  // four waves (pixels) per workgroup
    for (int b0 = 0; b0 < B;) {
        const int rem = B - b0;
        if (rem >= 4) {
            hipLaunchKernelGGL((back2d_kernel<T, 4>), dim3(nblk), dim3(256), 0, st, G, y, x, B, b0);
            b0 += 4;
        } else {
            hipLaunchKernelGGL((back2d_kernel<T, 1>), dim3(nblk), dim3(256), 0, st, G, y, x, B, b0);
            b0 += 1;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_fwd2d(const DevGeom &G, bool fp64, const void *x, void *y, int B, hipStream_t st)
{
    if (fp64) return fwd2d_all<double>(G, (const double *)x, (double *)y, B, st);
    return fwd2d_all<float>(G, (const float *)x, (float *)y, B, st);
}

hipError_t launch_back2d(const DevGeom &G, bool fp64, const void *y, void *x, int B, hipStream_t st)
{
    if (fp64) return back2d_all<double>(G, (const double *)y, (double *)x, B, st);
    return back2d_all<float>(G, (const float *)y, (float *)x, B, st);
}

}  // namespace smk
