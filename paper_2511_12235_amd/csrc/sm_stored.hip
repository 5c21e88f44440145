// sm_stored.hip -- stored-W mode: the system matrix of Sec. I (W in R^{M x N})
// and its transpose as device CSR arrays, for problems whose W fits in HBM,
// applied by a plain sparse matrix-vector product.
//
// Build: the FP64 weight pass of sm_csr.hip counts the entries of every row
// (rows of W: detector elements; rows of W^T: voxels), an exclusive scan
// gives the row offsets, a fill pass writes (column, value) pairs in arrival
// order, and a segmented radix sort (hipCUB) orders every row by column, so
// the arrays do not depend on scheduling.  The pattern is W > 1e-12 voxel
// measure decided in FP64; values are stored in the requested precision.
//
// Apply: one wave per row, lanes striding the row, a fixed-order butterfly
// over the wave; the sum of a row is the same on every call.
#include <hipcub/hipcub.hpp>

#include "sm_plan.h"

namespace smk {

template <typename V>
__global__ void __launch_bounds__(256)
spmv_kernel(int64_t n_rows, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ cols,
            const V *__restrict__ vals, const V *__restrict__ x, V *__restrict__ y)
{
    const int lane = threadIdx.x & 63;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = w0; i < n_rows; i += nw) {
        const int64_t a = row_ptr[i], e = row_ptr[i + 1];
        V acc = V(0);
        for (int64_t p = a + lane; p < e; p += 64) acc += vals[p] * x[cols[p]];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane == 0) y[i] = acc;
    }
}

template <typename V>
static hipError_t spmv_t(int64_t n_rows, const int64_t *row_ptr, const int32_t *cols, const void *vals,
                         const void *x, void *y, hipStream_t st)
{
    const int64_t waves = n_rows;
    int64_t blocks = (waves + 3) / 4;
    blocks = blocks < 1 ? 1 : (blocks > (1 << 20) ? (1 << 20) : blocks);
    hipLaunchKernelGGL(spmv_kernel<V>, dim3((unsigned)blocks), dim3(256), 0, st, n_rows, row_ptr,
                       cols, (const V *)vals, (const V *)x, (V *)y);
    return hipGetLastError();
}

}  // namespace smk

using smk::set_error;

namespace {

sm_status hip_err(hipError_t e, const char *what)
{
    return set_error(SM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Row counts and offsets of W (transposed = 0) or W^T (transposed = 1) into
// row_ptr (device, n_rows + 1); returns the entry count in *nnz.
sm_status count_rows(const sm_plan *p, int transposed, int64_t *row_ptr, int32_t *cnt,
                     int64_t *nnz, hipStream_t st)
{
    const double tau_keep = 1e-12 * p->G.a * p->G.b * p->G.c;
    const int64_t rows = transposed ? p->n_vox : p->n_rays;
    hipError_t e = hipMemsetAsync(cnt, 0, sizeof(int32_t) * rows, st);
    if (e == hipSuccess)
        e = transposed ? smk::launch_csr_count_vox(p->G, tau_keep, cnt, st)
                       : smk::launch_csr_count(p->G, tau_keep, cnt, st);
    if (e == hipSuccess) e = smk::launch_scan_counts(cnt, rows, row_ptr, st);
    if (e == hipSuccess) e = hipMemcpyAsync(nnz, row_ptr + rows, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e == hipSuccess ? SM_OK : hip_err(e, "stored-W count");
}

sm_status check_sizes(const sm_plan *p)
{
    if (p->n_vox > 2147483647LL || p->n_rays > 2147483647LL)
        return set_error(SM_EUNSUPPORTED, "stored W needs fewer than 2^31 voxels and detector elements");
    return SM_OK;
}

}  // namespace

extern "C" {

sm_status sm_stored_count(const sm_plan *p, int32_t transposed, int64_t *nnz)
{
    if (!p) return set_error(SM_EINVAL, "plan is NULL");
    if (!nnz) return set_error(SM_EINVAL, "nnz is NULL");
    sm_status s = smk::check_plan_device(p);
    if (s != SM_OK) return s;
    if ((s = check_sizes(p)) != SM_OK) return s;
    const int64_t rows = transposed ? p->n_vox : p->n_rays;
    int32_t *cnt = nullptr;
    int64_t *ptr = nullptr;
    hipError_t e = hipMalloc(&cnt, sizeof(int32_t) * rows);
    if (e == hipSuccess) e = hipMalloc(&ptr, sizeof(int64_t) * (rows + 1));
    if (e != hipSuccess) {
        hipFree(cnt);
        hipFree(ptr);
        return set_error(SM_ENOMEM, "stored-W count buffers: %s", hipGetErrorString(e));
    }
    s = count_rows(p, transposed, ptr, cnt, nnz, 0);
    hipFree(cnt);
    hipFree(ptr);
    return s;
}

sm_status sm_stored_fill(const sm_plan *p, int32_t transposed, sm_precision values, int64_t nnz,
                         int64_t *row_ptr, int32_t *col_idx, void *val, void *stream)
{
    if (!p) return set_error(SM_EINVAL, "plan is NULL");
    if (!row_ptr || (nnz > 0 && (!col_idx || !val)))
        return set_error(SM_EINVAL, "row_ptr, col_idx and val are required");
    if (values != SM_FP32 && values != SM_FP64) return set_error(SM_EINVAL, "bad value precision");
    sm_status s = smk::check_plan_device(p);
    if (s != SM_OK) return s;
    if ((s = check_sizes(p)) != SM_OK) return s;
    if (nnz < 0 || nnz > 2147483647LL)
        return set_error(SM_EUNSUPPORTED, "stored W holds at most 2^31-1 entries (nnz %lld)", (long long)nnz);
    hipStream_t st = (hipStream_t)stream;
    const bool f64 = values == SM_FP64;
    const size_t vb = f64 ? 8 : 4;
    const int64_t rows = transposed ? p->n_vox : p->n_rays;
    const double tau_keep = 1e-12 * p->G.a * p->G.b * p->G.c;
    int32_t *cnt = nullptr, *keys = nullptr;
    void *vin = nullptr, *tmp = nullptr;
    const int64_t ne = nnz > 0 ? nnz : 1;
    hipError_t e = hipMalloc(&cnt, sizeof(int32_t) * rows);
    if (e == hipSuccess) e = hipMalloc(&keys, sizeof(int32_t) * ne);
    if (e == hipSuccess) e = hipMalloc(&vin, vb * ne);
    if (e != hipSuccess) {
        hipFree(cnt);
        hipFree(keys);
        hipFree(vin);
        return set_error(SM_ENOMEM, "stored-W build buffers: %s", hipGetErrorString(e));
    }
    int64_t got = 0;
    s = count_rows(p, transposed, row_ptr, cnt, &got, st);
    if (s == SM_OK && got != nnz)
        s = set_error(SM_ERANGE, "the matrix has %lld entries, %lld given", (long long)got, (long long)nnz);
    if (s == SM_OK && nnz > 0) {
        e = hipMemsetAsync(cnt, 0, sizeof(int32_t) * rows, st);
        if (e == hipSuccess)
            e = transposed ? smk::launch_csr_fill_vox(p->G, f64, tau_keep, row_ptr, cnt, keys, vin, st)
                           : smk::launch_csr_fill(p->G, f64, tau_keep, row_ptr, cnt, keys, vin, st);
        size_t tb = 0;
        if (e == hipSuccess) {
            e = f64 ? hipcub::DeviceSegmentedRadixSort::SortPairs(
                          nullptr, tb, keys, col_idx, (const double *)vin, (double *)val, (int)nnz,
                          (int)rows, row_ptr, row_ptr + 1, 0, 32, st)
                    : hipcub::DeviceSegmentedRadixSort::SortPairs(
                          nullptr, tb, keys, col_idx, (const float *)vin, (float *)val, (int)nnz,
                          (int)rows, row_ptr, row_ptr + 1, 0, 32, st);
        }
        if (e == hipSuccess) e = hipMalloc(&tmp, tb > 0 ? tb : 1);
        if (e == hipSuccess) {
            e = f64 ? hipcub::DeviceSegmentedRadixSort::SortPairs(
                          tmp, tb, keys, col_idx, (const double *)vin, (double *)val, (int)nnz,
                          (int)rows, row_ptr, row_ptr + 1, 0, 32, st)
                    : hipcub::DeviceSegmentedRadixSort::SortPairs(
                          tmp, tb, keys, col_idx, (const float *)vin, (float *)val, (int)nnz,
                          (int)rows, row_ptr, row_ptr + 1, 0, 32, st);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) s = hip_err(e, "stored-W fill");
    }
    hipFree(cnt);
    hipFree(keys);
    hipFree(vin);
    hipFree(tmp);
    return s;
}

sm_status sm_stored_apply(int64_t n_rows, const int64_t *row_ptr, const int32_t *col_idx,
                          const void *val, sm_precision values, const void *x, void *y,
                          int32_t batch, int64_t x_stride, int64_t y_stride, void *stream)
{
    if (n_rows < 0 || batch < 1) return set_error(SM_EINVAL, "n_rows >= 0 and batch >= 1 required");
    if (!row_ptr || !col_idx || !val || !x || !y) return set_error(SM_EINVAL, "NULL array");
    if (values != SM_FP32 && values != SM_FP64) return set_error(SM_EINVAL, "bad value precision");
    if (batch > 1 && (x_stride <= 0 || y_stride < n_rows))
        return set_error(SM_EINVAL, "batch strides must be positive and y_stride >= n_rows");
    hipStream_t st = (hipStream_t)stream;
    const size_t vb = values == SM_FP64 ? 8 : 4;
    hipError_t e = hipSuccess;
    for (int b = 0; b < batch && e == hipSuccess; ++b) {
        const void *xb = (const char *)x + (size_t)b * x_stride * vb;
        void *yb = (char *)y + (size_t)b * y_stride * vb;
        e = values == SM_FP64 ? smk::spmv_t<double>(n_rows, row_ptr, col_idx, val, xb, yb, st)
                              : smk::spmv_t<float>(n_rows, row_ptr, col_idx, val, xb, yb, st);
    }
    return e == hipSuccess ? SM_OK : hip_err(e, "sm_stored_apply launch");
}

}  // extern "C"
