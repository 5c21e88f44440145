// sm_solve.hip -- reconstruction on top of the projector pair (Sec. IV,
// eq. "exp_tikh"): power iteration for ||W||_2, CGLS and Nesterov's
// accelerated gradient for  1/2 |s W u - p|^2 + lambda/2 |u|^2.
//
// Everything is stream-ordered.  Scalars of the iterations (norms, step
// sizes) live in a small device array S[batch][kNS] and the vector kernels
// read them from there, so an iteration never waits for the host.  Dot
// products accumulate in FP64 in a fixed order: a fixed grid of kDotBlocks
// workgroups each sums a grid-stride slice and reduces it in a tree, then one
// workgroup per batch element reduces the partials in a tree.
#include <math.h>

#include "sm_plan.h"

namespace smk {

constexpr int kDotBlocks = 512;  // fixed: the reduction order does not depend on the device
constexpr int kNS = 8;           // device scalars per batch element
enum { S_GAMMA = 0, S_DELTA = 1, S_ALPHA = 2, S_BETA = 3, S_GNEW = 4, S_SIG2 = 5, S_STEP = 6, S_NRM = 7 };
constexpr int kVecThreads = 256;

template <typename T>
__global__ void __launch_bounds__(256) dot_partial(const T *__restrict__ a, const T *__restrict__ b,
                                                   int64_t n, double *__restrict__ part)
{
    __shared__ double red[256];
    const int bb = blockIdx.y, tid = threadIdx.x;
    a += (int64_t)bb * n;
    b += (int64_t)bb * n;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += (int64_t)kDotBlocks * 256)
        acc += (double)a[i] * (double)b[i];
    red[tid] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) part[bb * kDotBlocks + blockIdx.x] = red[0];
}

// S[b][slot] = (add ? S[b][slot] : 0) + scale * sum of the partials of b
__global__ void __launch_bounds__(kDotBlocks) dot_final(const double *__restrict__ part, double *S,
                                                        int slot, double scale, int add)
{
    __shared__ double red[kDotBlocks];
    const int bb = blockIdx.x, tid = threadIdx.x;
    red[tid] = part[bb * kDotBlocks + tid];
    __syncthreads();
    for (int w = kDotBlocks / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) S[bb * kNS + slot] = (add ? S[bb * kNS + slot] : 0.0) + scale * red[0];
}

// y = a x + b y (host scalars)
template <typename T>
__global__ void __launch_bounds__(256) axpby_k(T *__restrict__ y, const T *__restrict__ x, int64_t n,
                                               double a, double b)
{
    const int bb = blockIdx.y;
    y += (int64_t)bb * n;
    x += (int64_t)bb * n;
    const T ta = T(a), tb = T(b);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        y[i] = ta * x[i] + tb * y[i];
}

// y += sign * S[b][slot] * x
template <typename T>
__global__ void __launch_bounds__(256) axpy_dev(T *__restrict__ y, const T *__restrict__ x, int64_t n,
                                                const double *__restrict__ S, int slot, double sign)
{
    const int bb = blockIdx.y;
    y += (int64_t)bb * n;
    x += (int64_t)bb * n;
    const T a = T(sign * S[bb * kNS + slot]);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        y[i] += a * x[i];
}

// p = s + S[b][slot] * p
template <typename T>
__global__ void __launch_bounds__(256) xpby_dev(T *__restrict__ p, const T *__restrict__ s, int64_t n,
                                                const double *__restrict__ S, int slot)
{
    const int bb = blockIdx.y;
    p += (int64_t)bb * n;
    s += (int64_t)bb * n;
    const T beta = T(S[bb * kNS + slot]);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = s[i] + beta * p[i];
}

// out = a + sign * S[b][slot] * g
template <typename T>
__global__ void __launch_bounds__(256) step_dev(T *__restrict__ out, const T *__restrict__ a,
                                                const T *__restrict__ g, int64_t n,
                                                const double *__restrict__ S, int slot, double sign)
{
    const int bb = blockIdx.y;
    out += (int64_t)bb * n;
    a += (int64_t)bb * n;
    g += (int64_t)bb * n;
    const T c = T(sign * S[bb * kNS + slot]);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = a[i] + c * g[i];
}

// v *= 1 / sqrt(S[b][slot])  (no-op for a zero norm)
template <typename T>
__global__ void __launch_bounds__(256) normalise_dev(T *__restrict__ v, int64_t n,
                                                     const double *__restrict__ S, int slot)
{
    const int bb = blockIdx.y;
    v += (int64_t)bb * n;
    const double q = S[bb * kNS + slot];
    const T c = T(q > 0.0 ? 1.0 / sqrt(q) : 1.0);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        v[i] *= c;
}

template <typename T>
__global__ void __launch_bounds__(256) copy_k(T *__restrict__ dst, const T *__restrict__ src, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        dst[i] = src[i];
}

// CG scalars: op 0: alpha = gamma / delta; op 1: beta = gnew / gamma, gamma = gnew
__global__ void cg_scalars(double *S, int B, int op)
{
    const int bb = threadIdx.x;
    if (bb >= B) return;
    double *s = S + bb * kNS;
    if (op == 0) {
        s[S_ALPHA] = s[S_DELTA] > 0.0 ? s[S_GAMMA] / s[S_DELTA] : 0.0;
    } else {
        s[S_BETA] = s[S_GAMMA] > 0.0 ? s[S_GNEW] / s[S_GAMMA] : 0.0;
        s[S_GAMMA] = s[S_GNEW];
    }
}

// step = 1 / (wscale^2 norm^2 + lambda) for every batch element
__global__ void nag_step(double *S, int B, const double *norm, double ws2, double lambda)
{
    const int bb = threadIdx.x;
    if (bb >= B) return;
    const double L = ws2 * norm[0] * norm[0] + lambda;
    S[bb * kNS + S_STEP] = L > 0.0 ? 1.0 / L : 0.0;
}

// dst[b] = S[b][slot]   (history of a scalar)
__global__ void take_scalar(double *dst, const double *S, int B, int slot)
{
    const int bb = threadIdx.x;
    if (bb < B) dst[bb] = S[bb * kNS + slot];
}

__global__ void sqrt_scalar(double *dst, const double *S, int slot)
{
    if (threadIdx.x == 0) dst[0] = sqrt(S[slot]);
}

}  // namespace smk

using namespace smk;

namespace {

struct Vec {
    void *p;
    int64_t n;  // elements per batch element
};

// Workspace carving: [projector ws | vectors | S | partials], 256-byte aligned.
struct SolveWs {
    int64_t proj;  // projector workspace bytes
    int64_t off[4];
    int64_t s_off, part_off, total;
};

SolveWs solve_layout(const sm_plan *p, sm_solver kind, int B, int64_t proj)
{
    const int64_t es = p->prec == SM_FP64 ? 8 : 4;
    const int64_t N = p->n_vox, M = p->n_rays;
    // vectors per solver: CGLS r, q (sino), s, p (vol); NAG res (sino), g, z, xprev (vol);
    // power u (sino), v, w (vol)
    int64_t sz[4] = {0, 0, 0, 0};
    if (kind == SM_SOLVER_CGLS) { sz[0] = M; sz[1] = M; sz[2] = N; sz[3] = N; }
    else if (kind == SM_SOLVER_NAG) { sz[0] = M; sz[1] = N; sz[2] = N; sz[3] = N; }
    else { sz[0] = M; sz[1] = N; sz[2] = N; }
    SolveWs L;
    L.proj = proj;
    int64_t o = align256(proj);
    for (int i = 0; i < 4; ++i) {
        L.off[i] = o;
        o = align256(o + sz[i] * B * es);
    }
    L.s_off = o;
    o = align256(o + (int64_t)B * kNS * 8);
    L.part_off = o;
    o = align256(o + (int64_t)B * kDotBlocks * 8);
    L.total = o;
    return L;
}

// The operator pair a solver applies: the consistent W of sm_forward/sm_back
// (line_k = 0) or the line-based model of sm_line_forward/sm_line_back.
struct Op {
    int line_k;
    sm_line_weight weight;
};

struct Ctx {
    const sm_plan *p;
    hipStream_t st;
    int B;
    bool f64;
    void *ws;
    int64_t proj;
    double *S, *part;
    Op op;
};

dim3 vec_grid(int64_t n, int B)
{
    int64_t nb = (n + kVecThreads - 1) / kVecThreads;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    return dim3((unsigned)nb, (unsigned)B);
}

hipError_t dot(Ctx &c, const void *a, const void *b, int64_t n, int slot, double scale, bool add)
{
    const dim3 g(kDotBlocks, c.B);
    if (c.f64)
        hipLaunchKernelGGL(dot_partial<double>, g, dim3(256), 0, c.st, (const double *)a, (const double *)b, n, c.part);
    else
        hipLaunchKernelGGL(dot_partial<float>, g, dim3(256), 0, c.st, (const float *)a, (const float *)b, n, c.part);
    hipLaunchKernelGGL(dot_final, dim3(c.B), dim3(kDotBlocks), 0, c.st, c.part, c.S, slot, scale, add ? 1 : 0);
    return hipGetLastError();
}

hipError_t axpby(Ctx &c, void *y, const void *x, int64_t n, double a, double b)
{
    if (c.f64) hipLaunchKernelGGL(axpby_k<double>, vec_grid(n, c.B), dim3(256), 0, c.st, (double *)y, (const double *)x, n, a, b);
    else hipLaunchKernelGGL(axpby_k<float>, vec_grid(n, c.B), dim3(256), 0, c.st, (float *)y, (const float *)x, n, a, b);
    return hipGetLastError();
}

hipError_t axpy_s(Ctx &c, void *y, const void *x, int64_t n, int slot, double sign)
{
    if (c.f64) hipLaunchKernelGGL(axpy_dev<double>, vec_grid(n, c.B), dim3(256), 0, c.st, (double *)y, (const double *)x, n, c.S, slot, sign);
    else hipLaunchKernelGGL(axpy_dev<float>, vec_grid(n, c.B), dim3(256), 0, c.st, (float *)y, (const float *)x, n, c.S, slot, sign);
    return hipGetLastError();
}

hipError_t xpby_s(Ctx &c, void *pv, const void *s, int64_t n, int slot)
{
    if (c.f64) hipLaunchKernelGGL(xpby_dev<double>, vec_grid(n, c.B), dim3(256), 0, c.st, (double *)pv, (const double *)s, n, c.S, slot);
    else hipLaunchKernelGGL(xpby_dev<float>, vec_grid(n, c.B), dim3(256), 0, c.st, (float *)pv, (const float *)s, n, c.S, slot);
    return hipGetLastError();
}

hipError_t step_s(Ctx &c, void *out, const void *a, const void *g, int64_t n, int slot, double sign)
{
    if (c.f64) hipLaunchKernelGGL(step_dev<double>, vec_grid(n, c.B), dim3(256), 0, c.st, (double *)out, (const double *)a, (const double *)g, n, c.S, slot, sign);
    else hipLaunchKernelGGL(step_dev<float>, vec_grid(n, c.B), dim3(256), 0, c.st, (float *)out, (const float *)a, (const float *)g, n, c.S, slot, sign);
    return hipGetLastError();
}

hipError_t normalise_s(Ctx &c, void *v, int64_t n, int slot)
{
    if (c.f64) hipLaunchKernelGGL(normalise_dev<double>, vec_grid(n, c.B), dim3(256), 0, c.st, (double *)v, n, c.S, slot);
    else hipLaunchKernelGGL(normalise_dev<float>, vec_grid(n, c.B), dim3(256), 0, c.st, (float *)v, n, c.S, slot);
    return hipGetLastError();
}

hipError_t copy(Ctx &c, void *dst, const void *src, int64_t n_total)
{
    const dim3 g = vec_grid(n_total, 1);
    if (c.f64) hipLaunchKernelGGL(copy_k<double>, g, dim3(256), 0, c.st, (double *)dst, (const double *)src, n_total);
    else hipLaunchKernelGGL(copy_k<float>, g, dim3(256), 0, c.st, (float *)dst, (const float *)src, n_total);
    return hipGetLastError();
}

hipError_t scalars(Ctx &c, int op)
{
    hipLaunchKernelGGL(cg_scalars, dim3(1), dim3(64), 0, c.st, c.S, c.B, op);
    return hipGetLastError();
}

hipError_t record(Ctx &c, double *hist, int row, int slot)
{
    if (!hist) return hipSuccess;
    hipLaunchKernelGGL(take_scalar, dim3(1), dim3(64), 0, c.st, hist + (int64_t)row * c.B, c.S, c.B, slot);
    return hipGetLastError();
}

sm_status fwd(Ctx &c, const void *x, void *y)
{
    if (c.op.line_k > 0) return sm_line_forward(c.p, c.op.line_k, c.op.weight, x, y, c.B, (void *)c.st);
    return sm_forward(c.p, x, y, c.B, c.ws, c.proj, (void *)c.st);
}

sm_status bwd(Ctx &c, const void *y, void *x)
{
    if (c.op.line_k > 0) return sm_line_back(c.p, c.op.line_k, c.op.weight, y, x, c.B, (void *)c.st);
    return sm_back(c.p, y, x, c.B, c.ws, c.proj, (void *)c.st);
}

sm_status start(const sm_plan *p, sm_solver kind, int32_t batch, void *ws, int64_t ws_bytes,
                void *stream, Op op, Ctx &c, SolveWs &L)
{
    if (!p) return set_error(SM_EINVAL, "plan is NULL");
    if (op.line_k < 0 || op.line_k > SM_LINE_MAX_K)
        return set_error(SM_EINVAL, "k must be in [1, %d]", SM_LINE_MAX_K);
    if (op.weight != SM_LINE_LENGTH && op.weight != SM_LINE_MEASURE)
        return set_error(SM_EINVAL, "bad line weighting");
    c.op = op;
    if (batch < 1 || batch > 64) return set_error(SM_EINVAL, "batch must be in [1, 64]");
    sm_status s = check_plan_device(p);
    if (s != SM_OK) return s;
    int64_t proj = 0;
    s = sm_workspace_size(p, batch, &proj);
    if (s != SM_OK) return s;
    L = solve_layout(p, kind, batch, proj);
    if (!ws || ws_bytes < L.total)
        return set_error(SM_EINVAL, "solver workspace too small: need %lld bytes", (long long)L.total);
    c.p = p;
    c.st = (hipStream_t)stream;
    c.B = batch;
    c.f64 = p->prec == SM_FP64;
    c.ws = ws;
    c.proj = proj;
    c.S = (double *)((char *)ws + L.s_off);
    c.part = (double *)((char *)ws + L.part_off);
    return SM_OK;
}

#define SM_TRY(expr)                                                      \
    do {                                                                  \
        hipError_t e_ = (expr);                                           \
        if (e_ != hipSuccess)                                             \
            return set_error(SM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)
#define SM_TRYS(expr)                    \
    do {                                 \
        sm_status s_ = (expr);           \
        if (s_ != SM_OK) return s_;      \
    } while (0)

}  // namespace

extern "C" {

sm_status sm_solver_workspace_size(const sm_plan *p, sm_solver kind, int32_t batch, int64_t *bytes)
{
    if (!p) return set_error(SM_EINVAL, "plan is NULL");
    if (!bytes) return set_error(SM_EINVAL, "bytes is NULL");
    if (kind != SM_SOLVER_CGLS && kind != SM_SOLVER_NAG && kind != SM_SOLVER_POWER)
        return set_error(SM_EINVAL, "unknown solver");
    if (batch < 1 || batch > 64) return set_error(SM_EINVAL, "batch must be in [1, 64]");
    if (kind == SM_SOLVER_POWER && batch != 1) return set_error(SM_EINVAL, "power iteration takes batch 1");
    int64_t proj = 0;
    SM_TRYS(sm_workspace_size(p, batch, &proj));
    *bytes = solve_layout(p, kind, batch, proj).total;
    return SM_OK;
}

}  // extern "C"

namespace {

sm_status power_norm_op(const sm_plan *p, Op op, const void *v0, int32_t iters, double *norm_dev,
                        void *ws, int64_t ws_bytes, void *stream)
{
    if (!v0 || !norm_dev) return set_error(SM_EINVAL, "v0 and norm_dev are required");
    if (iters < 1) return set_error(SM_EINVAL, "iters must be >= 1");
    Ctx c;
    SolveWs L;
    SM_TRYS(start(p, SM_SOLVER_POWER, 1, ws, ws_bytes, stream, op, c, L));
    const int64_t N = p->n_vox, M = p->n_rays;
    char *b = (char *)ws;
    void *u = b + L.off[0], *v = b + L.off[1], *w = b + L.off[2];
    SM_TRY(copy(c, v, v0, N));
    SM_TRY(dot(c, v, v, N, S_NRM, 1.0, false));
    SM_TRY(normalise_s(c, v, N, S_NRM));
    for (int k = 0; k < iters; ++k) {
        SM_TRYS(fwd(c, v, u));
        SM_TRY(dot(c, u, u, M, S_SIG2, 1.0, false));  // Rayleigh quotient v^T W^T W v
        SM_TRYS(bwd(c, u, w));
        SM_TRY(dot(c, w, w, N, S_NRM, 1.0, false));
        SM_TRY(copy(c, v, w, N));
        SM_TRY(normalise_s(c, v, N, S_NRM));
    }
    hipLaunchKernelGGL(sqrt_scalar, dim3(1), dim3(64), 0, c.st, norm_dev, c.S, (int)S_SIG2);
    SM_TRY(hipGetLastError());
    return SM_OK;
}

}  // namespace

extern "C" {

sm_status sm_power_norm(const sm_plan *p, const void *v0, int32_t iters, double *norm_dev,
                        void *ws, int64_t ws_bytes, void *stream)
{
    return power_norm_op(p, Op{0, SM_LINE_LENGTH}, v0, iters, norm_dev, ws, ws_bytes, stream);
}

sm_status sm_line_power_norm(const sm_plan *p, int32_t k, sm_line_weight weight, const void *v0,
                             int32_t iters, double *norm_dev, void *ws, int64_t ws_bytes, void *stream)
{
    if (k < 1) return set_error(SM_EINVAL, "k must be in [1, %d]", SM_LINE_MAX_K);
    return power_norm_op(p, Op{k, weight}, v0, iters, norm_dev, ws, ws_bytes, stream);
}

sm_status sm_cgls(const sm_plan *p, const void *y, void *x, int32_t batch, int32_t iters,
                  double lambda, double wscale, double *hist_dev, void *ws, int64_t ws_bytes,
                  void *stream)
{
    if (!y || !x) return set_error(SM_EINVAL, "y and x are required");
    if (iters < 0 || !(lambda >= 0.0) || !(wscale > 0.0) || !isfinite(lambda) || !isfinite(wscale))
        return set_error(SM_EINVAL, "need iters >= 0, lambda >= 0, wscale > 0");
    Ctx c;
    SolveWs L;
    SM_TRYS(start(p, SM_SOLVER_CGLS, batch, ws, ws_bytes, stream, Op{0, SM_LINE_LENGTH}, c, L));
    const int64_t N = p->n_vox, M = p->n_rays;
    const double s2 = wscale * wscale;
    char *b = (char *)ws;
    void *r = b + L.off[0], *q = b + L.off[1], *sv = b + L.off[2], *pv = b + L.off[3];
    // r = p - s W x ; sv = s W^T r - lambda x ; pv = sv ; gamma = |sv|^2
    SM_TRYS(fwd(c, x, r));
    SM_TRY(axpby(c, r, y, M, 1.0, -wscale));
    SM_TRYS(bwd(c, r, sv));
    SM_TRY(axpby(c, sv, x, N, -lambda, wscale));
    SM_TRY(copy(c, pv, sv, N * c.B));
    SM_TRY(dot(c, sv, sv, N, S_GAMMA, 1.0, false));
    SM_TRY(record(c, hist_dev, 0, S_GAMMA));
    for (int k = 0; k < iters; ++k) {
        // q = W p ; delta = s^2 |q|^2 + lambda |p|^2 ; alpha = gamma / delta
        SM_TRYS(fwd(c, pv, q));
        SM_TRY(dot(c, q, q, M, S_DELTA, s2, false));
        if (lambda > 0.0) SM_TRY(dot(c, pv, pv, N, S_DELTA, lambda, true));
        SM_TRY(scalars(c, 0));
        // x += alpha p ; r -= alpha s q
        SM_TRY(axpy_s(c, x, pv, N, S_ALPHA, 1.0));
        SM_TRY(axpy_s(c, r, q, M, S_ALPHA, -wscale));
        // sv = s W^T r - lambda x ; gnew = |sv|^2 ; beta = gnew / gamma
        SM_TRYS(bwd(c, r, sv));
        SM_TRY(axpby(c, sv, x, N, -lambda, wscale));
        SM_TRY(dot(c, sv, sv, N, S_GNEW, 1.0, false));
        SM_TRY(record(c, hist_dev, k + 1, S_GNEW));
        SM_TRY(scalars(c, 1));
        // p = sv + beta p
        SM_TRY(xpby_s(c, pv, sv, N, S_BETA));
    }
    return SM_OK;
}

}  // extern "C"

namespace {

sm_status nag_op(const sm_plan *p, Op op, const void *y, void *x, int32_t batch, int32_t iters,
                 double lambda, double wscale, const double *norm_dev, double *hist_dev, void *ws,
                 int64_t ws_bytes, void *stream)
{
    if (!y || !x || !norm_dev) return set_error(SM_EINVAL, "y, x and norm_dev are required");
    if (iters < 0 || !(lambda >= 0.0) || !(wscale > 0.0) || !isfinite(lambda) || !isfinite(wscale))
        return set_error(SM_EINVAL, "need iters >= 0, lambda >= 0, wscale > 0");
    Ctx c;
    SolveWs L;
    SM_TRYS(start(p, SM_SOLVER_NAG, batch, ws, ws_bytes, stream, op, c, L));
    const int64_t N = p->n_vox, M = p->n_rays;
    char *b = (char *)ws;
    void *res = b + L.off[0], *g = b + L.off[1], *z = b + L.off[2], *xprev = b + L.off[3];
    hipLaunchKernelGGL(nag_step, dim3(1), dim3(64), 0, c.st, c.S, c.B, norm_dev, wscale * wscale, lambda);
    SM_TRY(hipGetLastError());
    SM_TRY(copy(c, z, x, N * c.B));
    SM_TRY(copy(c, xprev, x, N * c.B));
    double t = 1.0;
    for (int k = 0; k < iters; ++k) {
        // g = s W^T (s W z - p) + lambda z
        SM_TRYS(fwd(c, z, res));
        SM_TRY(axpby(c, res, y, M, -1.0, wscale));
        SM_TRYS(bwd(c, res, g));
        SM_TRY(axpby(c, g, z, N, lambda, wscale));
        if (hist_dev) {
            SM_TRY(dot(c, g, g, N, S_NRM, 1.0, false));
            SM_TRY(record(c, hist_dev, k, S_NRM));
        }
        // x = z - g / L ; z = x + (t - 1) / t' (x - xprev) ; xprev = x
        SM_TRY(step_s(c, x, z, g, N, S_STEP, -1.0));
        const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
        const double mom = (t - 1.0) / tn;
        SM_TRY(copy(c, z, x, N * c.B));
        SM_TRY(axpby(c, z, xprev, N, -mom, 1.0 + mom));
        SM_TRY(copy(c, xprev, x, N * c.B));
        t = tn;
    }
    return SM_OK;
}

}  // namespace

extern "C" {

sm_status sm_nag(const sm_plan *p, const void *y, void *x, int32_t batch, int32_t iters,
                 double lambda, double wscale, const double *norm_dev, double *hist_dev, void *ws,
                 int64_t ws_bytes, void *stream)
{
    return nag_op(p, Op{0, SM_LINE_LENGTH}, y, x, batch, iters, lambda, wscale, norm_dev, hist_dev, ws,
                  ws_bytes, stream);
}

sm_status sm_line_nag(const sm_plan *p, int32_t k, sm_line_weight weight, const void *y, void *x,
                      int32_t batch, int32_t iters, double lambda, double wscale, const double *norm_dev,
                      double *hist_dev, void *ws, int64_t ws_bytes, void *stream)
{
    if (k < 1) return set_error(SM_EINVAL, "k must be in [1, %d]", SM_LINE_MAX_K);
    return nag_op(p, Op{k, weight}, y, x, batch, iters, lambda, wscale, norm_dev, hist_dev, ws, ws_bytes,
                  stream);
}

}  // extern "C"
