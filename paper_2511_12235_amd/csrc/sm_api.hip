// sm_api.hip -- the C ABI declared in include/sm.h: plan creation and
// validation, argument checks, workspace rules and kernel dispatch.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "sm_plan.h"

using smk::DevGeom;
using smk::LaunchCfg;

// Views per record chunk: keep the records of one chunk under 4 GiB (larger
// chunks mean fewer launches and fewer partly filled rounds of workgroups).
static const int64_t kRecordBudget = (int64_t)4 << 30;
// Resident waves of one adjoint round on MI355X: 256 CUs x 4 SIMDs x 6 waves.
static const int64_t kResidentWaves = 256 * 4 * 6;

namespace {

thread_local std::string g_err;

sm_status fail(sm_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
sm_status fail(sm_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

sm_status hip_fail(hipError_t e, const char *what)
{
    return fail(SM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

sm_status check_device(const sm_plan *p)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != p->device)
        return fail(SM_EINVAL, "plan was created on device %d but device %d is current", p->device, dev);
    return SM_OK;
}

const int kTimingPairs = 4096;

void timing_release(SmTiming *t)
{
    for (hipEvent_t e : t->ev) hipEventDestroy(e);
    t->ev.clear();
    t->kernel.clear();
    t->used = 0;
    t->overflow = false;
    t->on = false;
}

// Records the opening event of a timed dispatch; returns its pair index or -1.
int tm_begin(const sm_plan *p, int kernel, hipStream_t st)
{
    SmTiming *t = p->tm;
    std::lock_guard<std::mutex> lk(t->mu);
    if (!t->on) return -1;
    if (t->used >= kTimingPairs) {
        t->overflow = true;
        return -1;
    }
    const int q = t->used++;
    t->kernel[q] = kernel;
    hipEventRecord(t->ev[2 * q], st);
    return q;
}

void tm_end(const sm_plan *p, int q, hipStream_t st)
{
    if (q < 0) return;
    SmTiming *t = p->tm;
    std::lock_guard<std::mutex> lk(t->mu);
    hipEventRecord(t->ev[2 * q + 1], st);
}

// Widest detector-column span of any adjoint tile (tw x th pixels) over all
// views, computed with the same corner arithmetic the kernel uses.
__global__ void tile_span_kernel(DevGeom G, int tw, int th, int *out)
{
    const int ntx = (G.nx + tw - 1) / tw, nty = (G.ny + th - 1) / th;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)ntx * nty * G.n_p) return;
    const int view = (int)(q / ((int64_t)ntx * nty));
    const int t = (int)(q - (int64_t)view * ntx * nty);
    const int ty = t / ntx, tx = t - ty * ntx;
    const double2 cs = G.trig[view];
    int k0, k1;
    smk::corner_columns(G, cs.x, cs.y, tx * tw, min(tx * tw + tw, G.nx), ty * th,
                        min(ty * th + th, G.ny), k0, k1);
    if (k1 >= k0) atomicMax(out, k1 - k0 + 1);
}

}  // namespace

namespace smk {
sm_status set_error(sm_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

sm_status check_plan_device(const sm_plan *p) { return check_device(p); }
}  // namespace smk

namespace smk {

// Volume buffers of one call, behind the records of a chunk: the forward's
// voxel columns and max |x| per batch element, the adjoint's `groups`
// partial volumes.
int64_t fwd_volume_bytes(const sm_plan *p, int64_t batch)
{
    const int64_t es = p->prec == SM_FP64 ? 8 : 4;
    return smk::align256((int64_t)p->G.nx * p->G.ny * batch * p->G.nz * es) +
           smk::align256(batch * (int64_t)sizeof(unsigned));
}

int64_t back_volume_bytes(const sm_plan *p, int64_t batch, int groups)
{
    const int64_t npix = (int64_t)p->G.nx * p->G.ny;
    const int64_t es = p->prec == SM_FP64 ? 8 : 4;
    return (int64_t)groups * npix * batch * p->G.nz * es;
}

int64_t workspace_bytes(const sm_plan *p, int64_t batch)
{
    if (p->G.dim != 3) return 0;
    const int64_t fwd = fwd_volume_bytes(p, batch);
    const int64_t adj = back_volume_bytes(p, batch, p->L.back_groups);
    // the records of one chunk precede the volume buffer unless the plan keeps them
    return (p->rec_cache ? 0 : p->RL.data_off) + (fwd > adj ? fwd : adj);
}

int64_t record_bytes(const sm_plan *p)
{
    if (p->G.dim != 3) return 0;
    const int64_t chunks = (p->G.n_p + p->RL.views - 1) / p->RL.views;
    return chunks * p->RL.data_off;
}

// y = W x for a 3D plan: records of each chunk of RL.views views (from the
// plan's copy when it keeps them, else built into `recws`), the volume
// buffer at `vol`.
hipError_t run_forward3d(const sm_plan *p, const smk::RecLayout &RL, const void *x, void *y,
                         int batch, void *recws, void *vol, hipStream_t st)
{
    const bool f64 = p->prec == SM_FP64;
    void *X = vol;
    unsigned *xmax = (unsigned *)((char *)vol + smk::align256((int64_t)p->G.nx * p->G.ny * batch *
                                                              p->G.nz * (f64 ? 8 : 4)));
    int q = tm_begin(p, SM_KERNEL_PREFIX, st);
    hipError_t e = smk::launch_to_columns(x, X, xmax, f64, batch, p->G.nz, p->G.ny, p->G.nx, st);
    tm_end(p, q, st);
    for (int v0 = 0; v0 < p->G.n_p && e == hipSuccess; v0 += RL.views) {
        const int nvc = p->G.n_p - v0 < RL.views ? p->G.n_p - v0 : RL.views;
        void *rws = recws;
        if (p->rec_cache) {
            rws = (char *)p->rec_cache + (int64_t)(v0 / RL.views) * RL.data_off;
        } else {
            q = tm_begin(p, SM_KERNEL_RECORDS, st);
            e = smk::launch_records(p->G, RL, f64, v0, nvc, rws, st);
            tm_end(p, q, st);
            if (e != hipSuccess) break;
        }
        q = tm_begin(p, SM_KERNEL_FORWARD, st);
        e = smk::launch_fwd3d(p->G, p->L, RL, f64, v0, nvc, rws, X, xmax, y, batch, st);
        tm_end(p, q, st);
    }
    return e;
}

// x = W^T y for a 3D plan, records as run_forward3d; L.back_groups partial
// volumes at `vol`.
hipError_t run_back3d(const sm_plan *p, const smk::RecLayout &RL, const LaunchCfg &L, const void *y,
                      void *x, int batch, void *recws, void *vol, hipStream_t st)
{
    const bool f64 = p->prec == SM_FP64;
    hipError_t e = hipSuccess;
    int q;
    for (int v0 = 0; v0 < p->G.n_p && e == hipSuccess; v0 += RL.views) {
        const int nvc = p->G.n_p - v0 < RL.views ? p->G.n_p - v0 : RL.views;
        void *rws = recws;
        if (p->rec_cache) {
            rws = (char *)p->rec_cache + (int64_t)(v0 / RL.views) * RL.data_off;
        } else {
            q = tm_begin(p, SM_KERNEL_RECORDS, st);
            e = smk::launch_records(p->G, RL, f64, v0, nvc, rws, st);
            tm_end(p, q, st);
            if (e != hipSuccess) break;
        }
        q = tm_begin(p, SM_KERNEL_ADJOINT, st);
        e = smk::launch_back3d(p->G, L, RL, f64, v0, nvc, rws, y, vol, batch, v0 == 0, st);
        tm_end(p, q, st);
    }
    if (e == hipSuccess) {
        q = tm_begin(p, SM_KERNEL_TRANSPOSE, st);
        e = smk::launch_from_columns(vol, x, f64 ? 8 : 4, batch, p->G.nz, p->G.ny, p->G.nx,
                                     L.back_groups, st);
        tm_end(p, q, st);
    }
    return e;
}

hipError_t run_apply2d(const sm_plan *p, bool adjoint, const void *in, void *out, int batch,
                       hipStream_t st)
{
    const bool f64 = p->prec == SM_FP64;
    const int q = tm_begin(p, adjoint ? SM_KERNEL_ADJOINT : SM_KERNEL_FORWARD, st);
    const hipError_t e = adjoint ? smk::launch_back2d(p->G, f64, in, out, batch, st)
                                 : smk::launch_fwd2d(p->G, f64, in, out, batch, st);
    tm_end(p, q, st);
    return e;
}

// Arguments of an operator call other than the workspace.
sm_status check_operands(const sm_plan *p, const void *in, void *out, int32_t batch)
{
    if (!p) return fail(SM_EINVAL, "plan is NULL");
    if (!in || !out) return fail(SM_EINVAL, "input or output pointer is NULL");
    if (batch < 1) return fail(SM_EINVAL, "batch must be >= 1");
    if (p->G.dim == 3 && p->G.ny * (int64_t)batch > 65535) return fail(SM_EUNSUPPORTED, "ny * batch > 65535");
    return check_device(p);
}

sm_status check_apply(const sm_plan *p, const void *in, void *out, int32_t batch, void *ws,
                      int64_t ws_bytes)
{
    sm_status s = check_operands(p, in, out, batch);
    if (s != SM_OK) return s;
    if (p->G.dim == 3) {
        const int64_t need = workspace_bytes(p, batch);
        if (!ws || ws_bytes < need)
            return fail(SM_EINVAL, "workspace too small: need %lld bytes", (long long)need);
    }
    return SM_OK;
}

}  // namespace smk

using smk::check_apply;
using smk::record_bytes;
using smk::run_apply2d;
using smk::run_back3d;
using smk::run_forward3d;
using smk::workspace_bytes;

extern "C" {

const char *sm_status_str(sm_status s)
{
    switch (s) {
    case SM_OK: return "ok";
    case SM_EINVAL: return "invalid argument";
    case SM_ENOMEM: return "out of memory";
    case SM_EDEVICE: return "device error";
    case SM_EUNSUPPORTED: return "unsupported";
    case SM_ERANGE: return "buffer too small";
    }
    return "unknown status";
}

const char *sm_last_error(void) { return g_err.c_str(); }

sm_status sm_plan_create(const sm_geometry *g, sm_precision precision, sm_plan **out)
{
    if (!out) return fail(SM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g) return fail(SM_EINVAL, "geometry is NULL");
    if (precision != SM_FP32 && precision != SM_FP64) return fail(SM_EINVAL, "bad precision");
    if (g->dim != 2 && g->dim != 3) return fail(SM_EINVAL, "dim must be 2 or 3");
    if (g->reserved0 != 0) return fail(SM_EINVAL, "reserved0 must be 0");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->n_p < 1 || g->det_ny < 1 || g->det_nz < 1)
        return fail(SM_EINVAL, "sizes must be positive");
    if (g->dim == 2 && (g->nz != 1 || g->det_nz != 1))
        return fail(SM_EINVAL, "2D geometry needs nz == 1 and det_nz == 1");
    if (!finite_pos(g->a) || !finite_pos(g->b) || (g->dim == 3 && !finite_pos(g->c)))
        return fail(SM_EINVAL, "voxel side lengths must be finite and positive");
    if (!finite_pos(g->dy) || (g->dim == 3 && !finite_pos(g->dz)))
        return fail(SM_EINVAL, "detector pitch must be finite and positive");
    if (!finite_pos(g->s) || !isfinite(g->d) || !(g->s + g->d > 0.0))
        return fail(SM_EINVAL, "need s > 0 and s + d > 0");
    const int64_t n_vox = (int64_t)g->nx * g->ny * g->nz;
    const int64_t n_rays = (int64_t)g->n_p * g->det_ny * g->det_nz;
    if (n_vox > (int64_t)1 << 40 || n_rays > (int64_t)1 << 40)
        return fail(SM_EUNSUPPORTED, "problem too large");
    if (g->dim == 3 && g->det_nz > 1024) return fail(SM_EUNSUPPORTED, "det_nz > 1024");
    if (g->dim == 3 && g->nz > 1024) return fail(SM_EUNSUPPORTED, "nz > 1024");

    const double c = g->dim == 3 ? g->c : 1.0;
    const double dz = g->dim == 3 ? g->dz : 1.0;
    DevGeom G{};
    G.dim = g->dim;
    G.nx = g->nx;
    G.ny = g->ny;
    G.nz = g->nz;
    G.n_p = g->n_p;
    G.nu = g->det_ny;
    G.nv = g->det_nz;
    G.a = g->a;
    G.b = g->b;
    G.c = c;
    G.x0 = isnan(g->x0) ? -0.5 * g->nx * g->a : g->x0;
    G.y0 = isnan(g->y0) ? -0.5 * g->ny * g->b : g->y0;
    G.z0 = isnan(g->z0) ? -0.5 * g->nz * c : g->z0;
    G.s = g->s;
    G.D = g->s + g->d;
    G.du = g->dy;
    G.dv = dz;
    G.u0 = isnan(g->det_y0) ? -0.5 * g->det_ny * g->dy : g->det_y0;
    G.v0 = isnan(g->det_z0) ? -0.5 * g->det_nz * dz : g->det_z0;
    if (!isfinite(G.x0) || !isfinite(G.y0) || !isfinite(G.z0) || !isfinite(G.u0) || !isfinite(G.v0))
        return fail(SM_EINVAL, "grid or detector corner is not finite");

    std::vector<double2> trig(g->n_p);
    for (int v = 0; v < g->n_p; ++v) {
        double cp, sp;
        if (g->trig) {
            cp = g->trig[2 * v];
            sp = g->trig[2 * v + 1];
        } else if (g->phi) {
            cp = cos(g->phi[v]);
            sp = sin(g->phi[v]);
        } else {
            const double ph = 2.0 * M_PI * (double)v / (double)g->n_p;
            cp = cos(ph);
            sp = sin(ph);
        }
        if (!isfinite(cp) || !isfinite(sp)) return fail(SM_EINVAL, "view %d: non-finite angle", v);
        trig[v] = make_double2(cp, sp);
        // every grid corner must lie in front of the source (depth l > 0)
        for (int q = 0; q < 4; ++q) {
            const double x = G.x0 + (double)((q & 1) ? g->nx : 0) * G.a;
            const double y = G.y0 + (double)((q >> 1) ? g->ny : 0) * G.b;
            if (!(G.s - (x * cp + y * sp) > 0.0))
                return fail(SM_EINVAL, "view %d: the source lies inside or behind the grid", v);
        }
    }
    std::vector<double> tau(G.nv + 1);
    for (int r = 0; r <= G.nv; ++r) tau[r] = (G.v0 + (double)r * G.dv) / G.D;

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    sm_plan *p = new (std::nothrow) sm_plan();
    if (!p) return fail(SM_ENOMEM, "host allocation");
    p->device = dev;
    p->prec = precision;
    p->n_vox = n_vox;
    p->n_rays = n_rays;
    p->tm = new (std::nothrow) SmTiming();
    if (!p->tm) {
        delete p;
        return fail(SM_ENOMEM, "host allocation");
    }
    e = hipMalloc(&p->d_trig, sizeof(double2) * g->n_p);
    if (e == hipSuccess) e = hipMalloc(&p->d_tau, sizeof(double) * (G.nv + 1));
    if (e != hipSuccess) {
        hipFree(p->d_trig);
        delete p->tm;
        delete p;
        return fail(SM_ENOMEM, "device tables: %s", hipGetErrorString(e));
    }
    e = hipMemcpy(p->d_trig, trig.data(), sizeof(double2) * g->n_p, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_tau, tau.data(), sizeof(double) * (G.nv + 1), hipMemcpyHostToDevice);
    G.trig = p->d_trig;
    G.tau = p->d_tau;
    p->G = G;

    LaunchCfg &L = p->L;
    L.fwd_threads = 64 * ((G.nv + 63) / 64);
    L.back_threads = 64 * ((G.nz + 63) / 64);
    {
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lds <= 0)
            lds = 65536;
        L.lds_budget = lds < 65536 ? lds : 65536;
    }
    // adjoint tiles (tw x th pixels) of the four batch widths, then one pixel
    const int tw[5] = {4, 4, 2, 2, 1}, th[5] = {4, 2, 2, 1, 1};
    for (int i = 0; i < 4; ++i) L.back_pcols[i] = 1;
    L.rspan = 1;
    // Adjoint view runs: enough workgroups x waves to fill the device for
    // small volumes, then the run count (up to 4x that) whose waves fill the
    // last round of resident waves best, so that no round of the launch runs
    // a third empty.  A round is taken as kResidentWaves, the single-volume
    // adjoint's occupancy on MI355X at 256^3; the rule uses the geometry and
    // these constants only, so results do not depend on the device.  (Taking
    // the round from the kernel's occupancy at each geometry instead chose 5
    // runs at 128^3, where 6 measured faster: 3.59 against 3.37 ms.)
    {
        const int64_t tiles = (int64_t)((G.nx + 3) / 4) * ((G.ny + 3) / 4);
        const int64_t waves = tiles * (L.back_threads / 64);
        const int64_t wv = waves > 0 ? waves : 1;
        int64_t gmin = (8192 + wv - 1) / wv;
        gmin = gmin < 1 ? 1 : (gmin > 16 ? 16 : gmin);
        auto fill = [&](int64_t g) {
            const int64_t tail = (wv * g) % kResidentWaves;
            return tail == 0 ? 1.0 : (double)tail / (double)kResidentWaves;
        };
        int64_t best = gmin;
        for (int64_t g = gmin; g <= 4 * gmin && g <= 16; ++g) {
            if (fill(g) >= 0.9) {
                best = g;
                break;
            }
            if (fill(g) > fill(best) + 1e-9) best = g;
        }
        L.back_groups = (int)best;
    }
    p->RL = smk::RecLayout{};
    if (e == hipSuccess && G.dim == 3) {
        int *d_span = nullptr;
        e = hipMalloc(&d_span, sizeof(int) * 6);
        if (e == hipSuccess) e = hipMemset(d_span, 0, sizeof(int) * 6);
        for (int i = 0; i < 5 && e == hipSuccess; ++i) {
            const int64_t n = (int64_t)((G.nx + tw[i] - 1) / tw[i]) * ((G.ny + th[i] - 1) / th[i]) * G.n_p;
            hipLaunchKernelGGL(tile_span_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, G,
                               tw[i], th[i], d_span + i);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = smk::launch_strip_count(G, d_span + 5, 0);
        int span[6] = {1, 1, 1, 1, 1, 1};
        if (e == hipSuccess) e = hipMemcpy(span, d_span, sizeof(int) * 6, hipMemcpyDeviceToHost);
        hipFree(d_span);
        for (int i = 0; i < 4; ++i) L.back_pcols[i] = span[i] > 0 ? span[i] : 1;
        L.rspan = span[4] > 0 ? span[4] : 1;
        const int cap = span[5] > 0 ? span[5] : 1;
        const size_t rsz = precision == SM_FP64 ? sizeof(smk::Rec<double>) : sizeof(smk::Rec<float>);
        const int64_t per_view = (int64_t)G.nu * cap * (int64_t)rsz;
        int64_t V = kRecordBudget / (per_view > 0 ? per_view : 1);
        V = V < 1 ? 1 : (V > G.n_p ? G.n_p : V);
        // chunks of equal size: no short last chunk with its own launch tails
        const int64_t nchunks = (G.n_p + V - 1) / V;
        V = (G.n_p + nchunks - 1) / nchunks;
        p->RL = smk::make_layout(cap, G.nx > G.ny ? G.nx : G.ny, (int)V, G.nu, G.nx, G.ny, rsz);
        const size_t need = smk::back3d_lds_min(G, L, precision == SM_FP64);
        if (e == hipSuccess && !smk::fwd3d_fits(L, precision == SM_FP64)) {
            hipFree(p->d_trig);
            hipFree(p->d_tau);
            delete p->tm;
            delete p;
            return fail(SM_EUNSUPPORTED, "too many detector rows for the forward's LDS staging");
        }
        if (e == hipSuccess && need > (size_t)L.lds_budget) {
            hipFree(p->d_trig);
            hipFree(p->d_tau);
            delete p->tm;
            delete p;
            return fail(SM_EUNSUPPORTED,
                        "detector footprint too wide: the adjoint needs %zu bytes of LDS per "
                        "workgroup, %d available", need, L.lds_budget);
        }
    }
    if (e != hipSuccess) {
        hipFree(p->d_trig);
        hipFree(p->d_tau);
        delete p->tm;
        delete p;
        return hip_fail(e, "plan tables");
    }
    *out = p;
    return SM_OK;
}

sm_status sm_plan_destroy(sm_plan *p)
{
    if (!p) return SM_OK;
    timing_release(p->tm);
    delete p->tm;
    hipFree(p->rec_cache);
    hipFree(p->d_trig);
    hipFree(p->d_tau);
    delete p;
    return SM_OK;
}

sm_status sm_plan_record_bytes(const sm_plan *p, int64_t *bytes)
{
    if (!p) return fail(SM_EINVAL, "plan is NULL");
    if (!bytes) return fail(SM_EINVAL, "bytes is NULL");
    *bytes = record_bytes(p);
    return SM_OK;
}

sm_status sm_plan_keep_records(sm_plan *p, int64_t max_bytes, void *stream)
{
    if (!p) return fail(SM_EINVAL, "plan is NULL");
    if (max_bytes < 0) return fail(SM_EINVAL, "max_bytes must be >= 0");
    sm_status s = check_device(p);
    if (s != SM_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if (max_bytes == 0 || p->G.dim != 3) {  // release (nothing is kept in 2D)
        if (p->rec_cache) {
            hipError_t e = hipStreamSynchronize(st);
            if (e == hipSuccess) e = hipDeviceSynchronize();
            if (e != hipSuccess) return hip_fail(e, "sm_plan_keep_records");
            hipFree(p->rec_cache);
            p->rec_cache = nullptr;
        }
        return SM_OK;
    }
    if (p->rec_cache) return SM_OK;
    const int64_t total = record_bytes(p);
    if (total > max_bytes)
        return fail(SM_ERANGE, "the records need %lld bytes, %lld allowed", (long long)total,
                    (long long)max_bytes);
    void *buf = nullptr;
    hipError_t e = hipMalloc(&buf, (size_t)total);
    if (e != hipSuccess) return fail(SM_ENOMEM, "record buffer of %lld bytes: %s", (long long)total,
                                     hipGetErrorString(e));
    const smk::RecLayout &RL = p->RL;
    const bool f64 = p->prec == SM_FP64;
    for (int v0 = 0; v0 < p->G.n_p && e == hipSuccess; v0 += RL.views) {
        const int nvc = p->G.n_p - v0 < RL.views ? p->G.n_p - v0 : RL.views;
        e = smk::launch_records(p->G, RL, f64, v0, nvc, (char *)buf + (int64_t)(v0 / RL.views) * RL.data_off, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        hipFree(buf);
        return hip_fail(e, "sm_plan_keep_records");
    }
    p->rec_cache = buf;
    return SM_OK;
}

sm_status sm_plan_sizes(const sm_plan *p, int64_t *n_vox, int64_t *n_rays)
{
    if (!p) return fail(SM_EINVAL, "plan is NULL");
    if (n_vox) *n_vox = p->n_vox;
    if (n_rays) *n_rays = p->n_rays;
    return SM_OK;
}

sm_status sm_plan_launch_shape(const sm_plan *p, int32_t *views_per_chunk, int32_t *adjoint_runs)
{
    if (!p) return fail(SM_EINVAL, "plan is NULL");
    const bool d3 = p->G.dim == 3;
    if (views_per_chunk) *views_per_chunk = d3 ? p->RL.views : p->G.n_p;
    if (adjoint_runs) *adjoint_runs = d3 ? p->L.back_groups : 1;
    return SM_OK;
}

sm_status sm_workspace_size(const sm_plan *p, int32_t batch, int64_t *bytes)
{
    if (!p) return fail(SM_EINVAL, "plan is NULL");
    if (!bytes) return fail(SM_EINVAL, "bytes is NULL");
    if (batch < 1) return fail(SM_EINVAL, "batch must be >= 1");
    *bytes = workspace_bytes(p, batch);
    return SM_OK;
}

sm_status sm_forward(const sm_plan *p, const void *x, void *y, int32_t batch, void *ws,
                     int64_t ws_bytes, void *stream)
{
    sm_status s = check_apply(p, x, y, batch, ws, ws_bytes);
    if (s != SM_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (p->G.dim == 2) {
        e = run_apply2d(p, false, x, y, batch, st);
    } else {
        void *vol = (char *)ws + (p->rec_cache ? 0 : p->RL.data_off);
        e = run_forward3d(p, p->RL, x, y, batch, ws, vol, st);
    }
    return e == hipSuccess ? SM_OK : hip_fail(e, "sm_forward launch");
}

sm_status sm_back(const sm_plan *p, const void *y, void *x, int32_t batch, void *ws,
                  int64_t ws_bytes, void *stream)
{
    sm_status s = check_apply(p, y, x, batch, ws, ws_bytes);
    if (s != SM_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (p->G.dim == 2) {
        e = run_apply2d(p, true, y, x, batch, st);
    } else {
        void *vol = (char *)ws + (p->rec_cache ? 0 : p->RL.data_off);
        e = run_back3d(p, p->RL, p->L, y, x, batch, ws, vol, st);
    }
    return e == hipSuccess ? SM_OK : hip_fail(e, "sm_back launch");
}

sm_status sm_timing_enable(sm_plan *p, int32_t enable)
{
    if (!p) return fail(SM_EINVAL, "plan is NULL");
    sm_status s = check_device(p);
    if (s != SM_OK) return s;
    SmTiming *t = p->tm;
    std::lock_guard<std::mutex> lk(t->mu);
    timing_release(t);
    if (!enable) return SM_OK;
    t->ev.assign(2 * kTimingPairs, nullptr);
    t->kernel.assign(kTimingPairs, 0);
    for (size_t i = 0; i < t->ev.size(); ++i) {
        hipError_t e = hipEventCreate(&t->ev[i]);
        if (e != hipSuccess) {
            t->ev.resize(i);
            timing_release(t);
            return hip_fail(e, "hipEventCreate");
        }
    }
    t->on = true;
    return SM_OK;
}

sm_status sm_timing_read(sm_plan *p, sm_kernel_time *times_host)
{
    if (!p) return fail(SM_EINVAL, "plan is NULL");
    if (!times_host) return fail(SM_EINVAL, "times_host is NULL");
    SmTiming *t = p->tm;
    std::lock_guard<std::mutex> lk(t->mu);
    if (!t->on) return fail(SM_EINVAL, "timing is not enabled on this plan");
    for (int k = 0; k < SM_KERNEL_COUNT; ++k) times_host[k] = sm_kernel_time{0, 0.0};
    for (int q = 0; q < t->used; ++q) {
        hipError_t e = hipEventSynchronize(t->ev[2 * q + 1]);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t->ev[2 * q], t->ev[2 * q + 1]);
        if (e != hipSuccess) {
            t->used = 0;
            return hip_fail(e, "timing events");
        }
        times_host[t->kernel[q]].launches += 1;
        times_host[t->kernel[q]].ms += (double)ms;
    }
    const bool over = t->overflow;
    t->used = 0;
    t->overflow = false;
    if (over) return fail(SM_ERANGE, "more dispatches than timing events; the excess was not timed");
    return SM_OK;
}

sm_status sm_footprints(const sm_plan *p, int32_t view, int32_t *boxes_host)
{
    if (!p) return fail(SM_EINVAL, "plan is NULL");
    if (!boxes_host) return fail(SM_EINVAL, "boxes_host is NULL");
    if (view < 0 || view >= p->G.n_p) return fail(SM_EINVAL, "view out of range");
    sm_status s = check_device(p);
    if (s != SM_OK) return s;
    int32_t *d = nullptr;
    const size_t bytes = sizeof(int32_t) * 4 * (size_t)p->n_vox;
    hipError_t e = hipMalloc(&d, bytes);
    if (e != hipSuccess) return fail(SM_ENOMEM, "footprint buffer: %s", hipGetErrorString(e));
    e = smk::launch_footprints(p->G, view, d, 0);
    if (e == hipSuccess) e = hipMemcpy(boxes_host, d, bytes, hipMemcpyDeviceToHost);
    hipFree(d);
    return e == hipSuccess ? SM_OK : hip_fail(e, "sm_footprints");
}

sm_status sm_weights_csr(const sm_plan *p, sm_precision values, int64_t *nnz_inout,
                         int64_t *row_ptr_host, int32_t *col_idx_host, void *val_host)
{
    if (!p) return fail(SM_EINVAL, "plan is NULL");
    if (!nnz_inout) return fail(SM_EINVAL, "nnz_inout is NULL");
    if (values != SM_FP32 && values != SM_FP64) return fail(SM_EINVAL, "bad value precision");
    if (row_ptr_host && (!col_idx_host || !val_host))
        return fail(SM_EINVAL, "col_idx_host and val_host are required with row_ptr_host");
    if (row_ptr_host && p->n_vox > 2147483647LL) return fail(SM_EUNSUPPORTED, "more than 2^31-1 voxels");
    if (p->n_vox * p->G.n_p > ((int64_t)1 << 40)) return fail(SM_EUNSUPPORTED, "problem too large for CSR");
    sm_status s = check_device(p);
    if (s != SM_OK) return s;
    const double tau_keep = 1e-12 * p->G.a * p->G.b * p->G.c;
    const int64_t M = p->n_rays;
    int32_t *d_cnt = nullptr, *d_cols = nullptr;
    int64_t *d_ptr = nullptr;
    void *d_vals = nullptr;
    hipError_t e = hipMalloc(&d_cnt, sizeof(int32_t) * M);
    if (e == hipSuccess) e = hipMalloc(&d_ptr, sizeof(int64_t) * (M + 1));
    if (e == hipSuccess) e = hipMemset(d_cnt, 0, sizeof(int32_t) * M);
    if (e == hipSuccess) e = smk::launch_csr_count(p->G, tau_keep, d_cnt, 0);
    if (e == hipSuccess) e = smk::launch_scan_counts(d_cnt, M, d_ptr, 0);
    int64_t nnz = 0;
    if (e == hipSuccess) e = hipMemcpy(&nnz, d_ptr + M, sizeof(int64_t), hipMemcpyDeviceToHost);
    sm_status st = SM_OK;
    if (e != hipSuccess) {
        st = hip_fail(e, "sm_weights_csr count");
    } else if (!row_ptr_host) {
        *nnz_inout = nnz;
    } else if (nnz > 400000000LL) {
        st = fail(SM_EUNSUPPORTED, "%lld entries exceed the CSR limit", (long long)nnz);
    } else if (*nnz_inout < nnz) {
        *nnz_inout = nnz;
        st = fail(SM_ERANGE, "need room for %lld entries", (long long)nnz);
    } else {
        const size_t vb = values == SM_FP64 ? 8 : 4;
        e = hipMalloc(&d_cols, sizeof(int32_t) * (nnz > 0 ? nnz : 1));
        if (e == hipSuccess) e = hipMalloc(&d_vals, vb * (nnz > 0 ? nnz : 1));
        if (e == hipSuccess) e = hipMemset(d_cnt, 0, sizeof(int32_t) * M);
        if (e == hipSuccess)
            e = smk::launch_csr_fill(p->G, values == SM_FP64, tau_keep, d_ptr, d_cnt, d_cols, d_vals, 0);
        if (e == hipSuccess) e = smk::launch_csr_sort(d_ptr, M, d_cols, d_vals, values == SM_FP64, 0);
        if (e == hipSuccess)
            e = hipMemcpy(row_ptr_host, d_ptr, sizeof(int64_t) * (M + 1), hipMemcpyDeviceToHost);
        if (e == hipSuccess && nnz > 0)
            e = hipMemcpy(col_idx_host, d_cols, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost);
        if (e == hipSuccess && nnz > 0) e = hipMemcpy(val_host, d_vals, vb * nnz, hipMemcpyDeviceToHost);
        if (e != hipSuccess) st = hip_fail(e, "sm_weights_csr fill");
        else *nnz_inout = nnz;
    }
    hipFree(d_cnt);
    hipFree(d_ptr);
    hipFree(d_cols);
    hipFree(d_vals);
    return st;
}

}  // extern "C"
