// sm_line.hip -- the line-based comparison model of Sec. IV: every detector
// element sampled by k (2D) or k x k (3D) lines from the source, the lines'
// weights averaged (the paper's complexity experiment raises k to approach
// the area-based matrix), applied matrix-free in both directions.
//
// Sub-line g along a detector axis (g = m k + s) sits at c0 + (g + 1/2) h / k.
// In the view frame (depth, lateral, height) its points are alpha (D, u, v),
// alpha >= 0; in world coordinates S + alpha d with S = (s cos phi,
// s sin phi, 0) and d = (-(D cos phi + u sin phi), u cos phi - D sin phi, v).
// Voxel j holds the piece alpha in [max(0, lo_x, lo_y, lo_z), min(hi_x, hi_y,
// hi_z)], (lo, hi) the crossings of its two planes on each axis; on an axis
// the line runs parallel to, the voxel whose half-open slab holds S keeps it.
// Weight of a piece:
//   length : R (a1 - a0) / k^(dim-1), R = |d| (the classical line model);
//   measure: the midpoint rule over the element of its exact measure in line
//            coordinates, h_u D (a1^2 - a0^2) / (2k) in 2D and
//            h_u h_v D (a1^3 - a0^3) / (3k^2) in 3D, which tends to the
//            consistent W of Sec. I as k grows.
//
// Forward: one thread per detector element walks each of its sub-lines voxel
// by voxel, taking the plane crossings of the axes in increasing alpha; sums
// in FP64, one store, no atomics.  Adjoint: a gather over the sub-lines whose
// detector points fall in the voxel's shadow, each clipped against the voxel.
// In 3D one workgroup owns a voxel column with its lanes along z: per view
// the first wave clips the column's sub-line columns (the x and y slabs,
// shared by every voxel of the column) into LDS, and each lane adds the z
// slab of its own voxel for the sub-line rows of its shadow.  In 2D one
// thread owns a pixel.  Both sides compute
// every crossing, direction and weight with the same expressions under
// contraction off, so a piece has one value in both directions and the pair
// is adjoint up to the order of the sums.
#include "sm_plan.h"

namespace smk {

struct LineCfg {
    int k;
    int measure;        // 0: path lengths, 1: measure quadrature
    double du_k, dv_k;  // sub-line pitch along u and v
    double wl;          // 1 / k^(dim-1)
    double wm;          // h_u D / (2k) in 2D, h_u h_v D / (3k^2) in 3D
    int vtab;           // 3D adjoint: sub-row positions and inverses tabled in LDS
};

constexpr int kLineEntries = 16;  // sub-line columns of one view clipped per pass (3D adjoint)
constexpr int kLineVtab = 1024;   // largest tabled sub-row count

__device__ __forceinline__ double plane_coord(double o, double h, int p)
{
#pragma clang fp contract(off)
    return o + (double)p * h;
}

__device__ __forceinline__ double plane_alpha(double o, double h, int p, double S, double inv)
{
#pragma clang fp contract(off)
    return (plane_coord(o, h, p) - S) * inv;
}

__device__ __forceinline__ double sub_pos(double c0, double hk, int g)
{
#pragma clang fp contract(off)
    return c0 + ((double)g + 0.5) * hk;
}

__device__ __forceinline__ void sub_dir(double D, double cp, double sp, double u, double &dx, double &dy)
{
#pragma clang fp contract(off)
    dx = -(D * cp + u * sp);
    dy = u * cp - D * sp;
}

__device__ __forceinline__ double line_norm(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    return sqrt(dx * dx + dy * dy + dz * dz);
}

template <int DIM>
__device__ __forceinline__ double piece_weight(const LineCfg &C, double R, double a0, double a1)
{
#pragma clang fp contract(off)
    if (!C.measure) return C.wl * R * (a1 - a0);
    if (DIM == 2) return C.wm * ((a1 - a0) * (a1 + a0));
    return C.wm * ((a1 - a0) * (a1 * a1 + a1 * a0 + a0 * a0));
}

// Voxel index of the half-open slab holding S on an axis the line is parallel to.
__device__ __forceinline__ double par_cell(double o, double h, double S) { return floor((S - o) / h); }

// Crossing interval of voxel i on one axis; false when the line misses the slab.
__device__ __forceinline__ bool slab(double o, double h, int i, double S, double d, double &lo, double &hi)
{
    if (d != 0.0) {
        const double inv = 1.0 / d;
        const double a = plane_alpha(o, h, i, S, inv), b = plane_alpha(o, h, i + 1, S, inv);
        lo = fmin(a, b);
        hi = fmax(a, b);
        return true;
    }
    lo = -INFINITY;
    hi = INFINITY;
    return par_cell(o, h, S) == (double)i;
}

// One axis of a sub-line walk: next plane p to cross, current voxel i.
struct Axis {
    double S, o, h, inv, an;  // an: crossing of plane p (infinity when none is left)
    int n, st, p, i;
};

__device__ __forceinline__ bool axis_init(Axis &A, double S, double d, double o, double h, int n, double &lo,
                                          double &hi)
{
    A.S = S;
    A.o = o;
    A.h = h;
    A.n = n;
    A.an = INFINITY;
    A.p = 0;
    if (d != 0.0) {
        A.inv = 1.0 / d;
        A.st = d > 0.0 ? 1 : -1;
        const double a0 = plane_alpha(o, h, 0, S, A.inv), a1 = plane_alpha(o, h, n, S, A.inv);
        lo = fmin(a0, a1);
        hi = fmax(a0, a1);
        A.i = 0;
        return true;
    }
    A.inv = 0.0;
    A.st = 0;
    lo = -INFINITY;
    hi = INFINITY;
    const double f = par_cell(o, h, S);
    A.i = f >= 0.0 && f < (double)n ? (int)f : 0;
    return f >= 0.0 && f < (double)n;
}

// Place the axis at the entry alpha_in: the voxel with crossing(entry plane)
// <= alpha_in < crossing(exit plane), found from the position and corrected
// against the crossings themselves (the position is off by rounding only).
__device__ __forceinline__ void axis_start(Axis &A, double d, double ain)
{
    if (A.st == 0) return;
    const double f = (A.S + ain * d - A.o) / A.h;
    int p;
    if (A.st > 0) {  // planes crossed: p, p + 1, ..., n; voxel p - 1
        p = (int)fmin(fmax(floor(f) + 1.0, 1.0), (double)A.n);
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            if (p > 1 && plane_alpha(A.o, A.h, p - 1, A.S, A.inv) > ain) --p;
            if (p < A.n && plane_alpha(A.o, A.h, p, A.S, A.inv) <= ain) ++p;
        }
        A.i = p - 1;
    } else {  // planes crossed: p, p - 1, ..., 0; voxel p
        p = (int)fmin(fmax(ceil(f) - 1.0, 0.0), (double)(A.n - 1));
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            if (p < A.n - 1 && plane_alpha(A.o, A.h, p + 1, A.S, A.inv) > ain) ++p;
            if (p > 0 && plane_alpha(A.o, A.h, p, A.S, A.inv) <= ain) --p;
        }
        A.i = p;
    }
    A.p = p;
    A.an = plane_alpha(A.o, A.h, p, A.S, A.inv);
}

__device__ __forceinline__ void axis_step(Axis &A)
{
    A.p += A.st;
    A.i += A.st;
    A.an = A.p >= 0 && A.p <= A.n ? plane_alpha(A.o, A.h, A.p, A.S, A.inv) : INFINITY;
}

__device__ __forceinline__ int clampi(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

template <typename T, int DIM, int NBAT>
__global__ void __launch_bounds__(256) line_fwd_kernel(DevGeom G, LineCfg C, const T *__restrict__ x,
                                                        T *__restrict__ y, int b0)
{
    const int64_t nel = (int64_t)G.n_p * G.nv * G.nu;
    const int64_t e = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (e >= nel) return;
    const int m = (int)(e % G.nu);
    const int64_t rest = e / G.nu;
    const int r = (int)(rest % G.nv);
    const int view = (int)(rest / G.nv);
    const double2 cs = G.trig[view];
    const double cp = cs.x, sp = cs.y;
    const double Sx = G.s * cp, Sy = G.s * sp;
    const size_t nvox = (size_t)G.nx * G.ny * G.nz;
    const int cap = G.nx + G.ny + (DIM == 3 ? G.nz : 0) + 4;
    double acc[NBAT];
#pragma unroll
    for (int b = 0; b < NBAT; ++b) acc[b] = 0.0;
    const int kv = DIM == 3 ? C.k : 1;
    for (int t = 0; t < kv; ++t) {
        const double v = DIM == 3 ? sub_pos(G.v0, C.dv_k, r * C.k + t) : 0.0;
        for (int s = 0; s < C.k; ++s) {
            const double u = sub_pos(G.u0, C.du_k, m * C.k + s);
            double dx, dy;
            sub_dir(G.D, cp, sp, u, dx, dy);
            Axis X, Y, Z;
            double lx, hx, ly, hy, lz = -INFINITY, hz = INFINITY;
            bool ok = axis_init(X, Sx, dx, G.x0, G.a, G.nx, lx, hx);
            ok = axis_init(Y, Sy, dy, G.y0, G.b, G.ny, ly, hy) && ok;
            if (DIM == 3) ok = axis_init(Z, 0.0, v, G.z0, G.c, G.nz, lz, hz) && ok;
            const double ain = fmax(0.0, fmax(lx, fmax(ly, lz)));
            const double aout = fmin(hx, fmin(hy, hz));
            if (!ok || !(ain < aout)) continue;
            axis_start(X, dx, ain);
            axis_start(Y, dy, ain);
            if (DIM == 3) axis_start(Z, v, ain);
            const double R = C.measure ? 0.0 : line_norm(dx, dy, DIM == 3 ? v : 0.0);
            double acur = ain;
            for (int it = 0; it < cap; ++it) {
                const double an = fmin(X.an, DIM == 3 ? fmin(Y.an, Z.an) : Y.an);
                const double a1 = fmin(an, aout);
                if (a1 > acur) {
                    const double w = piece_weight<DIM>(C, R, acur, a1);
                    const int iz = DIM == 3 ? clampi(Z.i, G.nz) : 0;
                    const size_t vox = ((size_t)iz * G.ny + clampi(Y.i, G.ny)) * G.nx + clampi(X.i, G.nx);
#pragma unroll
                    for (int b = 0; b < NBAT; ++b) acc[b] += w * (double)x[(size_t)(b0 + b) * nvox + vox];
                }
                if (!(an < aout)) break;
                if (X.an == an) axis_step(X);
                else if (Y.an == an) axis_step(Y);
                else if (DIM == 3) axis_step(Z);
                acur = a1 > acur ? a1 : acur;
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NBAT; ++b) y[(size_t)(b0 + b) * nel + e] = T(acc[b]);
}

// First and last sub-line whose detector point lies in (lo, hi), one extra
// on each side against rounding (a sub-line that misses gets weight zero).
__device__ __forceinline__ void sub_range(double lo, double hi, double c0, double hk, int n, int &g0, int &g1)
{
    const double f0 = ceil((lo - c0) / hk - 0.5) - 1.0, f1 = floor((hi - c0) / hk - 0.5) + 1.0;
    g0 = (int)fmax(f0, 0.0);
    g1 = (int)fmin(f1, (double)(n - 1));
}

template <typename T, int DIM, int NBAT>
__global__ void __launch_bounds__(256) line_back_kernel(DevGeom G, LineCfg C, const T *__restrict__ y,
                                                         T *__restrict__ x, int b0)
{
    const int64_t nvox = (int64_t)G.nx * G.ny * G.nz;
    const int64_t q = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (q >= nvox) return;
    // voxel order (iy, ix, iz), z fastest: a wave shares its voxel column
    const int iz = (int)(q % G.nz);
    const int64_t col = q / G.nz;
    const int ix = (int)(col % G.nx), iy = (int)(col / G.nx);
    const double X0 = G.x0 + (double)ix * G.a, X1 = G.x0 + (double)(ix + 1) * G.a;
    const double Y0 = G.y0 + (double)iy * G.b, Y1 = G.y0 + (double)(iy + 1) * G.b;
    const double Z0 = G.z0 + (double)iz * G.c, Z1 = G.z0 + (double)(iz + 1) * G.c;
    const int nsu = G.nu * C.k, nsv = G.nv * C.k;
    const int64_t nel = (int64_t)G.n_p * G.nv * G.nu;
    double acc[NBAT];
#pragma unroll
    for (int b = 0; b < NBAT; ++b) acc[b] = 0.0;
    for (int view = 0; view < G.n_p; ++view) {
        const double2 cs = G.trig[view];
        const double cp = cs.x, sp = cs.y;
        const double Sx = G.s * cp, Sy = G.s * sp;
        // detector shadow: u over the column's four corners, v over the eight
        double umin = INFINITY, umax = -INFINITY, lmin = INFINITY, lmax = -INFINITY;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double xc = (c & 1) ? X1 : X0, yc = (c & 2) ? Y1 : Y0;
            const double l = G.s - (xc * cp + yc * sp), t = yc * cp - xc * sp;
            const double u = G.D * t / l;
            umin = fmin(umin, u);
            umax = fmax(umax, u);
            lmin = fmin(lmin, l);
            lmax = fmax(lmax, l);
        }
        int gu0, gu1, gv0 = 0, gv1 = 0;
        sub_range(umin, umax, G.u0, C.du_k, nsu, gu0, gu1);
        if (DIM == 3) {
            const double vmin = fmin(G.D * Z0 / lmin, G.D * Z0 / lmax);
            const double vmax = fmax(G.D * Z1 / lmin, G.D * Z1 / lmax);
            sub_range(vmin, vmax, G.v0, C.dv_k, nsv, gv0, gv1);
        }
        const T *yv = y + (size_t)view * G.nv * G.nu;
        for (int gu = gu0; gu <= gu1; ++gu) {
            const double u = sub_pos(G.u0, C.du_k, gu);
            double dx, dy;
            sub_dir(G.D, cp, sp, u, dx, dy);
            double lx, hx, ly, hy;
            if (!slab(G.x0, G.a, ix, Sx, dx, lx, hx)) continue;
            if (!slab(G.y0, G.b, iy, Sy, dy, ly, hy)) continue;
            const double A0 = fmax(0.0, fmax(lx, ly)), A1 = fmin(hx, hy);
            if (!(A0 < A1)) continue;
            const int m = gu / C.k;
            if (DIM == 2) {
                const double R = C.measure ? 0.0 : line_norm(dx, dy, 0.0);
                const double w = piece_weight<DIM>(C, R, A0, A1);
#pragma unroll
                for (int b = 0; b < NBAT; ++b) acc[b] += w * (double)yv[(size_t)(b0 + b) * nel + m];
                continue;
            }
            for (int gv = gv0; gv <= gv1; ++gv) {
                const double v = sub_pos(G.v0, C.dv_k, gv);
                double lz, hz;
                if (!slab(G.z0, G.c, iz, 0.0, v, lz, hz)) continue;
                const double a0 = fmax(0.0, fmax(lx, fmax(ly, lz))), a1 = fmin(hx, fmin(hy, hz));
                if (!(a0 < a1)) continue;
                const double R = C.measure ? 0.0 : line_norm(dx, dy, v);
                const double w = piece_weight<DIM>(C, R, a0, a1);
                const size_t el = (size_t)(gv / C.k) * G.nu + m;
#pragma unroll
                for (int b = 0; b < NBAT; ++b) acc[b] += w * (double)yv[(size_t)(b0 + b) * nel + el];
            }
        }
    }
    const size_t out = ((size_t)iz * G.ny + iy) * G.nx + ix;
#pragma unroll
    for (int b = 0; b < NBAT; ++b) x[(size_t)(b0 + b) * nvox + out] = T(acc[b]);
}

// 3D adjoint.  A pass clips, for VB = blockDim / kLineEntries views at once,
// up to kLineEntries sub-line columns of each view's shadow (one thread each)
// into LDS; then every lane adds its voxel's pieces for those entries.
// LDS: sub-row table v, 1/v (C.vtab) | per-view meta | entries (per sub-line
// column: the column's alpha interval [A0, A1], its inverses, the
// direction's x and y, the detector column).
struct LineMeta {
    int g0, n;  // first sub-line column of the column's shadow and their count
};

template <typename T, int NBAT>
__global__ void __launch_bounds__(256) line_back3d_kernel(DevGeom G, LineCfg C, const T *__restrict__ y,
                                                           T *__restrict__ x, int b0)
{
    extern __shared__ __align__(16) unsigned char lsm[];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int VB = nthr / kLineEntries;  // views per pass
    const int nsu = G.nu * C.k, nsv = G.nv * C.k;
    double *vt = reinterpret_cast<double *>(lsm);
    double *vinv = vt + (C.vtab ? nsv : 0);
    double *eA0 = vinv + (C.vtab ? nsv : 0);  // [VB][kLineEntries] each
    double *eA1 = eA0 + nthr, *eiA0 = eA1 + nthr, *eiA1 = eiA0 + nthr, *edx = eiA1 + nthr, *edy = edx + nthr;
    int *em = reinterpret_cast<int *>(edy + nthr);
    LineMeta *meta = reinterpret_cast<LineMeta *>(em + nthr);  // [VB]

    const int col = xcd_remap(blockIdx.x, gridDim.x);
    const int ix = col % G.nx, iy = col / G.nx;
    const double X0 = G.x0 + (double)ix * G.a, X1 = G.x0 + (double)(ix + 1) * G.a;
    const double Y0 = G.y0 + (double)iy * G.b, Y1 = G.y0 + (double)(iy + 1) * G.b;
    const int64_t nel = (int64_t)G.n_p * G.nv * G.nu;
    const size_t nvox = (size_t)G.nx * G.ny * G.nz;
    const double inv_dvk = 1.0 / C.dv_k, inv_k = 1.0 / C.k;
    if (C.vtab) {
        for (int g = tid; g < nsv; g += nthr) {
            const double v = sub_pos(G.v0, C.dv_k, g);
            vt[g] = v;
            vinv[g] = v != 0.0 ? 1.0 / v : 0.0;
        }
    }
    // this thread's slot in the clip phase
    const int cs_v = tid / kLineEntries, cs_i = tid - cs_v * kLineEntries;
    for (int z0 = 0; z0 < G.nz; z0 += nthr) {
        const int iz = z0 + tid;
        const bool act = iz < G.nz;
        // the voxel's z planes, as plane_alpha forms them (the source is at z = 0)
        const double Z0 = plane_coord(G.z0, G.c, iz), Z1 = plane_coord(G.z0, G.c, iz + 1);
        double acc[NBAT];
#pragma unroll
        for (int b = 0; b < NBAT; ++b) acc[b] = 0.0;
        for (int vbase = 0; vbase < G.n_p; vbase += VB) {
            for (int gb = 0;; gb += kLineEntries) {
                __syncthreads();  // previous entries consumed (and the table written)
                {
                    const int view = vbase + cs_v;
                    double A0 = INFINITY, A1 = -INFINITY, dx = 0.0, dy = 0.0;
                    int m = 0, n = 0, g0 = 0;
                    if (view < G.n_p) {
                        const double2 cs = G.trig[view];
                        const double cp = cs.x, sp = cs.y;
                        // the column's shadow (a range only: sub-lines outside it miss)
                        double umin = INFINITY, umax = -INFINITY;
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            const double xc = (c & 1) ? X1 : X0, yc = (c & 2) ? Y1 : Y0;
                            const double l = G.s - (xc * cp + yc * sp), t = yc * cp - xc * sp;
                            const double u = G.D * t / l;
                            umin = fmin(umin, u);
                            umax = fmax(umax, u);
                        }
                        int g1;
                        sub_range(umin, umax, G.u0, C.du_k, nsu, g0, g1);
                        n = g1 >= g0 ? g1 - g0 + 1 : 0;
                        const int i = gb + cs_i;
                        if (i < n) {
                            const int gu = g0 + i;
                            const double u = sub_pos(G.u0, C.du_k, gu);
                            sub_dir(G.D, cp, sp, u, dx, dy);
                            double lx, hx, ly, hy;
                            if (slab(G.x0, G.a, ix, G.s * cp, dx, lx, hx) &&
                                slab(G.y0, G.b, iy, G.s * sp, dy, ly, hy)) {
                                A0 = fmax(0.0, fmax(lx, ly));
                                A1 = fmin(hx, hy);
                            }
                            m = (int)(((double)gu + 0.5) * inv_k);
                        }
                    }
                    eA0[tid] = A0;
                    eA1[tid] = A1;
                    eiA0[tid] = 1.0 / A0;
                    eiA1[tid] = 1.0 / A1;
                    edx[tid] = dx;
                    edy[tid] = dy;
                    em[tid] = m;
                    if (cs_i == 0) meta[cs_v] = LineMeta{g0, n};
                }
                __syncthreads();
                int nmax = 0;
                for (int vs = 0; vs < VB; ++vs) {
                    const int view = vbase + vs;
                    const int n = meta[vs].n;
                    nmax = n > nmax ? n : nmax;
                    const int ne = n - gb < kLineEntries ? n - gb : kLineEntries;
                    if (!act || ne <= 0) continue;
                    const T *yv = y + (size_t)view * G.nv * G.nu;
                    const int base = vs * kLineEntries;
                    for (int e = base; e < base + ne; ++e) {
                        const double A0 = eA0[e], A1 = eA1[e];
                        if (!(A0 < A1)) continue;
                        const double dx = edx[e], dy = edy[e];
                        const int m = em[e];
                        // heights v whose line meets the slab for some alpha in [A0, A1]
                        // (a 1e-9 sub-row margin covers rounding; the slab test decides)
                        const double vlo = Z0 >= 0.0 ? Z0 * eiA1[e] : Z0 * eiA0[e];
                        const double vhi = Z1 >= 0.0 ? Z1 * eiA0[e] : Z1 * eiA1[e];
                        const int gv0 = (int)fmax(ceil((vlo - G.v0) * inv_dvk - 0.5 - 1e-9), 0.0);
                        const int gv1 = (int)fmin(floor((vhi - G.v0) * inv_dvk - 0.5 + 1e-9), (double)(nsv - 1));
                        for (int gv = gv0; gv <= gv1; ++gv) {
                            double v, iv;
                            if (C.vtab) {
                                v = vt[gv];
                                iv = vinv[gv];
                            } else {
                                v = sub_pos(G.v0, C.dv_k, gv);
                                iv = v != 0.0 ? 1.0 / v : 0.0;
                            }
                            double lz, hz;
                            if (v != 0.0) {
                                const double a = (Z0 - 0.0) * iv, bq = (Z1 - 0.0) * iv;  // plane_alpha
                                lz = fmin(a, bq);
                                hz = fmax(a, bq);
                            } else {
                                if (par_cell(G.z0, G.c, 0.0) != (double)iz) continue;
                                lz = -INFINITY;
                                hz = INFINITY;
                            }
                            const double a0 = fmax(A0, lz), a1 = fmin(A1, hz);
                            if (!(a0 < a1)) continue;
                            const double R = C.measure ? 0.0 : line_norm(dx, dy, v);
                            const double w = piece_weight<3>(C, R, a0, a1);
                            const int r = (int)(((double)gv + 0.5) * inv_k);  // gv / k: the fraction stays >= 1/(2k)
                            const size_t el = (size_t)r * G.nu + m;
#pragma unroll
                            for (int b = 0; b < NBAT; ++b) acc[b] += w * (double)yv[(size_t)(b0 + b) * nel + el];
                        }
                    }
                }
                if (gb + kLineEntries >= nmax) break;
            }
        }
        if (act) {
            const size_t out = ((size_t)iz * G.ny + iy) * G.nx + ix;
#pragma unroll
            for (int b = 0; b < NBAT; ++b) x[(size_t)(b0 + b) * nvox + out] = T(acc[b]);
        }
    }
}

static size_t line_back3d_lds(const DevGeom &G, const LineCfg &C, int nthr)
{
    const size_t tab = C.vtab ? 2 * sizeof(double) * (size_t)G.nv * C.k : 0;
    return tab + (size_t)nthr * (6 * sizeof(double) + sizeof(int)) +
           sizeof(LineMeta) * (size_t)(nthr / kLineEntries);
}

template <typename T, int DIM>
static hipError_t line_launch(const DevGeom &G, const LineCfg &C, bool adjoint, const void *in, void *out,
                              int B, hipStream_t st)
{
    const int64_t n = adjoint ? (int64_t)G.nx * G.ny * G.nz : (int64_t)G.n_p * G.nv * G.nu;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    for (int b0 = 0; b0 < B;) {
        const int nb = B - b0 >= 4 ? 4 : 1;
        if (adjoint && DIM == 3) {
            // one workgroup per voxel column, lanes along z
            const int zt = G.nz < 256 ? G.nz : 256;
            const int nt = 64 * ((zt + 63) / 64);
            const size_t lds = line_back3d_lds(G, C, nt);
            const unsigned cols = (unsigned)((int64_t)G.nx * G.ny);
            if (nb == 4)
                hipLaunchKernelGGL((line_back3d_kernel<T, 4>), dim3(cols), dim3(nt), lds, st, G, C,
                                   (const T *)in, (T *)out, b0);
            else
                hipLaunchKernelGGL((line_back3d_kernel<T, 1>), dim3(cols), dim3(nt), lds, st, G, C,
                                   (const T *)in, (T *)out, b0);
        } else if (adjoint) {
            if (nb == 4)
                hipLaunchKernelGGL((line_back_kernel<T, DIM, 4>), dim3(blocks), dim3(256), 0, st, G, C,
                                   (const T *)in, (T *)out, b0);
            else
                hipLaunchKernelGGL((line_back_kernel<T, DIM, 1>), dim3(blocks), dim3(256), 0, st, G, C,
                                   (const T *)in, (T *)out, b0);
        } else {
            if (nb == 4)
                hipLaunchKernelGGL((line_fwd_kernel<T, DIM, 4>), dim3(blocks), dim3(256), 0, st, G, C,
                                   (const T *)in, (T *)out, b0);
            else
                hipLaunchKernelGGL((line_fwd_kernel<T, DIM, 1>), dim3(blocks), dim3(256), 0, st, G, C,
                                   (const T *)in, (T *)out, b0);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        b0 += nb;
    }
    return hipSuccess;
}

}  // namespace smk

using smk::set_error;

namespace {

sm_status line_apply(const sm_plan *p, int32_t k, sm_line_weight weight, const void *in, void *out,
                     int32_t batch, void *stream, bool adjoint)
{
    if (!p) return set_error(SM_EINVAL, "plan is NULL");
    if (!in || !out) return set_error(SM_EINVAL, "input or output pointer is NULL");
    if (batch < 1) return set_error(SM_EINVAL, "batch must be >= 1");
    if (k < 1 || k > SM_LINE_MAX_K) return set_error(SM_EINVAL, "k must be in [1, %d]", SM_LINE_MAX_K);
    if (weight != SM_LINE_LENGTH && weight != SM_LINE_MEASURE) return set_error(SM_EINVAL, "bad line weighting");
    const smk::DevGeom &G = p->G;
    if ((int64_t)G.n_p * G.nv * G.nu > ((int64_t)1 << 38) || (int64_t)G.nx * G.ny * G.nz > ((int64_t)1 << 38))
        return set_error(SM_EUNSUPPORTED, "problem too large for the line projector");
    sm_status s = smk::check_plan_device(p);
    if (s != SM_OK) return s;
    smk::LineCfg C;
    C.k = k;
    C.measure = weight == SM_LINE_MEASURE;
    C.du_k = G.du / k;
    C.dv_k = G.dv / k;
    C.wl = G.dim == 3 ? 1.0 / ((double)k * k) : 1.0 / k;
    C.wm = G.dim == 3 ? G.du * G.dv * G.D / (3.0 * k * k) : G.du * G.D / (2.0 * k);
    C.vtab = (int64_t)G.nv * k <= smk::kLineVtab;
    hipStream_t st = (hipStream_t)stream;
    const bool f64 = p->prec == SM_FP64;
    hipError_t e;
    if (G.dim == 3)
        e = f64 ? smk::line_launch<double, 3>(G, C, adjoint, in, out, batch, st)
                : smk::line_launch<float, 3>(G, C, adjoint, in, out, batch, st);
    else
        e = f64 ? smk::line_launch<double, 2>(G, C, adjoint, in, out, batch, st)
                : smk::line_launch<float, 2>(G, C, adjoint, in, out, batch, st);
    if (e != hipSuccess)
        return set_error(SM_EDEVICE, "%s launch: %s", adjoint ? "sm_line_back" : "sm_line_forward",
                         hipGetErrorString(e));
    return SM_OK;
}

}  // namespace

extern "C" {

sm_status sm_line_forward(const sm_plan *plan, int32_t k, sm_line_weight weight, const void *x, void *y,
                          int32_t batch, void *stream)
{
    return line_apply(plan, k, weight, x, y, batch, stream, false);
}

sm_status sm_line_back(const sm_plan *plan, int32_t k, sm_line_weight weight, const void *y, void *x,
                       int32_t batch, void *stream)
{
    return line_apply(plan, k, weight, y, x, batch, stream, true);
}

}  // extern "C"
