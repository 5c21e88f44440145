// sm_common.h -- device-side geometry and weight evaluation shared by the
// forward, adjoint and CSR kernels.
//
// Paper: Simbrunner, Krenn, Zach, Habring, "Computation of a Consistent
// System Matrix for Cone-beam Computed Tomography", arXiv 2511.12235.
//
// Coordinates.  For view phi with (cp, sp) = (cos phi, sin phi) a point p has
// depth l = s - (x cp + y sp) and lateral offset t = y cp - x sp (appendix,
// eq. "tan beta"); its detector coordinates are u = D t / l and v = D z / l
// (eq. "z expr 1" with tan(alpha) = v / D).  Everything below works in
// coordinates local to a voxel column: l' = l - lc and t' = t - tc, where
// (lc, tc) is the column centre, so magnitudes are O(voxel) and FP64
// cancellation happens only once, in lc and tc.
//
// Decomposition.  The boundary between detector columns is the vertical plane
// through the source t = (u_k / D) l; the boundary between rows is the tilted
// plane z = tau_r l with tau_r = v_r / D.  Seen from the top, detector column
// k cuts pixel (ix, iy) in a convex polygon P (the paper's triangles and
// trapezoids of Sec. III-B).  Because the row planes depend on (x, y) only
// through l, the volume of P x [za, za + c] below row plane r is
//     H = integral over P of clamp(e + tau l', 0, c) dA,  e = tau lc - za,
// a one-dimensional integral of the chord length w(l') of P against a clamped
// linear height.  w is piecewise linear with kinks at the vertex depths of P,
// so between consecutive vertex depths every piece is a prismatoid whose
// volume is exact by the prismatoid rule (appendix, "Prismatoid"); the piece
// cut by a row plane is the tetrahedron / wedge of Sec. III-C.  The weight of
// detector element (k, r) is the difference of H between its two row planes
// (the vol_res differencing of Sec. III-C).  Summing the pieces in depth order
// from the far end, with moments taken about each breakpoint, keeps every term
// non-negative, so nothing cancels near phi = k pi / 2 where the closed forms
// of the paper divide by sin(phi) or by vanishing depth gaps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smk {

// ---------------------------------------------------------------------------
// device geometry (plain values; passed to kernels by value)
// ---------------------------------------------------------------------------
struct DevGeom {
    int dim, nx, ny, nz, n_p, nu, nv;
    int pad;
    double a, b, c;
    double x0, y0, z0;
    double s, D;            // source-origin, source-detector distance
    double du, dv, u0, v0;  // detector pitch and first corner (u: columns, v: rows)
    const double2 *trig;    // n_p (cos, sin)
    const double *tau;      // nv + 1 row-plane slopes v_r / D
};

constexpr int MAXB = 8;  // breakpoints of a strip polygon (<= 6 in exact arithmetic)

// Strip record: pixel (ix, iy) cut by detector column k in one view.
// tab[0] lists the breakpoints in ascending l', tab[1] in ascending -l'
// (the mirror image used by row planes with tau < 0).  Each entry is
// (depth, chord width, S0, S1) with S0 = integral of w beyond the depth and
// S1 = first moment of w beyond the depth about the depth itself.
template <typename T>
struct alignas(16) Rec {
    double lc;          // depth of the column centre
    double lmin, lmax;  // absolute depth range of the polygon
    double ilmin, ilmax;  // their reciprocals
    T area;             // polygon area
    int n;              // number of breakpoints, 0 when the polygon is empty
    int k;              // detector column
    int pix;            // pixel index iy * nx + ix (or a kernel-local index)
    T tab[2][MAXB][4];
};

__device__ __forceinline__ double2 view_trig(const DevGeom &G, int view) { return G.trig[view]; }

// ---------------------------------------------------------------------------
// strip polygon: pixel rectangle cut by the wedge u_k <= u <= u_{k+1}
// ---------------------------------------------------------------------------
// Builds the record in FP64 (the plane/face intersections and every sign
// decision), then stores the tables in T.
template <typename T>
__host__ __device__ void build_record(const DevGeom &G, double cp, double sp, int ix, int iy, int k,
                             Rec<T> &R)
{
    const double xc = G.x0 + ((double)ix + 0.5) * G.a;
    const double yc = G.y0 + ((double)iy + 0.5) * G.b;
    const double lc = G.s - (xc * cp + yc * sp);
    const double tc = yc * cp - xc * sp;
    const double ha = 0.5 * G.a, hb = 0.5 * G.b;

    // pixel corners in cyclic order, local (depth, lateral)
    double cd[4], ct[4];
    {
        const double qx[4] = {-ha, ha, ha, -ha};
        const double qy[4] = {-hb, -hb, hb, hb};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            cd[j] = -(qx[j] * cp + qy[j] * sp);
            ct[j] = qy[j] * cp - qx[j] * sp;
        }
    }
    // column planes: t' - mu l' + eps = 0 with mu = u / D, eps = tc - mu lc
    const double mu0 = (G.u0 + (double)k * G.du) / G.D;
    const double mu1 = (G.u0 + (double)(k + 1) * G.du) / G.D;
    const double ep0 = tc - mu0 * lc, ep1 = tc - mu1 * lc;
    double g0[4], g1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        g0[j] = ct[j] - mu0 * cd[j] + ep0;  // >= 0: u >= u_k
        g1[j] = ct[j] - mu1 * cd[j] + ep1;  // <= 0: u <= u_{k+1}
    }

    // polygon vertices (cyclic): kept corners and crossings in edge order
    double vd[MAXB], vt[MAXB];
    int m = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int jn = (j + 1) & 3;
        if (g0[j] >= 0.0 && g1[j] <= 0.0 && m < MAXB) {
            vd[m] = cd[j];
            vt[m] = ct[j];
            ++m;
        }
        double s0 = -1.0, s1 = -1.0;
        if ((g0[j] > 0.0 && g0[jn] < 0.0) || (g0[j] < 0.0 && g0[jn] > 0.0)) s0 = g0[j] / (g0[j] - g0[jn]);
        if ((g1[j] > 0.0 && g1[jn] < 0.0) || (g1[j] < 0.0 && g1[jn] > 0.0)) s1 = g1[j] / (g1[j] - g1[jn]);
        double sa = s0, sb = s1;
        if (sa > sb) {
            double tmp = sa;
            sa = sb;
            sb = tmp;
        }
        if (sa >= 0.0 && m < MAXB) {
            vd[m] = cd[j] + sa * (cd[jn] - cd[j]);
            vt[m] = ct[j] + sa * (ct[jn] - ct[j]);
            ++m;
        }
        if (sb >= 0.0 && m < MAXB) {
            vd[m] = cd[j] + sb * (cd[jn] - cd[j]);
            vt[m] = ct[j] + sb * (ct[jn] - ct[j]);
            ++m;
        }
    }

    R.lc = lc;
    R.k = k;
    if (m < 3) {
        R.n = 0;
        R.area = T(0);
        R.lmin = lc;
        R.lmax = lc;
        R.ilmin = 1.0 / lc;
        R.ilmax = R.ilmin;
        return;
    }

    // breakpoints: vertex depths in ascending order (insertion sort, m <= 8)
    double bd[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) bd[i] = (i < m) ? vd[i] : 1e300;
#pragma unroll
    for (int i = 1; i < MAXB; ++i) {
#pragma unroll
        for (int j = i; j > 0; --j) {
            const double lo = bd[j - 1], hi = bd[j];
            const bool sw = lo > hi;
            bd[j - 1] = sw ? hi : lo;
            bd[j] = sw ? lo : hi;
        }
    }

    // chord width at each breakpoint: extent in t' of the polygon's
    // intersection with the line l' = depth; an edge of zero depth extent
    // contributes both end points (the inner limit at an extreme depth).
    double bw[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        double tmin = 1e300, tmax = -1e300;
        const double dq = bd[i];
        for (int e = 0; e < m; ++e) {
            const int en = (e + 1 == m) ? 0 : e + 1;
            double da = vd[e], db = vd[en], ta = vt[e], tb = vt[en];
            if (da > db) {
                double t1 = da; da = db; db = t1;
                t1 = ta; ta = tb; tb = t1;
            }
            if (dq < da || dq > db) continue;
            if (db == da) {
                tmin = fmin(tmin, fmin(ta, tb));
                tmax = fmax(tmax, fmax(ta, tb));
            } else {
                const double tq = ta + (tb - ta) * ((dq - da) / (db - da));
                tmin = fmin(tmin, tq);
                tmax = fmax(tmax, tq);
            }
        }
        bw[i] = (i < m && tmax >= tmin) ? (tmax - tmin) : 0.0;
    }

    // suffix moments (ascending table) and prefix moments (mirrored table);
    // each slab between breakpoints is a prismatoid: integral of w is
    // L (w_i + w_i+1) / 2, the moment about the near end L^2 (w_near/3 + w_far/6)
    double S0[MAXB], S1[MAXB], P0[MAXB], P1[MAXB];
    S0[m - 1] = 0.0;
    S1[m - 1] = 0.0;
    for (int i = m - 2; i >= 0; --i) {
        const double L = bd[i + 1] - bd[i];
        S0[i] = S0[i + 1] + 0.5 * L * (bw[i] + bw[i + 1]);
        S1[i] = S1[i + 1] + L * S0[i + 1] + L * L * (bw[i] * (1.0 / 6.0) + bw[i + 1] * (1.0 / 3.0));
    }
    P0[0] = 0.0;
    P1[0] = 0.0;
    for (int i = 1; i < m; ++i) {
        const double L = bd[i] - bd[i - 1];
        P0[i] = P0[i - 1] + 0.5 * L * (bw[i - 1] + bw[i]);
        P1[i] = P1[i - 1] + L * P0[i - 1] + L * L * (bw[i] * (1.0 / 6.0) + bw[i - 1] * (1.0 / 3.0));
    }
    const double area = S0[0];
    R.n = (area > 0.0) ? m : 0;
    R.area = T(area);
    R.lmin = lc + bd[0];
    R.lmax = lc + bd[m - 1];
    R.ilmin = 1.0 / R.lmin;
    R.ilmax = 1.0 / R.lmax;
    for (int i = 0; i < m; ++i) {
        R.tab[0][i][0] = T(bd[i]);
        R.tab[0][i][1] = T(bw[i]);
        R.tab[0][i][2] = T(S0[i]);
        R.tab[0][i][3] = T(S1[i]);
        const int j = m - 1 - i;
        R.tab[1][j][0] = T(-bd[i]);
        R.tab[1][j][1] = T(bw[i]);
        R.tab[1][j][2] = T(P0[i]);
        R.tab[1][j][3] = T(P1[i]);
    }
}

// ---------------------------------------------------------------------------
// cumulative sub-volume below a row plane
// ---------------------------------------------------------------------------
// Psi(lambda) = integral over P of (l'' - lambda)_+ dA for lambda inside the
// table's depth range (l'' = l' for table 0, -l' for table 1).
template <typename T>
__host__ __device__ inline T psi_inside(const T (*tab)[4], int n, T lam)
{
    int i = 0;
    for (int j = 1; j < n - 1; ++j) i += (lam >= tab[j][0]) ? 1 : 0;
    const T d0 = tab[i][0], w0 = tab[i][1];
    const T d1 = tab[i + 1][0], w1 = tab[i + 1][1], s0 = tab[i + 1][2], s1 = tab[i + 1][3];
    const T L = d1 - d0;
    T h = d1 - lam;
    h = h < T(0) ? T(0) : (h > L ? L : h);
    const T wl = w1 + (w0 - w1) * (L > T(0) ? h / L : T(0));
    return h * h * (wl * T(1.0 / 6.0) + w1 * T(1.0 / 3.0)) + s1 + h * s0;
}

// Volume of (polygon x [za, za + c]) below the plane z = tau l, given
// e = tau lc - za (plane height above the voxel bottom at the column centre),
// at = |tau|, inv_at = 1 / at (unused when at == 0) and sg = (tau < 0).
template <typename T>
__host__ __device__ inline T eval_H(const Rec<T> &R, int sg, T at, T inv_at, T e, T c)
{
    const T (*tab)[4] = R.tab[sg];
    const int n = R.n;
    const T d0 = tab[0][0], dn = tab[n - 1][0];
    const T A = R.area;
    const T lo = e + at * d0, hi = e + at * dn;
    if (hi <= T(0)) return T(0);
    if (lo >= c) return c * A;
    const T p0 = (lo >= T(0)) ? (lo * A + at * tab[0][3]) : at * psi_inside(tab, n, -e * inv_at);
    const T p1 = (hi <= c) ? T(0) : at * psi_inside(tab, n, (c - e) * inv_at);
    return p0 - p1;
}

// ---------------------------------------------------------------------------
// 2D: area of the pixel on the u <= u* side (the paper's sweep of Sec. III-B)
// ---------------------------------------------------------------------------
// The boundary ray of detector coordinate u* is t' - mu l' + eps = 0 in local
// coordinates, i.e. g(q) = alpha qx + beta qy + eps with alpha = mu cp - sp,
// beta = cp + mu sp.  With p = |alpha| a and q = |beta| b the corner values of
// g are eps -/+ (p + q)/2 and eps -/+ |p - q|/2 (the sorted Gamma_1..4).  The
// area below g = 0 is a corner triangle (the atom A_3), a triangle plus a
// trapezoid (A_4), or the pixel minus a corner triangle, written in ratios
// that stay bounded when alpha or beta vanish.
template <typename T>
__host__ __device__ inline T sweep_area(double cp, double sp, double lc, double tc, double mu,
                                        T a, T b)
{
    const double alpha = mu * cp - sp, beta = cp + mu * sp;
    const double eps = tc - mu * lc;
    const T e = T(eps);
    const T p = T(fabs(alpha)) * a, q = T(fabs(beta)) * b;
    const T hs = T(0.5) * (p + q);
    const T mn = p < q ? p : q, mx = p < q ? q : p;
    const T ab = a * b;
    const T g1 = e - hs, g4 = e + hs;
    if (g1 >= T(0)) return T(0);
    if (g4 <= T(0)) return ab;
    if (-g1 <= mn) return T(0.5) * ab * ((-g1) / p) * ((-g1) / q);
    if (g4 <= mn) return ab - T(0.5) * ab * (g4 / p) * (g4 / q);
    return ab * (T(0.5) - e / mx);
}

// ---------------------------------------------------------------------------
// strip enumeration: which pixels can meet the wedge u_lo <= u <= u_hi
// ---------------------------------------------------------------------------
// Major axis x when |cp| >= |sp| (rays run mostly along x), else y.  For one
// major cell the wedge covers an interval of the minor axis bounded by the two
// boundary rays evaluated at both ends of the cell.
struct StripAxis {
    bool major_x;
    int n_major, n_minor;
};

__host__ __device__ inline StripAxis strip_axis(const DevGeom &G, double cp, double sp)
{
    StripAxis A;
    A.major_x = fabs(cp) >= fabs(sp);
    A.n_major = A.major_x ? G.nx : G.ny;
    A.n_minor = A.major_x ? G.ny : G.nx;
    return A;
}

// Minor-index range [j0, j1] of major cell i (empty when j0 > j1).
__host__ __device__ inline void strip_minor_range(const DevGeom &G, const StripAxis &A, double cp,
                                                  double sp, double ulo, double uhi, int i,
                                                  int &j0, int &j1)
{
    double lo = 1e300, hi = -1e300;
    if (A.major_x) {
        const double xa = G.x0 + (double)i * G.a, xb = xa + G.a;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double us = q ? uhi : ulo;
            const double den = G.D * cp + us * sp;
            const double ya = (us * G.s + xa * (G.D * sp - us * cp)) / den;
            const double yb = (us * G.s + xb * (G.D * sp - us * cp)) / den;
            lo = fmin(lo, fmin(ya, yb));
            hi = fmax(hi, fmax(ya, yb));
        }
        const double pad = 1e-9 * G.b;
        double f0 = floor((lo - pad - G.y0) / G.b), f1 = floor((hi + pad - G.y0) / G.b);
        if (!(f0 == f0) || !(f1 == f1)) { f0 = 0; f1 = A.n_minor - 1; }
        j0 = (int)fmin(fmax(f0, 0.0), (double)A.n_minor);
        j1 = (int)fmax(fmin(f1, (double)(A.n_minor - 1)), -1.0);
    } else {
        const double ya = G.y0 + (double)i * G.b, yb = ya + G.b;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double us = q ? uhi : ulo;
            const double den = us * cp - G.D * sp;
            const double xa = (us * (G.s - ya * sp) - G.D * ya * cp) / den;
            const double xb = (us * (G.s - yb * sp) - G.D * yb * cp) / den;
            lo = fmin(lo, fmin(xa, xb));
            hi = fmax(hi, fmax(xa, xb));
        }
        const double pad = 1e-9 * G.a;
        double f0 = floor((lo - pad - G.x0) / G.a), f1 = floor((hi + pad - G.x0) / G.a);
        if (!(f0 == f0) || !(f1 == f1)) { f0 = 0; f1 = A.n_minor - 1; }
        j0 = (int)fmin(fmax(f0, 0.0), (double)A.n_minor);
        j1 = (int)fmax(fmin(f1, (double)(A.n_minor - 1)), -1.0);
    }
}

// Detector-column range that the rectangle spanned by pixel corners
// [ixa, ixb] x [iya, iyb] can meet in a view: a superset of the footprint of
// every pixel inside it (cells outside have zero weight).  The same corner
// arithmetic serves single pixels and whole tiles, so a tile's range bounds
// the ranges of its pixels exactly.
__host__ __device__ inline void corner_columns(const DevGeom &G, double cp, double sp, int ixa,
                                               int ixb, int iya, int iyb, int &k0, int &k1)
{
    double umin = 1e300, umax = -1e300;
    for (int q = 0; q < 4; ++q) {
        const double x = G.x0 + (double)((q & 1) ? ixb : ixa) * G.a;
        const double y = G.y0 + (double)((q >> 1) ? iyb : iya) * G.b;
        const double l = G.s - (x * cp + y * sp);
        const double t = y * cp - x * sp;
        const double u = G.D * t / l;
        umin = fmin(umin, u);
        umax = fmax(umax, u);
    }
    const double pad = 1e-9 * G.du;
    const double f0 = floor((umin - pad - G.u0) / G.du), f1 = floor((umax + pad - G.u0) / G.du);
    k0 = (int)fmin(fmax(f0, 0.0), (double)G.nu);
    k1 = (int)fmax(fmin(f1, (double)(G.nu - 1)), -1.0);
}

__device__ __forceinline__ void pixel_columns(const DevGeom &G, double cp, double sp, int ix,
                                              int iy, int &k0, int &k1)
{
    corner_columns(G, cp, sp, ix, ix + 1, iy, iy + 1, k0, k1);
}

// XCD-aware block order: consecutive logical blocks land on the same XCD so
// that neighbouring work shares that XCD's L2 (workgroups are dispatched
// round-robin over the 8 XCDs).
__device__ __forceinline__ int xcd_remap(int b, int nblocks)
{
    const int nx = 8;
    const int per = (nblocks + nx - 1) / nx;
    const int xcd = b % nx, slot = b / nx;
    const int full = nblocks % nx == 0 ? nx : nblocks % nx;  // XCDs holding `per` blocks
    // XCDs [0, full) own `per` logical blocks, the rest own per - 1
    int base = xcd < full ? xcd * per : full * per + (xcd - full) * (per - 1);
    return base + slot;
}

}  // namespace smk
