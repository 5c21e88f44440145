// sm_common.h -- geometry and weight evaluation shared by the record,
// forward, adjoint and CSR kernels (device and host).
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
// trapezoids of Sec. III-B).  The row planes depend on (x, y) only through l,
// so the volume of the column P x [z, inf) lying below plane r is
//     K(z) = integral over P of (e + tau l')_+ dA,   e = tau lc - z,
// a one-dimensional integral of the chord length w(l') of P against a
// truncated linear height.  w is piecewise linear with kinks at the vertex
// depths of P; between consecutive vertex depths each piece is a prismatoid
// whose volume the prismatoid rule gives exactly (appendix, "Prismatoid"), and
// the piece cut by the plane is the tetrahedron / wedge of Sec. III-C.  The
// volume of voxel [za, zb] below the plane is K(za) - K(zb), and the weight of
// detector element (k, r) is the difference of that between its two row
// planes (the vol_res differencing of Sec. III-C).  Summing pieces from the
// far end with moments about each breakpoint keeps every term non-negative,
// so nothing cancels near phi = k pi / 2, where the paper's closed forms
// divide by sin(phi) or by vanishing depth gaps.
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

constexpr int MAXV = 6;  // vertices of a strip polygon (rectangle cut by two lines)

// Strip record: pixel `pix` cut by detector column k in one view.  Depths
// l' are measured from lc, the depth of the strip polygon's centroid (its
// area-weighted mean depth), so that the first moment of the chord width
// about the origin vanishes.  tab[i] = (depth l', half the chord width w / 2,
// S0, S1) for the breakpoints in ascending depth, S0 = integral of w beyond
// the depth, S1 = first moment of w beyond the depth about the depth itself.
// Area A = tab[0][2].  The header also holds the row-plane index scales D / (L dv) at
// the nearest and farthest depth L (see plane_split), the same two depths in
// voxel heights (see plane_faces), c A and A lc dv / D (the step of the linear
// volume A (tau lc - z) from one row plane to the next), all computed in FP64.
// 144 bytes for T = float, 256 for T = double.
template <typename T>
struct alignas(16) Rec {
    double lc;  // depth of the centroid
    int n;      // number of breakpoints, 0 when the polygon is empty
    int pix;    // pixel index iy * nx + ix
    T kLo, kHi; // D / (Llo dv), D / (Lhi dv)
    T hLo, hHi; // Llo / c, Lhi / c
    T cA;       // c A
    T bA;       // A lc dv / D
    alignas(16) T tab[MAXV][4];
};

// A strip record as the adjoint stages it in LDS (sm_back3d.hip): the fields
// its terms read, and in place of the breakpoint table's first row (whose
// depth and area are kept as d0 and A) the cubic coefficient g6[i] of Psi on
// segment i, taken once from the table (see K_cut) instead of in every
// straddle term.  seg[i] is table row i + 1, the far end of segment i; seg[4]
// holds the farthest depth (later rows repeat the last breakpoint).  The
// row-plane index scales are held in both orders, k4 = (kLo, kHi, kHi, kLo),
// so that a lane reads the pair plane_split needs at a face of its sign
// (k4 + 2 at z >= 0, k4 below) instead of selecting.  160 bytes in FP32,
// 288 in FP64.
template <typename T>
struct alignas(16) AdjRec {
    double lc;
    int n;
    int unused_;
    T k4[4];
    T cA, bA, d0, A;
    T g6[MAXV - 1];
    alignas(16) T seg[MAXV - 1][4];
};

// Stride of a strip record staged in LDS.  Lanes that gather different
// records read the same field offset; a stride of a whole number of 128-byte
// lines would put that field of every record in the same LDS bank, so such
// records get 16 bytes of padding.
template <typename T>
constexpr size_t lds_rec_stride()
{
    return sizeof(Rec<T>) % 128 == 0 ? sizeof(Rec<T>) + 16 : sizeof(Rec<T>);
}

template <typename T>
__device__ __forceinline__ const Rec<T> &lds_rec(const unsigned char *base, int i)
{
    return *reinterpret_cast<const Rec<T> *>(base + (size_t)i * lds_rec_stride<T>());
}

// one v_min_f64 / v_max_f64 each (the inputs are finite)
__host__ __device__ inline double dmin_(double a, double b) { return fmin(a, b); }
__host__ __device__ inline double dmax_(double a, double b) { return fmax(a, b); }

// a / b in FP64 for the strip polygons: the hardware reciprocal estimate
// refined by two Newton steps (each squares its relative error), then one
// product: within a unit or two in the last place of the quotient, in five
// instructions instead of the eleven of a correctly rounded division.  b is
// finite and nonzero at every call.
__host__ __device__ inline double qdiv_(double a, double b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(b);
    r = fma(fma(-b, r, 1.0), r, r);
    r = fma(fma(-b, r, 1.0), r, r);
    return a * r;
#else
    return a / b;
#endif
}

// ---------------------------------------------------------------------------
// strip polygon: pixel rectangle cut by the wedge u_k <= u <= u_{k+1}
// ---------------------------------------------------------------------------
// FP64 throughout (the plane/face intersections and every sign decision);
// the tables are stored in T.  `ws` is scratch for up to 8 vertices: a
// pointer, or a strided view (LdsVerts) into a workgroup's shared array.
struct LdsVerts {
    double2 *p;  // vertex 0 of this thread
    int stride;  // elements between consecutive vertices
    __host__ __device__ double2 &operator[](int i) const { return p[i * stride]; }
};

template <typename T, typename RecT, typename WS>
__host__ __device__ inline void build_record(const DevGeom &G, double cp, double sp, int ix, int iy,
                                             int k, RecT &R, WS ws)
{
    const double xc = G.x0 + ((double)ix + 0.5) * G.a;
    const double yc = G.y0 + ((double)iy + 0.5) * G.b;
    const double lc = G.s - (xc * cp + yc * sp);
    const double tc = yc * cp - xc * sp;
    const double ha = 0.5 * G.a, hb = 0.5 * G.b;

    // column planes: t' - mu l' + eps = 0 with mu = u / D, eps = tc - mu lc
    const double mu0 = qdiv_(G.u0 + (double)k * G.du, G.D);
    const double mu1 = qdiv_(G.u0 + (double)(k + 1) * G.du, G.D);
    const double ep0 = tc - mu0 * lc, ep1 = tc - mu1 * lc;
    // pixel corner j in cyclic order, local (depth, lateral), and its signed
    // distances to the two column planes (>= 0: u >= u_k; <= 0: u <= u_k+1)
    auto corner = [&](int j, double &cd, double &ct, double &g0, double &g1) {
        const double qx = (j == 1 || j == 2) ? ha : -ha;
        const double qy = j >= 2 ? hb : -hb;
        cd = -(qx * cp + qy * sp);
        ct = qy * cp - qx * sp;
        g0 = ct - mu0 * cd + ep0;
        g1 = ct - mu1 * cd + ep1;
    };
    // polygon vertices in cyclic order: kept corners and crossings in edge
    // order (one edge at a time, so that few values stay live)
    int m = 0;
#pragma unroll 1
    for (int j = 0; j < 4; ++j) {
        double cdj, ctj, g0j, g1j, cdn, ctn, g0n, g1n;
        corner(j, cdj, ctj, g0j, g1j);
        corner((j + 1) & 3, cdn, ctn, g0n, g1n);
        if (g0j >= 0.0 && g1j <= 0.0) {
            if (m < 8) ws[m] = make_double2(cdj, ctj);
            ++m;
        }
        double s0 = -1.0, s1 = -1.0;
        if ((g0j > 0.0 && g0n < 0.0) || (g0j < 0.0 && g0n > 0.0)) s0 = qdiv_(g0j, g0j - g0n);
        if ((g1j > 0.0 && g1n < 0.0) || (g1j < 0.0 && g1n > 0.0)) s1 = qdiv_(g1j, g1j - g1n);
        const double sa = dmin_(s0, s1), sb = dmax_(s0, s1);
        if (sa >= 0.0) {
            if (m < 8) ws[m] = make_double2(cdj + sa * (cdn - cdj), ctj + sa * (ctn - ctj));
            ++m;
        }
        if (sb >= 0.0) {
            if (m < 8) ws[m] = make_double2(cdj + sb * (cdn - cdj), ctj + sb * (ctn - ctj));
            ++m;
        }
    }
    if (m > 8) m = 8;
    // drop vertices that repeat their predecessor (rounding residue of a cut
    // through a corner); a convex cut of a rectangle by two lines keeps <= 6
    {
        const double tol = 1e-12 * (G.a + G.b);
        int w = 0;
        for (int i = 0; i < m; ++i) {
            const double2 v = ws[i];
            if (w > 0) {
                const double2 p = ws[w - 1];
                if (fabs(v.x - p.x) <= tol && fabs(v.y - p.y) <= tol) continue;
            }
            ws[w++] = v;
        }
        while (w > 1 && fabs(ws[w - 1].x - ws[0].x) <= tol && fabs(ws[w - 1].y - ws[0].y) <= tol) --w;
        m = w > MAXV ? MAXV : w;
    }

    R.lc = lc;
    R.kLo = T(0);
    R.kHi = T(0);
    R.hLo = T(0);
    R.hHi = T(0);
    R.cA = T(0);
    R.bA = T(0);
    if (m < 3) {
        R.n = 0;
        return;
    }

    // breakpoints: vertex depths in ascending order
    double bd[MAXV];
#pragma unroll
    for (int i = 0; i < MAXV; ++i) bd[i] = (i < m) ? ws[i].x : 1e300;
#pragma unroll
    for (int i = 1; i < MAXV; ++i) {
#pragma unroll
        for (int j = i; j > 0; --j) {
            const double lo = bd[j - 1], hi = bd[j];
            bd[j - 1] = dmin_(lo, hi);
            bd[j] = dmax_(lo, hi);
        }
    }
    // the farthest breakpoint (static indices only: no scratch)
    double dlast = bd[0];
#pragma unroll
    for (int i = 1; i < MAXV; ++i)
        if (i < m) dlast = bd[i];
    // chord width at each breakpoint: extent in t' of the polygon's section at
    // that depth; an edge of zero depth extent contributes both end points
    // (the inner limit at an extreme depth).  One edge at a time, updating
    // the extremes of every breakpoint, so that few values stay live.
    double tmn[MAXV], tmx[MAXV];
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
        tmn[i] = 1e300;
        tmx[i] = -1e300;
    }
#pragma unroll 1
    for (int e = 0; e < m; ++e) {
        const double2 p = ws[e];
        const double2 q = ws[e + 1 < m ? e + 1 : 0];
        const bool sw = p.x > q.x;
        const double ea = sw ? q.x : p.x, eb = sw ? p.x : q.x;
        const double ta = sw ? q.y : p.y, tb = sw ? p.y : q.y;
        const bool flat = eb == ea;
        const double sl = flat ? 0.0 : qdiv_(tb - ta, eb - ea);
#pragma unroll
        for (int i = 0; i < MAXV; ++i) {
            const double dq = bd[i];
            if (dq >= ea && dq <= eb) {
                if (flat) {
                    tmn[i] = dmin_(tmn[i], dmin_(ta, tb));
                    tmx[i] = dmax_(tmx[i], dmax_(ta, tb));
                } else {
                    const double tq = ta + sl * (dq - ea);
                    tmn[i] = dmin_(tmn[i], tq);
                    tmx[i] = dmax_(tmx[i], tq);
                }
            }
        }
    }
    double bw[MAXV];
#pragma unroll
    for (int i = 0; i < MAXV; ++i) bw[i] = (i < m && tmx[i] >= tmn[i]) ? (tmx[i] - tmn[i]) : 0.0;
    // suffix moments: each slab between breakpoints is a prismatoid; its
    // integral of w is L (w_i + w_i+1) / 2 and its moment about the near end
    // L^2 (w_i / 6 + w_i+1 / 3)
    double S0[MAXV], S1[MAXV];
#pragma unroll
    for (int i = 0; i < MAXV; ++i) S0[i] = S1[i] = 0.0;
#pragma unroll
    for (int i = MAXV - 2; i >= 0; --i) {
        if (i < m - 1) {
            const double L = bd[i + 1] - bd[i];
            S0[i] = S0[i + 1] + 0.5 * L * (bw[i] + bw[i + 1]);
            S1[i] = S1[i + 1] + L * S0[i + 1] + L * L * (bw[i] * (1.0 / 6.0) + bw[i + 1] * (1.0 / 3.0));
        }
    }
    R.n = S0[0] > 0.0 ? m : 0;
    double lbo = 0.0;  // centroid depth relative to the pixel centre
    if (S0[0] > 0.0) {
        const double Ddv = G.D / G.dv;
        lbo = bd[0] + qdiv_(S1[0], S0[0]);
        R.lc = lc + lbo;
        R.kLo = T(qdiv_(Ddv, lc + bd[0]));
        R.kHi = T(qdiv_(Ddv, lc + dlast));
        const double rc = qdiv_(1.0, G.c);  // the same for every record: hoisted
        R.hLo = T((lc + bd[0]) * rc);
        R.hHi = T((lc + dlast) * rc);
        R.cA = T(G.c * S0[0]);
        R.bA = T(S0[0] * qdiv_(G.dv, G.D) * R.lc);
    }
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
        R.tab[i][0] = T((i < m ? bd[i] : dlast) - lbo);
        R.tab[i][1] = T(0.5 * bw[i]);  // half the chord width (see K_cut)
        R.tab[i][2] = T(S0[i]);
        R.tab[i][3] = T(S1[i]);
    }
}

// ---------------------------------------------------------------------------
// cumulative volume above a face and below a row plane
// ---------------------------------------------------------------------------
__host__ __device__ inline float rcp_(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
// FP64: the hardware estimate refined by two Newton steps (each squares the
// relative error), instead of a correctly rounded division
__host__ __device__ inline double rcp_(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    return fma(fma(-x, r, 1.0), r, r);
#else
    return 1.0 / x;
#endif
}

// Psi(lam) = integral over P of (l' - lam)_+ dA for lam inside [d_0, d_n-1].
template <typename T>
__host__ __device__ inline T psi_inside(const T (*tab)[4], int n, T lam)
{
    T d0 = tab[0][0], w0 = tab[0][1], d1 = tab[1][0], w1 = tab[1][1], s0 = tab[1][2],
      s1 = tab[1][3];
#pragma unroll
    for (int j = 1; j < MAXV - 1; ++j) {
        if (j < n - 1 && lam >= tab[j][0]) {
            d0 = tab[j][0];
            w0 = tab[j][1];
            d1 = tab[j + 1][0];
            w1 = tab[j + 1][1];
            s0 = tab[j + 1][2];
            s1 = tab[j + 1][3];
        }
    }
    const T L = d1 - d0;
    T h = d1 - lam;
    h = h < T(0) ? T(0) : (h > L ? L : h);
    const T wl = w1 + (w0 - w1) * (L > T(0) ? h * rcp_(L) : T(0));  // half widths
    return h * h * (wl * T(1.0 / 3.0) + w1 * T(2.0 / 3.0)) + s1 + h * s0;
}

// K = integral over P of (e + tau l')_+ dA: the volume of the column above a
// face and below the plane z = tau l, with e = tau lc - z_face the plane's
// height above the face at the column centre.  inv_tau = 1 / tau (any value
// when tau == 0).
template <typename T>
__host__ __device__ inline T eval_K(const T (*tab)[4], int n, T tau, T inv_tau, T e)
{
    const T d0 = tab[0][0], dn = tab[n - 1][0], A = tab[0][2], S1 = tab[0][3];
    const T h0 = e + tau * d0, h1 = e + tau * dn;  // heights at the near and far ends
    const T hmax = h0 > h1 ? h0 : h1, hmin = h0 > h1 ? h1 : h0;
    if (hmax <= T(0)) return T(0);
    if (hmin >= T(0)) return h0 * A + tau * S1;  // e A + tau * (first moment)
    const T lam = -e * inv_tau;                  // depth where the plane meets the face
    const T psi = psi_inside(tab, n, lam);
    if (tau > T(0)) return tau * psi;
    // tau < 0: integral of (lam - l')_+ = Psi - S1 + (lam - d0) A
    return (-tau) * (psi - S1 + (lam - d0) * A);
}

// ---------------------------------------------------------------------------
// classification of row planes against faces for one strip record
// ---------------------------------------------------------------------------
// Over the strip, plane z = tau l spans heights [lo, hi] with
// lo = tau Llo, hi = tau Lhi for tau >= 0 (swapped for tau < 0), Llo / Lhi
// being the nearest / farthest (absolute) depth of the strip polygon.
// Against a face at height z a plane is wholly below (K = 0), wholly above
// (K = the linear integral A (tau lc - z), lc the centroid depth of the
// strip) or straddles it (K from the chord table).  Both walks below only need the split to be
// consistent: K_cut is exact for a sloped plane anywhere, and a plane put on
// the wrong side of a face by rounding is off by a volume of rounding size.
// A horizontal plane (tau = 0) spans the single height 0, so both splits put
// it wholly on one side of every face (a face at height exactly 0 counts as
// both, with K = 0 either way); only rounding of a face that should sit at
// 0 can make it straddle, where its K is of rounding size.

// Clamp to [0, top]: one median instruction in FP32 on the device, a min and
// a max in FP64 (these run once or twice per record and lane).
__host__ __device__ inline float clamp0(float v, float top)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_fmed3f(v, 0.0f, top);
#else
    return v < 0.0f ? 0.0f : (v > top ? top : v);
#endif
}
__host__ __device__ inline double clamp0(double v, double top) { return fmin(fmax(v, 0.0), top); }

// floor(v) + 1 clamped to [0, top] (top an integer), as an int.  FP32 on the
// device: clamp to [-1, top - 1] first (same result, and the conversion stays
// in range), then one floor-and-convert instruction, which the compiler does
// not form from floor and a conversion; three instructions instead of four.
__host__ __device__ inline int floor1_clamp(float v, float top)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const float c = __builtin_amdgcn_fmed3f(v, -1.0f, top - 1.0f);
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(c));
    return r + 1;
#else
    const float a = floorf(v) + 1.0f;
    return (int)(a < 0.0f ? 0.0f : (a > top ? top : a));
#endif
}
__host__ __device__ inline int floor1_clamp(double v, double top) { return (int)clamp0(floor(v) + 1.0, top); }

// Row planes: indices < ph lie wholly below z, indices >= pa wholly above.
// tau_q = (v0 + q dv) / D, kLo = D / (Llo dv), kHi = D / (Lhi dv); k is the
// pair (kHi, kLo) for z >= 0 and (kLo, kHi) for z < 0 (plane q's highest
// point over the strip is at the far depth when tau_q >= 0).
template <typename T>
__host__ __device__ inline void plane_split(T z, const T *k, T v0dv, int nv, int &ph, int &pa)
{
    const T xh = z * k[0] - v0dv;  // hi(q) = z at this index
    const T xl = z * k[1] - v0dv;  // lo(q) = z at this index
    const T top = T(nv + 1);
    ph = floor1_clamp(xh, top);
    pa = (int)clamp0(T(ceil(xl)), top);
}

// Voxel faces z_j = z0 + j c against plane tau over the strip, whose nearest
// and farthest depths in voxel heights are hLo = Llo / c and hHi = Lhi / c
// (z0c = z0 / c): faces < fa lie wholly below the plane, faces >= fb wholly
// above it.  The plane's heights over the strip in voxel heights are tau hLo
// and tau hHi, so each end of the range takes one multiply-add; their order
// follows the sign of tau, which a min and a max settle without a select
// (rounding is monotone, so they pick the same values a select would).
template <typename T>
__host__ __device__ inline void plane_faces(T tau, T hLo, T hHi, T z0c, int nz, int &fa, int &fb)
{
    const T top = T(nz + 1);
    const T e0 = fma(tau, hLo, -z0c), e1 = fma(tau, hHi, -z0c);
    fa = floor1_clamp(T(fmin(e0, e1)), top);
    fb = (int)clamp0(T(ceil(fmax(e0, e1))), top);
}

// The uniform part of a strip record used by K_cut; `tab` points at the
// chord table (an LDS copy in the kernels).
template <typename T>
struct StripTab {
    const T (*tab)[4];
    T d0, A, b1, b2, b3, b4;  // nearest depth, area, interior breakpoints
};

template <typename T>
__host__ __device__ inline StripTab<T> strip_tab(const T (*tab)[4], const T (*rows)[4])
{
    StripTab<T> S;
    S.tab = rows;
    S.d0 = tab[0][0];
    S.A = tab[0][2];
    S.b1 = tab[1][0];
    S.b2 = tab[2][0];
    S.b3 = tab[3][0];
    S.b4 = tab[4][0];
    return S;
}

// K = integral over P of (e + tau l')_+ dA for a sloped plane (see eval_K).
// The segment of the breakpoint table holding lam = -e / tau is found by
// counting breakpoints; Psi continues linearly below the nearest depth
// (Psi(lam) = S1 + (d0 - lam) A there) and is zero beyond the farthest, so
// the result is exact wherever the plane lies.  For tau > 0, K = tau Psi(lam).
// For tau < 0, writing (w)_+ = w + (-w)_+ gives the plane's linear volume
// e A + tau M1 plus (-tau) Psi(lam), M1 being the first moment of the chord
// width about the depth origin, which is zero at the centroid: both signs
// take |tau| Psi and the negative one adds e A.  A horizontal plane gets 0
// (it never straddles a face; see above).
template <typename T>
__host__ __device__ inline T K_cut(const StripTab<T> &S, T tau, T inv_tau, T e)
{
    const T lam = -e * inv_tau;
    // row offset in bytes: the breakpoints at or below lam, counted (the
    // compiler adds two of the comparisons as carries), times the row size
    constexpr int RB = 4 * (int)sizeof(T);
    const int jo = RB * ((int)(lam >= S.b1) + (int)(lam >= S.b2) + (int)(lam >= S.b3) + (int)(lam >= S.b4));
    const T *r0 = reinterpret_cast<const T *>(reinterpret_cast<const char *>(S.tab) + jo);
    const T *r1 = r0 + 4;
    const T dA = r0[0], w0 = r0[1];
    const T dB = r1[0], w1 = r1[1], s0 = r1[2], s1 = r1[3];
    const T L = dB - dA;
    T h = dB - lam;
    h = clamp0(h, L);  // L >= 0: breakpoints ascend
    // Psi = s1 + h s0 + h^2 w1 / 2 + h^3 g / 6 with g the chord width's slope
    // over the segment, in Horner form; the table holds half widths, so
    // w1 / 2 is read directly and g / 6 = (w0/2 - w1/2) / (3 L).  h <= L, so
    // a zero-length segment gives h = 0, and the guard keeps g finite there.
    const T g6 = (w0 - w1) * rcp_(L > T(1e-30) ? L : T(1e-30)) * T(1.0 / 3.0);
    T psi = fma(h, fma(h, fma(h, g6, w1), s0), s1);
    const T below = S.d0 - lam;
    psi += (below > T(0) ? below : T(0)) * S.A;
    const T kp = fabs(tau) * psi;
    return tau < T(0) ? kp + e * S.A : kp;
}

// The adjoint's view of an AdjRec (uniform per record) and K_cut on it.
template <typename T>
struct AdjTab {
    const T (*seg)[4];
    const T *g6;
    T d0, dn, A, b1, b2, b3, b4;  // nearest and farthest depth, area, interior breakpoints
};

template <typename T>
__host__ __device__ inline AdjTab<T> adj_tab(const AdjRec<T> &R)
{
    AdjTab<T> S;
    S.seg = R.seg;
    S.g6 = R.g6;
    S.d0 = R.d0;
    S.dn = R.seg[MAXV - 2][0];
    S.A = R.A;
    S.b1 = R.seg[0][0];
    S.b2 = R.seg[1][0];
    S.b3 = R.seg[2][0];
    S.b4 = R.seg[3][0];
    return S;
}

// Clamp to [lo, hi] (lo <= hi): one median instruction in FP32 on the device.
__host__ __device__ inline float clamp_(float v, float lo, float hi)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_fmed3f(v, lo, hi);
#else
    return v < lo ? lo : (v > hi ? hi : v);
#endif
}
__host__ __device__ inline double clamp_(double v, double lo, double hi) { return fmin(fmax(v, lo), hi); }

// K_cut with the segment coefficients staged: the segment j holding lam as
// in K_cut, then h = dB - lam with lam clamped to [d0, dn] first, which puts
// h in [0, L] as K_cut's clamp does (below the nearest depth the first
// segment is taken whole; beyond the farthest h = 0).
template <typename T>
__host__ __device__ inline T K_cut(const AdjTab<T> &S, T tau, T inv_tau, T e)
{
    const T lam = -e * inv_tau;
    const int j = (int)(lam >= S.b1) + (int)(lam >= S.b2) + (int)(lam >= S.b3) + (int)(lam >= S.b4);
    const T *r = S.seg[j];
    const T dB = r[0], w1 = r[1], s0 = r[2], s1 = r[3];
    const T h = dB - clamp_(lam, S.d0, S.dn);
    T psi = fma(h, fma(h, fma(h, S.g6[j], w1), s0), s1);
    const T below = S.d0 - lam;
    psi += (below > T(0) ? below : T(0)) * S.A;
    const T kp = fabs(tau) * psi;
    return tau < T(0) ? kp + e * S.A : kp;
}

// The part of G_p of one plane for one strip record that needs no chord
// table: the linear volume at face f = fa - 1 (the first voxel not wholly
// below the plane).  Faces fa .. je are straddled (empty when je < fa); their
// terms come from straddle_term.  Xc[b] is the voxel column (x_0 .. x_{nz-1})
// of batch element b.
template <typename T, int NBAT>
__host__ __device__ inline void plane_lin(const DevGeom &G, const StripTab<T> &S, double lc,
                                          T hLo, T hHi, double tau, T tauf, T z0c,
                                          const T *const (&Xc)[NBAT], int &f_out, int &fa_out,
                                          int &je_out, T (&gs)[NBAT])
{
    const int nz = G.nz;
    int fa, fb;
    plane_faces<T>(tauf, hLo, hHi, z0c, nz, fa, fb);
    const int f = max(fa - 1, 0);  // fa <= nz + 1
    f_out = f;
    fa_out = fa;
    je_out = fb - 1 < nz ? fb - 1 : nz;
#pragma unroll
    for (int b = 0; b < NBAT; ++b) gs[b] = T(0);
    if (fa >= 1 && fa <= nz) {  // face f wholly below the plane: linear volume
        const T K = S.A * T(tau * lc - (G.z0 + (double)f * G.c));
#pragma unroll
        for (int b = 0; b < NBAT; ++b) gs[b] = K * Xc[b][f];  // f = fa - 1 < nz
    }
}

// Term K_p(z_j) (x_j - x_{j-1}) of a straddled face j (x_{-1} = x_nz = 0).
template <typename T, int NBAT>
__host__ __device__ inline void straddle_term(const DevGeom &G, const StripTab<T> &S, double lc,
                                              double tau, T tauf, T invt, int j,
                                              const T *const (&Xc)[NBAT], T (&out)[NBAT])
{
    const int nz = G.nz;
    const T K = K_cut<T>(S, tauf, invt, T(tau * lc - (G.z0 + (double)j * G.c)));
#pragma unroll
    for (int b = 0; b < NBAT; ++b) {
        const T xj = j < nz ? Xc[b][j] : T(0);
        const T xm = j >= 1 ? Xc[b][j - 1] : T(0);
        out[b] = K * (xj - xm);
    }
}

// G_p of one plane for one strip record; f_out = first voxel not wholly below.
template <typename T, int NBAT>
__host__ __device__ inline void plane_G(const DevGeom &G, const StripTab<T> &S, double lc,
                                        T hLo, T hHi, double tau, T tauf, T invt, T z0c,
                                        const T *const (&Xc)[NBAT], int &f_out, T (&gs)[NBAT])
{
    int fa, je;
    plane_lin<T, NBAT>(G, S, lc, hLo, hHi, tau, tauf, z0c, Xc, f_out, fa, je, gs);
    for (int j = fa; j <= je; ++j) {
        T t[NBAT];
        straddle_term<T, NBAT>(G, S, lc, tau, tauf, invt, j, Xc, t);
#pragma unroll
        for (int b = 0; b < NBAT; ++b) gs[b] += t[b];
    }
}

// Row plane q in the adjoint's LDS table: its slope in FP64 (for face
// heights), in T and the inverse in T (for K_cut), side by side so that one
// address and one wide read serve a straddle term (16 bytes in FP32; 24 in
// FP64, where LDS bounds the adjoint's occupancy).
template <typename T>
struct alignas(sizeof(T) == 4 ? 16 : 8) PlaneRow {
    double tau;
    T tf, inv;
};

// The part of one strip record's contribution to voxel [za, zb] of its column
// in the adjoint that needs no chord table: c A y[pab - 1] for the planes
// wholly above the voxel plus the linear volumes at za of the planes wholly
// above za that reach below zb.  Planes pha .. paa - 1 straddle za and
// phb .. pab - 1 straddle zb (adj_straddle gives their terms).
// Y[b * ystride + q] holds y[q] of batch element b for q in [-1, nv];
// pl holds the plane slopes; cA = c A and bA = A lc dv / D come with the
// record, ka and kb are the index-scale pairs for za and zb (see plane_split).
//
// The linear volumes are K_q = A (tau_q lc - za) = alpha + (q - a) bA for
// q = a .. e - 1 (a = paa, e = pab; the slopes tau_q are dv / D apart), with
// alpha = K_a.  Summed by parts,
//     sum_q K_q (y[q-1] - y[q]) = alpha (y[a-1] - y[e-1])
//                                 + bA sum_{q=a}^{e-2} (y[q] - y[e-1]),
// one FP64 product per record instead of one per plane.  A voxel holds one or
// two planes (the row pitch is close to the voxel's projected height), so the
// second sum is taken without a loop for e - a <= 2 and the loop runs only
// for the rare e - a > 2.  Every batch width takes the same steps, so that a
// volume's result does not depend on the batch it is applied in.
template <typename T, int NBAT>
__host__ __device__ inline void adj_lin(const AdjTab<T> &S, double lc, T cA, T bA, const T *ka, const T *kb,
                                        const PlaneRow<T> *pl, double za, double zb, T v0dv, int nv,
                                        const T *Y, size_t ystride, int &pha, int &paa, int &phb,
                                        int &pab, T (&sum)[NBAT])
{
    plane_split<T>(T(za), ka, v0dv, nv, pha, paa);
    plane_split<T>(T(zb), kb, v0dv, nv, phb, pab);
    const int n = pab - paa;      // >= 0: zb > za
    const int qa = min(paa, nv);  // a plane index even when n = 0 and a = nv + 1
    const T alpha = S.A * T(pl[qa].tau * lc - za);
    // Without selects: y[a-1] - y[e-1] is exactly 0 when n = 0 (a = e), and
    // the first term of the second sum, read at min(a, e - 1), is exactly 0
    // when n < 2; every index stays in [-1, nv].
    const int q1 = min(paa, pab - 1);
#pragma unroll
    for (int b = 0; b < NBAT; ++b) {
        const T *Yb = Y + b * ystride;
        const T ye = Yb[pab - 1];
        T d = Yb[q1] - ye;
        if (n >= 3) {  // rare: tested on n, the loop bounds only inside
            for (int q = paa + 1; q < pab - 1; ++q) d += Yb[q] - ye;
        }
        sum[b] = fma(cA, ye, fma(alpha, Yb[paa - 1] - ye, bA * d));
    }
}

// Straddle term t of a voxel (t < na: plane pha + t at za, added; else plane
// phb + t - na at zb, subtracted): the plane q, the face height e and the
// signed row differences; the term is K_cut(e) * dY.
template <typename T, int NBAT>
__host__ __device__ inline int adj_straddle(int t, int na, int pha, int phb, const PlaneRow<T> *pl,
                                            double lc, double za, double zb, const T *Y,
                                            size_t ystride, T &e, T (&dY)[NBAT])
{
    const bool top = t >= na;
    const int q = (top ? phb - na : pha) + t;
    e = T(pl[q].tau * lc - (top ? zb : za));
#pragma unroll
    for (int b = 0; b < NBAT; ++b) {
        const T d = Y[b * ystride + q - 1] - Y[b * ystride + q];
        dY[b] = top ? -d : d;
    }
    return q;
}

// One strip record's contribution to voxel [za, zb] of its column in the
// adjoint: sum_q (K_q(za) - K_q(zb)) (y[q-1] - y[q]) with y[-1] = y[nv] = 0.
template <typename T, int NBAT>
__host__ __device__ inline void adj_terms(const AdjTab<T> &S, double lc, T cA, T bA, const T *ka,
                                          const T *kb, const PlaneRow<T> *pl,
                                          double za, double zb, T v0dv, int nv, const T *Y,
                                          size_t ystride, T (&sum)[NBAT])
{
    int pha, paa, phb, pab;
    adj_lin<T, NBAT>(S, lc, cA, bA, ka, kb, pl, za, zb, v0dv, nv, Y, ystride, pha, paa, phb,
                     pab, sum);
    const int na = max(paa - pha, 0);
    const int nb = max(pab - phb, 0);
    for (int t = 0; t < na + nb; ++t) {
        T e, dY[NBAT];
        const int q = adj_straddle<T, NBAT>(t, na, pha, phb, pl, lc, za, zb, Y, ystride, e, dY);
        const T K = K_cut<T>(S, pl[q].tf, pl[q].inv, e);
#pragma unroll
        for (int b = 0; b < NBAT; ++b) sum[b] += K * dY[b];
    }
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
        for (int q = 0; q < 2; ++q) {
            const double us = q ? uhi : ulo;
            const double den = G.D * cp + us * sp;
            const double ya = (us * G.s + xa * (G.D * sp - us * cp)) / den;
            const double yb = (us * G.s + xb * (G.D * sp - us * cp)) / den;
            lo = dmin_(lo, dmin_(ya, yb));
            hi = dmax_(hi, dmax_(ya, yb));
        }
        const double pad = 1e-9 * G.b;
        double f0 = floor((lo - pad - G.y0) / G.b), f1 = floor((hi + pad - G.y0) / G.b);
        if (!(f0 == f0) || !(f1 == f1)) { f0 = 0; f1 = A.n_minor - 1; }
        j0 = (int)dmin_(dmax_(f0, 0.0), (double)A.n_minor);
        j1 = (int)dmax_(dmin_(f1, (double)(A.n_minor - 1)), -1.0);
    } else {
        const double ya = G.y0 + (double)i * G.b, yb = ya + G.b;
        for (int q = 0; q < 2; ++q) {
            const double us = q ? uhi : ulo;
            const double den = us * cp - G.D * sp;
            const double xa = (us * (G.s - ya * sp) - G.D * ya * cp) / den;
            const double xb = (us * (G.s - yb * sp) - G.D * yb * cp) / den;
            lo = dmin_(lo, dmin_(xa, xb));
            hi = dmax_(hi, dmax_(xa, xb));
        }
        const double pad = 1e-9 * G.a;
        double f0 = floor((lo - pad - G.x0) / G.a), f1 = floor((hi + pad - G.x0) / G.a);
        if (!(f0 == f0) || !(f1 == f1)) { f0 = 0; f1 = A.n_minor - 1; }
        j0 = (int)dmin_(dmax_(f0, 0.0), (double)A.n_minor);
        j1 = (int)dmax_(dmin_(f1, (double)(A.n_minor - 1)), -1.0);
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
        umin = dmin_(umin, u);
        umax = dmax_(umax, u);
    }
    const double pad = 1e-9 * G.du;
    const double f0 = floor((umin - pad - G.u0) / G.du), f1 = floor((umax + pad - G.u0) / G.du);
    k0 = (int)dmin_(dmax_(f0, 0.0), (double)G.nu);
    k1 = (int)dmax_(dmin_(f1, (double)(G.nu - 1)), -1.0);
}

__host__ __device__ inline void pixel_columns(const DevGeom &G, double cp, double sp, int ix,
                                              int iy, int &k0, int &k1)
{
    corner_columns(G, cp, sp, ix, ix + 1, iy, iy + 1, k0, k1);
}

// Position of pixel (ix, iy) in the walk of a strip whose per-major table is
// (j0[i], off[i], off[i+1]); -1 when the pixel is not in the strip.
__host__ __device__ inline int strip_position(bool major_x, int ix, int iy, const int *j0,
                                              const int *off)
{
    const int i = major_x ? ix : iy, j = major_x ? iy : ix;
    const int a = j0[i], cnt = off[i + 1] - off[i];
    return (j >= a && j < a + cnt) ? off[i] + (j - a) : -1;
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
    const int base = xcd < full ? xcd * per : full * per + (xcd - full) * (per - 1);
    return base + slot;
}

}  // namespace smk
