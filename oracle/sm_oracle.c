/*
 * sm_oracle.c -- plain, slow, FP64 reference for the exact cone-beam system
 * matrix of Simbrunner, Krenn, Zach, Habring, "Computation of a Consistent
 * System Matrix for Cone-beam Computed Tomography" (arXiv 2511.12235).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is loaded by the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark; the product path
 * never links, loads or calls it.  It shares no source, header, table or
 * helper with the HIP implementation.
 *
 * What it computes (Sec. I, eqs. "inverse problem" and "ip", and the
 * definition of consistency that follows them): the system-matrix entry W_ij
 * is the measure (area in 2D, volume in 3D, absolute units) of the part of
 * voxel j that lies inside the beam of detector element i, i.e. inside the
 * pyramid (wedge in 2D) spanned by the point source and the element.  The
 * oracle evaluates that definition directly: it clips the voxel box by the
 * planes bounding the beam (Sutherland-Hodgman on every face, a cap polygon
 * per cutting plane) and measures the clipped convex body.  None of the
 * paper's closed forms are used here; the tests compare those closed forms
 * against this clipping result instead.
 *
 * Geometry (Sec. III-A, eq. "z rotation" and the appendix "Fundamental
 * relations"): the source sits at S = (s cos(phi), s sin(phi), 0); the flat
 * detector is perpendicular to S->O at distance d beyond the origin, so the
 * source-detector distance is D = s + d.  For a point p = (x, y, z),
 *     l(p) = s - (x cos(phi) + y sin(phi))      depth along the central ray,
 *     t(p) = y cos(phi) - x sin(phi)            lateral offset,
 * and its detector coordinates are u = D t / l (the tan(beta) relation
 * "tan beta" times s + d) and v = D z / l (the z-relation "z expr 1").
 * Detector column m_y covers [det_y0 + m_y dy, det_y0 + (m_y + 1) dy] in u,
 * row m_z covers [det_z0 + m_z dz, det_z0 + (m_z + 1) dz] in v.  The beam of
 * element (m_y, m_z) is
 *     { l > 0,  u_k <= D t / l <= u_{k+1},  v_r <= D z / l <= v_{r+1} },
 * bounded by the four planes  D t - u_k l >= 0,  u_{k+1} l - D t >= 0,
 * D z - v_r l >= 0,  v_{r+1} l - D z >= 0 (all through S).  In 2D the z
 * coordinate is dropped (Sec. III-A, first paragraph).
 *
 * Voxel (ix, iy, iz) is [x0 + ix a, x0 + (ix+1) a] x [y0 + iy b, ...] x
 * [z0 + iz c, ...] (Sec. III-A, vertices V_{n,ij}); its linear index is
 * j = (iz ny + iy) nx + ix.  Measurement index i = (view det_nz + m_z)
 * det_ny + m_y (Sec. I: M = N_d N_p measurements).
 *
 * Footprint (eq. "relevant detectors 2d" and the 3D row bounds of Sec.
 * III-C): with strict inequalities, a column/row is relevant when its open
 * interval meets the open interval spanned by the voxel's detector
 * coordinates.  The box is computed with the fixed FP64 expression order
 * documented at fp_corner(); this file must be compiled without FMA
 * contraction so the box is reproducible bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t dim;             /* 2 or 3 */
    int32_t nx, ny, nz;      /* voxel counts (nz = 1 in 2D) */
    double a, b, c;          /* voxel side lengths (c unused in 2D) */
    double x0, y0, z0;       /* grid minimum corner */
    int32_t n_p;             /* number of views */
    int32_t pad0;
    const double *phi;       /* n_p rotation angles (radians) */
    const double *trig;      /* optional n_p (cos, sin) pairs; overrides phi */
    double s, d;             /* source-origin, origin-detector distances */
    int32_t det_ny, det_nz;  /* detector columns (along u), rows (along v) */
    double dy, dz;           /* detector element side lengths */
    double det_y0, det_z0;   /* coordinate of the first detector corner */
} orc_geom;

/* ------------------------------------------------------------------ */
/* per-view trigonometry                                                */
/* ------------------------------------------------------------------ */
static void view_trig(const orc_geom *g, int view, double *cp, double *sp)
{
    if (g->trig) {
        *cp = g->trig[2 * view];
        *sp = g->trig[2 * view + 1];
    } else {
        *cp = cos(g->phi[view]);
        *sp = sin(g->phi[view]);
    }
}

/* ------------------------------------------------------------------ */
/* footprint box                                                        */
/* ------------------------------------------------------------------ */
/* Depth and detector-u of one top-view corner, in this exact order:
 *   l = s - (x*cp + y*sp);  t = y*cp - x*sp;  u = (D*t)/l.            */
static void fp_corner(const orc_geom *g, double cp, double sp, double x, double y,
                      double *l, double *u)
{
    const double D = g->s + g->d;
    double ll = g->s - (x * cp + y * sp);
    double tt = y * cp - x * sp;
    *l = ll;
    *u = (D * tt) / ll;
}

/* Cells m in [0, n) of the grid o + m p (p > 0) whose open interval meets the
 * open interval (lo, hi): o + m p < hi and o + (m + 1) p > lo.  The floor
 * estimate only seeds the walk; the exact comparisons decide.              */
static void cell_range(double lo, double hi, double o, double p, int n,
                       int *first, int *last)
{
    double e = floor((lo - o) / p);
    int m = e < 0 ? 0 : (e > n ? n : (int)e);
    while (m > 0 && o + (double)m * p > lo) m--;
    while (m < n && !(o + (double)(m + 1) * p > lo)) m++;
    *first = m;
    e = floor((hi - o) / p);
    m = e < -1 ? -1 : (e > n - 1 ? n - 1 : (int)e);
    while (m < n - 1 && o + (double)(m + 1) * p < hi) m++;
    while (m >= 0 && !(o + (double)m * p < hi)) m--;
    *last = m;
}

/* Footprint of voxel (ix, iy, iz) in one view.  Returns 1 when non-empty,
 * 0 when empty, -1 when a corner has l <= 0 (source inside the grid).     */
static int footprint(const orc_geom *g, double cp, double sp, int ix, int iy, int iz,
                     int box[4])
{
    const double D = g->s + g->d;
    const double xs[2] = { g->x0 + (double)ix * g->a, g->x0 + (double)(ix + 1) * g->a };
    const double ys[2] = { g->y0 + (double)iy * g->b, g->y0 + (double)(iy + 1) * g->b };
    double umin = INFINITY, umax = -INFINITY, lmin = INFINITY, lmax = -INFINITY;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double l, u;
            fp_corner(g, cp, sp, xs[i], ys[j], &l, &u);
            if (!(l > 0.0)) return -1;
            if (u < umin) umin = u;
            if (u > umax) umax = u;
            if (l < lmin) lmin = l;
            if (l > lmax) lmax = l;
        }
    cell_range(umin, umax, g->det_y0, g->dy, g->det_ny, &box[0], &box[1]);
    if (g->dim == 2) {
        box[2] = 0;
        box[3] = 0;
    } else {
        const double za = g->z0 + (double)iz * g->c;
        const double zb = g->z0 + (double)(iz + 1) * g->c;
        double v1 = (D * za) / lmin, v2 = (D * za) / lmax;
        double v3 = (D * zb) / lmin, v4 = (D * zb) / lmax;
        double vmin = v1 < v2 ? v1 : v2;
        double vmax = v3 > v4 ? v3 : v4;
        cell_range(vmin, vmax, g->det_z0, g->dz, g->det_nz, &box[2], &box[3]);
    }
    return (box[0] <= box[1] && box[2] <= box[3]) ? 1 : 0;
}

/* ------------------------------------------------------------------ */
/* 2D: rectangle clipped by half-planes, shoelace area                  */
/* ------------------------------------------------------------------ */
#define P2MAX 16

/* plane: pl[0] + pl[1] qx + pl[2] qy >= 0 */
static int clip_poly2(double (*in)[2], int n, double (*out)[2], const double pl[3])
{
    int m = 0;
    for (int i = 0; i < n; ++i) {
        const double *p = in[i], *q = in[(i + 1) % n];
        double fp = pl[0] + pl[1] * p[0] + pl[2] * p[1];
        double fq = pl[0] + pl[1] * q[0] + pl[2] * q[1];
        if (fp >= 0.0) {
            out[m][0] = p[0];
            out[m][1] = p[1];
            ++m;
        }
        if ((fp > 0.0 && fq < 0.0) || (fp < 0.0 && fq > 0.0)) {
            double t = fp / (fp - fq);
            out[m][0] = p[0] + t * (q[0] - p[0]);
            out[m][1] = p[1] + t * (q[1] - p[1]);
            ++m;
        }
    }
    return m;
}

static double shoelace(double (*p)[2], int n)
{
    double acc = 0.0;
    for (int i = 0; i < n; ++i) {
        const double *a = p[i], *b = p[(i + 1) % n];
        acc += a[0] * b[1] - a[1] * b[0];
    }
    return 0.5 * fabs(acc);
}

/* Area of [-hx,hx] x [-hy,hy] inside all half-planes (np rows of 3). */
double orc_clip_rect(double hx, double hy, const double *planes, int np)
{
    double A[P2MAX][2], B[P2MAX][2];
    int n = 4;
    A[0][0] = -hx; A[0][1] = -hy;
    A[1][0] = hx;  A[1][1] = -hy;
    A[2][0] = hx;  A[2][1] = hy;
    A[3][0] = -hx; A[3][1] = hy;
    for (int k = 0; k < np && n >= 3; ++k) {
        n = clip_poly2(A, n, B, planes + 3 * k);
        memcpy(A, B, sizeof(double) * 2 * (size_t)n);
    }
    return n >= 3 ? shoelace(A, n) : 0.0;
}

/* ------------------------------------------------------------------ */
/* 3D: convex polyhedron clipped by half-spaces                         */
/* ------------------------------------------------------------------ */
#define PF_MAXV 24
#define PH_MAXF 16
#define CAP_MAX (2 * PH_MAXF * PF_MAXV)

typedef struct {
    int n;
    double v[PF_MAXV][3];
} pface;

typedef struct {
    int nf;
    pface f[PH_MAXF];
} phedron;

static double plane_eval(const double pl[4], const double *q)
{
    return pl[0] + pl[1] * q[0] + pl[2] * q[1] + pl[3] * q[2];
}

static void box_hedron(phedron *P, double hx, double hy, double hz)
{
    /* corners indexed by bits (x, y, z) */
    double C[8][3];
    for (int i = 0; i < 8; ++i) {
        C[i][0] = (i & 1) ? hx : -hx;
        C[i][1] = (i & 2) ? hy : -hy;
        C[i][2] = (i & 4) ? hz : -hz;
    }
    static const int F[6][4] = {
        { 0, 2, 6, 4 }, /* x = -hx */
        { 1, 5, 7, 3 }, /* x = +hx */
        { 0, 4, 5, 1 }, /* y = -hy */
        { 2, 3, 7, 6 }, /* y = +hy */
        { 0, 1, 3, 2 }, /* z = -hz */
        { 4, 6, 7, 5 }, /* z = +hz */
    };
    P->nf = 6;
    for (int f = 0; f < 6; ++f) {
        P->f[f].n = 4;
        for (int k = 0; k < 4; ++k) memcpy(P->f[f].v[k], C[F[f][k]], sizeof(double) * 3);
    }
}

/* Order coplanar points by angle around their centroid in the plane with
 * normal nrm (insertion sort; the point sets are tiny).                   */
static void sort_cap(double (*pts)[3], int n, const double nrm[3])
{
    double cen[3] = { 0, 0, 0 };
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) cen[k] += pts[i][k];
    for (int k = 0; k < 3; ++k) cen[k] /= n;
    /* orthonormal basis e1, e2 of the plane */
    double e1[3];
    if (fabs(nrm[0]) <= fabs(nrm[1]) && fabs(nrm[0]) <= fabs(nrm[2])) {
        e1[0] = 0; e1[1] = nrm[2]; e1[2] = -nrm[1];
    } else if (fabs(nrm[1]) <= fabs(nrm[2])) {
        e1[0] = -nrm[2]; e1[1] = 0; e1[2] = nrm[0];
    } else {
        e1[0] = nrm[1]; e1[1] = -nrm[0]; e1[2] = 0;
    }
    double e2[3] = { nrm[1] * e1[2] - nrm[2] * e1[1], nrm[2] * e1[0] - nrm[0] * e1[2],
                     nrm[0] * e1[1] - nrm[1] * e1[0] };
    double ang[CAP_MAX];
    for (int i = 0; i < n; ++i) {
        double r[3] = { pts[i][0] - cen[0], pts[i][1] - cen[1], pts[i][2] - cen[2] };
        ang[i] = atan2(r[0] * e2[0] + r[1] * e2[1] + r[2] * e2[2],
                       r[0] * e1[0] + r[1] * e1[1] + r[2] * e1[2]);
    }
    for (int i = 1; i < n; ++i) {
        double a = ang[i], p[3] = { pts[i][0], pts[i][1], pts[i][2] };
        int j = i - 1;
        while (j >= 0 && ang[j] > a) {
            ang[j + 1] = ang[j];
            memcpy(pts[j + 1], pts[j], sizeof(double) * 3);
            --j;
        }
        ang[j + 1] = a;
        memcpy(pts[j + 1], p, sizeof(double) * 3);
    }
}

/* Keep the part of P where pl >= 0; closes the cut with a cap face. */
static void clip_hedron(phedron *P, const double pl[4])
{
    static __thread phedron out;
    static __thread double cap[CAP_MAX][3];
    int ncap = 0, cut = 0;
    out.nf = 0;
    for (int f = 0; f < P->nf; ++f) {
        const pface *F = &P->f[f];
        pface *G = &out.f[out.nf];
        G->n = 0;
        for (int i = 0; i < F->n; ++i) {
            const double *p = F->v[i], *q = F->v[(i + 1) % F->n];
            double fp = plane_eval(pl, p), fq = plane_eval(pl, q);
            if (fp < 0.0) cut = 1;
            if (fp >= 0.0) {
                memcpy(G->v[G->n++], p, sizeof(double) * 3);
                if (fp == 0.0 && ncap < CAP_MAX) memcpy(cap[ncap++], p, sizeof(double) * 3);
            }
            if ((fp > 0.0 && fq < 0.0) || (fp < 0.0 && fq > 0.0)) {
                double t = fp / (fp - fq);
                double x[3] = { p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1]),
                                p[2] + t * (q[2] - p[2]) };
                memcpy(G->v[G->n++], x, sizeof(double) * 3);
                if (ncap < CAP_MAX) memcpy(cap[ncap++], x, sizeof(double) * 3);
            }
        }
        if (G->n >= 3) out.nf++;
    }
    /* A cap is needed only when something was cut away; a face lying in the
     * plane (all other vertices inside) must not be duplicated.           */
    if (cut && ncap >= 3 && out.nf > 0 && out.nf < PH_MAXF) {
        double nn = sqrt(pl[1] * pl[1] + pl[2] * pl[2] + pl[3] * pl[3]);
        double nrm[3] = { pl[1] / nn, pl[2] / nn, pl[3] / nn };
        sort_cap(cap, ncap, nrm);
        pface *G = &out.f[out.nf];
        int m = ncap < PF_MAXV ? ncap : PF_MAXV;
        G->n = m;
        for (int i = 0; i < m; ++i) memcpy(G->v[i], cap[i], sizeof(double) * 3);
        out.nf++;
    }
    *P = out;
}

/* Volume of a convex polyhedron: sum over faces of pyramids with apex at the
 * vertex mean (inside, by convexity).  Orientation-independent.           */
static double hedron_volume(const phedron *P)
{
    double ref[3] = { 0, 0, 0 };
    int cnt = 0;
    for (int f = 0; f < P->nf; ++f)
        for (int i = 0; i < P->f[f].n; ++i) {
            for (int k = 0; k < 3; ++k) ref[k] += P->f[f].v[i][k];
            ++cnt;
        }
    if (cnt == 0) return 0.0;
    for (int k = 0; k < 3; ++k) ref[k] /= cnt;
    double vol = 0.0;
    for (int f = 0; f < P->nf; ++f) {
        const pface *F = &P->f[f];
        double r0[3] = { F->v[0][0] - ref[0], F->v[0][1] - ref[1], F->v[0][2] - ref[2] };
        double acc = 0.0;
        for (int i = 1; i + 1 < F->n; ++i) {
            double r1[3] = { F->v[i][0] - ref[0], F->v[i][1] - ref[1], F->v[i][2] - ref[2] };
            double r2[3] = { F->v[i + 1][0] - ref[0], F->v[i + 1][1] - ref[1],
                             F->v[i + 1][2] - ref[2] };
            /* det(r0, r1, r2) */
            acc += r0[0] * (r1[1] * r2[2] - r1[2] * r2[1]) - r0[1] * (r1[0] * r2[2] - r1[2] * r2[0]) +
                   r0[2] * (r1[0] * r2[1] - r1[1] * r2[0]);
        }
        vol += fabs(acc) / 6.0;
    }
    return vol;
}

/* Volume of [-hx,hx] x [-hy,hy] x [-hz,hz] inside all half-spaces
 * (np rows of 4: alpha, bx, by, bz;  alpha + b.q >= 0).                   */
double orc_clip_box(double hx, double hy, double hz, const double *planes, int np)
{
    phedron P;
    box_hedron(&P, hx, hy, hz);
    for (int k = 0; k < np && P.nf > 0; ++k) clip_hedron(&P, planes + 4 * k);
    return P.nf > 0 ? hedron_volume(&P) : 0.0;
}

/* ------------------------------------------------------------------ */
/* cell measure: voxel (ix,iy,iz) inside the beam of element (k, r)     */
/* ------------------------------------------------------------------ */
/* The beam's bounding planes written in coordinates q relative to the voxel
 * centre (xc, yc, zc):  l = lc - (qx cp + qy sp),  t = tc + (qy cp - qx sp).  */
static double cell_measure_c(const orc_geom *g, double cp, double sp, int ix, int iy,
                             int iz, int k, int r)
{
    const double D = g->s + g->d;
    const double xc = g->x0 + ((double)ix + 0.5) * g->a;
    const double yc = g->y0 + ((double)iy + 0.5) * g->b;
    const double lc = g->s - (xc * cp + yc * sp);
    const double tc = yc * cp - xc * sp;
    const double uk = g->det_y0 + (double)k * g->dy;
    const double uk1 = g->det_y0 + (double)(k + 1) * g->dy;
    /* D t - u l >= 0 :  (D tc - u lc) + qx (-D sp + u cp) + qy (D cp + u sp) */
    if (g->dim == 2) {
        double pl[6] = { D * tc - uk * lc, -D * sp + uk * cp, D * cp + uk * sp,
                         -(D * tc - uk1 * lc), -(-D * sp + uk1 * cp), -(D * cp + uk1 * sp) };
        return orc_clip_rect(0.5 * g->a, 0.5 * g->b, pl, 2);
    }
    const double zc = g->z0 + ((double)iz + 0.5) * g->c;
    const double vr = g->det_z0 + (double)r * g->dz;
    const double vr1 = g->det_z0 + (double)(r + 1) * g->dz;
    /* D z - v l >= 0 :  (D zc - v lc) + qx (v cp) + qy (v sp) + qz D */
    double pl[16] = {
        D * tc - uk * lc,      -D * sp + uk * cp,    D * cp + uk * sp,    0.0,
        -(D * tc - uk1 * lc),  -(-D * sp + uk1 * cp), -(D * cp + uk1 * sp), 0.0,
        D * zc - vr * lc,      vr * cp,              vr * sp,             D,
        -(D * zc - vr1 * lc),  -(vr1 * cp),          -(vr1 * sp),         -D,
    };
    return orc_clip_box(0.5 * g->a, 0.5 * g->b, 0.5 * g->c, pl, 4);
}

/* ------------------------------------------------------------------ */
/* exported entry points                                                */
/* ------------------------------------------------------------------ */

/* 0 when every voxel corner has l > 0 in every view, else -1. */
int orc_validate(const orc_geom *g)
{
    double xs[2] = { g->x0, g->x0 + (double)g->nx * g->a };
    double ys[2] = { g->y0, g->y0 + (double)g->ny * g->b };
    for (int v = 0; v < g->n_p; ++v) {
        double cp, sp;
        view_trig(g, v, &cp, &sp);
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                if (!(g->s - (xs[i] * cp + ys[j] * sp) > 0.0)) return -1;
    }
    return 0;
}

/* Footprint boxes of every voxel in one view: out[j*4 + {0..3}] =
 * (first column, last column, first row, last row); empty boxes have
 * first > last.  Returns -1 on invalid geometry.                          */
int orc_footprints(const orc_geom *g, int view, int32_t *out)
{
    double cp, sp;
    view_trig(g, view, &cp, &sp);
    for (int iz = 0; iz < g->nz; ++iz)
        for (int iy = 0; iy < g->ny; ++iy)
            for (int ix = 0; ix < g->nx; ++ix) {
                int box[4];
                if (footprint(g, cp, sp, ix, iy, iz, box) < 0) return -1;
                size_t j = ((size_t)iz * g->ny + iy) * g->nx + ix;
                for (int k = 0; k < 4; ++k) out[4 * j + k] = box[k];
            }
    return 0;
}

/* Exact measure of voxel (ix,iy,iz) inside element (k, r) in one view. */
double orc_cell_measure(const orc_geom *g, int view, int ix, int iy, int iz, int k, int r)
{
    double cp, sp;
    view_trig(g, view, &cp, &sp);
    return cell_measure_c(g, cp, sp, ix, iy, iz, k, r);
}

/* Exact measure of the whole grid box inside element (k, r) in one view
 * (the row sum of W for that element).                                   */
double orc_ray_gridbox(const orc_geom *g, int view, int k, int r)
{
    double cp, sp;
    view_trig(g, view, &cp, &sp);
    const double D = g->s + g->d;
    const double xc = g->x0 + 0.5 * (double)g->nx * g->a;
    const double yc = g->y0 + 0.5 * (double)g->ny * g->b;
    const double lc = g->s - (xc * cp + yc * sp);
    const double tc = yc * cp - xc * sp;
    const double uk = g->det_y0 + (double)k * g->dy;
    const double uk1 = g->det_y0 + (double)(k + 1) * g->dy;
    const double hx = 0.5 * (double)g->nx * g->a, hy = 0.5 * (double)g->ny * g->b;
    if (g->dim == 2) {
        double pl[6] = { D * tc - uk * lc, -D * sp + uk * cp, D * cp + uk * sp,
                         -(D * tc - uk1 * lc), -(-D * sp + uk1 * cp), -(D * cp + uk1 * sp) };
        return orc_clip_rect(hx, hy, pl, 2);
    }
    const double zc = g->z0 + 0.5 * (double)g->nz * g->c;
    const double hz = 0.5 * (double)g->nz * g->c;
    const double vr = g->det_z0 + (double)r * g->dz;
    const double vr1 = g->det_z0 + (double)(r + 1) * g->dz;
    double pl[16] = {
        D * tc - uk * lc,      -D * sp + uk * cp,    D * cp + uk * sp,    0.0,
        -(D * tc - uk1 * lc),  -(-D * sp + uk1 * cp), -(D * cp + uk1 * sp), 0.0,
        D * zc - vr * lc,      vr * cp,              vr * sp,             D,
        -(D * zc - vr1 * lc),  -(vr1 * cp),          -(vr1 * sp),         -D,
    };
    return orc_clip_box(hx, hy, hz, pl, 4);
}

/* orc_ray_gridbox for every element of one view, out[r * det_ny + k]
 * (parallel over rows; each element is the same single clip).            */
void orc_ray_gridbox_view(const orc_geom *g, int view, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < g->det_nz; ++r)
        for (int k = 0; k < g->det_ny; ++k)
            out[(int64_t)r * g->det_ny + k] = orc_ray_gridbox(g, view, k, r);
}

/* Visit every kept entry (W > tau) of one view, voxels in ascending j, cells
 * of a voxel in ascending (r, k).  Returns the number of entries or -1.    */
typedef void (*entry_fn)(void *ctx, int64_t i, int64_t j, double w);

static int64_t walk_view(const orc_geom *g, int view, double tau, entry_fn fn, void *ctx)
{
    double cp, sp;
    view_trig(g, view, &cp, &sp);
    int64_t cnt = 0;
    for (int iz = 0; iz < g->nz; ++iz)
        for (int iy = 0; iy < g->ny; ++iy)
            for (int ix = 0; ix < g->nx; ++ix) {
                int box[4];
                int st = footprint(g, cp, sp, ix, iy, iz, box);
                if (st < 0) return -1;
                if (st == 0) continue;
                int64_t j = ((int64_t)iz * g->ny + iy) * g->nx + ix;
                for (int r = box[2]; r <= box[3]; ++r)
                    for (int k = box[0]; k <= box[1]; ++k) {
                        double w = cell_measure_c(g, cp, sp, ix, iy, iz, k, r);
                        if (w > tau) {
                            int64_t i = ((int64_t)view * g->det_nz + r) * g->det_ny + k;
                            if (fn) fn(ctx, i, j, w);
                            ++cnt;
                        }
                    }
            }
    return cnt;
}

typedef struct {
    int64_t pos;
    int64_t *rows;
    int32_t *cols;
    double *vals;
} fill_ctx;

static void fill_entry(void *ctx, int64_t i, int64_t j, double w)
{
    fill_ctx *f = (fill_ctx *)ctx;
    f->rows[f->pos] = i;
    f->cols[f->pos] = (int32_t)j;
    f->vals[f->pos] = w;
    f->pos++;
}

/* Number of kept entries per view for views [v0, v1): counts[v - v0].
 * Returns the total or -1.                                               */
int64_t orc_count(const orc_geom *g, int v0, int v1, double tau, int64_t *counts)
{
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int v = v0; v < v1; ++v) {
        int64_t c = walk_view(g, v, tau, NULL, NULL);
        if (c < 0) bad = 1;
        counts[v - v0] = c;
    }
    if (bad) return -1;
    int64_t tot = 0;
    for (int v = v0; v < v1; ++v) tot += counts[v - v0];
    return tot;
}

/* Fill entries of views [v0, v1) given the per-view counts from orc_count.
 * Within a view the entries are ordered by voxel j, then (r, k); the Python
 * wrapper sorts them by (i, j).                                          */
int orc_fill(const orc_geom *g, int v0, int v1, double tau, const int64_t *counts,
             int64_t *rows, int32_t *cols, double *vals)
{
    int n = v1 - v0;
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!off) return -1;
    off[0] = 0;
    for (int v = 0; v < n; ++v) off[v + 1] = off[v] + counts[v];
#pragma omp parallel for schedule(dynamic, 1)
    for (int v = v0; v < v1; ++v) {
        fill_ctx f = { off[v - v0], rows, cols, vals };
        walk_view(g, v, tau, fill_entry, &f);
    }
    free(off);
    return 0;
}

/* y = W x for the listed views (y holds n_sel * det_nz * det_ny values in
 * view-list order).  Each view is summed serially in voxel order, so the
 * result does not depend on the thread count.                            */
typedef struct {
    const double *x;
    double *y;
    int64_t ybase;
} fwd_ctx;

static void fwd_entry(void *ctx, int64_t i, int64_t j, double w)
{
    fwd_ctx *f = (fwd_ctx *)ctx;
    f->y[i - f->ybase] += w * f->x[j];
}

int orc_forward(const orc_geom *g, const double *x, const int32_t *views, int n_sel,
                double tau, double *y)
{
    const int64_t per = (int64_t)g->det_nz * g->det_ny;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int q = 0; q < n_sel; ++q) {
        double *yq = y + (int64_t)q * per;
        for (int64_t i = 0; i < per; ++i) yq[i] = 0.0;
        fwd_ctx f = { x, yq, (int64_t)views[q] * per };
        if (walk_view(g, views[q], tau, fwd_entry, &f) < 0) bad = 1;
    }
    return bad ? -1 : 0;
}

/* x_j = sum_i W_ij y_i for the listed voxels j (all views, all cells).    */
int orc_back(const orc_geom *g, const double *y, const int64_t *vox, int64_t n_sel,
             double tau, double *x)
{
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n_sel; ++q) {
        int64_t j = vox[q];
        int ix = (int)(j % g->nx);
        int iy = (int)((j / g->nx) % g->ny);
        int iz = (int)(j / ((int64_t)g->nx * g->ny));
        double acc = 0.0;
        for (int v = 0; v < g->n_p; ++v) {
            double cp, sp;
            view_trig(g, v, &cp, &sp);
            int box[4];
            int st = footprint(g, cp, sp, ix, iy, iz, box);
            if (st < 0) { bad = 1; break; }
            if (st == 0) continue;
            for (int r = box[2]; r <= box[3]; ++r)
                for (int k = box[0]; k <= box[1]; ++k) {
                    double w = cell_measure_c(g, cp, sp, ix, iy, iz, k, r);
                    if (w > tau) acc += w * y[((int64_t)v * g->det_nz + r) * g->det_ny + k];
                }
        }
        x[q] = acc;
    }
    return bad ? -1 : 0;
}

/* y_i = sum_j W_ij x_j for a list of rays i (brute force over all voxels:
 * every voxel whose footprint box holds the element is clipped).  Parallel
 * over rays; each ray is summed serially in voxel order.                  */
int orc_forward_rays(const orc_geom *g, const double *x, const int64_t *rays, int64_t n_sel,
                     double tau, double *y)
{
    int bad = 0;
    const int64_t per = (int64_t)g->det_nz * g->det_ny;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < n_sel; ++q) {
        const int64_t i = rays[q];
        const int view = (int)(i / per);
        const int r = (int)((i % per) / g->det_ny);
        const int k = (int)(i % g->det_ny);
        double cp, sp;
        view_trig(g, view, &cp, &sp);
        double acc = 0.0;
        for (int iz = 0; iz < g->nz; ++iz)
            for (int iy = 0; iy < g->ny; ++iy)
                for (int ix = 0; ix < g->nx; ++ix) {
                    int box[4];
                    int st = footprint(g, cp, sp, ix, iy, iz, box);
                    if (st < 0) { bad = 1; continue; }
                    if (st == 0 || k < box[0] || k > box[1] || r < box[2] || r > box[3]) continue;
                    double w = cell_measure_c(g, cp, sp, ix, iy, iz, k, r);
                    if (w > tau) acc += w * x[((int64_t)iz * g->ny + iy) * g->nx + ix];
                }
        y[q] = acc;
    }
    return bad ? -1 : 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
