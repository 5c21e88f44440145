// Host check of the adjoint's staged strip record (test helper, built and run
// by tests/test_host_kcut.py; no GPU needed).
//
// The adjoint evaluates K (Sec. III-C: the volume of a strip column above a
// face and below a row plane) on a staged copy of each strip record: the
// cubic coefficient of Psi on every segment is taken once per record, and
// lambda is clamped to [d0, dn] before h = dB - lambda.  The forward
// evaluates it on the record itself: the coefficient per term, and h clamped
// to [0, L].  This program builds the records of a small cone-beam scan with
// build_record, converts each as the adjoint's staging does, and checks that
// both forms give the same K bit for bit (host arithmetic) for face heights
// that put lambda below the nearest depth, inside the table and beyond the
// farthest depth, on rising, falling and level planes.  It also checks the
// plane split the adjoint takes from the staged index-scale pairs (the pair
// chosen by the sign of the face height) against each plane's height range
// over the strip: planes put wholly below a face reach no higher than it,
// planes put wholly above reach no lower, and every plane clear of the face
// by more than rounding is put on its side.  Last, the adjoint's linear part
// of a record (adj_lin: the planes reaching into a voxel from above its
// bottom face summed by parts, with the absent terms read as exact zeros)
// against the direct sum over those planes of A (tau_q lc - za) times
// y[q-1] - y[q], plus c A y for the planes wholly above the voxel.  And the
// zero header an empty slot gets in FP32 single-volume launches: its terms
// (adj_terms) are exactly zero for every voxel, without reading the table
// (filled with NaN here).
#include "../paper_2511_12235_amd/csrc/sm_common.h"

#include <cmath>
#include <cstdio>
#include <cstring>

using namespace smk;

template <typename T>
static AdjRec<T> staged(const Rec<T> &R)
{
    AdjRec<T> A;
    std::memset(&A, 0, sizeof A);
    A.lc = R.lc;
    A.n = R.n;
    A.k4[0] = R.kLo;
    A.k4[1] = R.kHi;
    A.k4[2] = R.kHi;
    A.k4[3] = R.kLo;
    A.cA = R.cA;
    A.bA = R.bA;
    A.d0 = R.tab[0][0];
    A.A = R.tab[0][2];
    for (int r = 1; r < MAXV; ++r) {
        for (int c = 0; c < 4; ++c) A.seg[r - 1][c] = R.tab[r][c];
        const T L = R.tab[r][0] - R.tab[r - 1][0];
        A.g6[r - 1] = (R.tab[r - 1][1] - R.tab[r][1]) * rcp_(L > T(1e-30) ? L : T(1e-30)) * T(1.0 / 3.0);
    }
    return A;
}

template <typename T>
static long check(const DevGeom &G, long &checked)
{
    long bad = 0;
    double2 scratch[8];
    const int nview = 7;
    const double angles[nview] = {0.0, 0.5 * M_PI, 0.3, 1.1, 2.0, 3.9, 5.5};
    for (int v = 0; v < nview; ++v) {
        const double cp = std::cos(angles[v]), sp = std::sin(angles[v]);
        for (int iy = 0; iy < G.ny; ++iy)
            for (int ix = 0; ix < G.nx; ++ix)
                for (int k = 0; k < G.nu; ++k) {
                    Rec<T> R;
                    std::memset(&R, 0, sizeof R);
                    build_record<T>(G, cp, sp, ix, iy, k, R, scratch);
                    if (R.n == 0) continue;
                    const AdjRec<T> A = staged(R);
                    const StripTab<T> S = strip_tab<T>(R.tab, R.tab);
                    const AdjTab<T> Q = adj_tab<T>(A);
                    const T d0 = R.tab[0][0], dn = R.tab[MAXV - 1][0];
                    for (int q = 0; q <= G.nv; ++q) {
                        const T tau = T(G.tau[q]);
                        const T inv = tau != T(0) ? T(1) / tau : T(0);
                        for (int i = 0; i <= 40; ++i) {
                            // lambda from below d0 to beyond dn
                            const T lam = d0 - T(0.5) + (dn - d0 + T(1)) * T(i) / T(40);
                            const T e = tau != T(0) ? -lam * tau : T(0.25) * T(i - 20);
                            const T k1 = K_cut<T>(S, tau, inv, e), k2 = K_cut<T>(Q, tau, inv, e);
                            ++checked;
                            if (std::memcmp(&k1, &k2, sizeof(T)) != 0) {
                                if (bad < 5)
                                    std::printf("mismatch %s view %d pixel (%d,%d) column %d plane %d: %.17g %.17g\n",
                                                sizeof(T) == 4 ? "fp32" : "fp64", v, ix, iy, k, q,
                                                (double)k1, (double)k2);
                                ++bad;
                            }
                        }
                    }
                }
    }
    return bad;
}

// Row planes q < ph must lie below face z and q >= pa above it (within tol),
// and planes clear of z by more than tol must be classified so.
template <typename T>
static long check_splits(const DevGeom &G, long &checked)
{
    long bad = 0;
    double2 scratch[8];
    const double tol = sizeof(T) == 4 ? 1e-4 : 1e-9;
    const double angles[4] = {0.0, 0.7, 2.3, 4.4};
    for (int v = 0; v < 4; ++v) {
        const double cp = std::cos(angles[v]), sp = std::sin(angles[v]);
        for (int iy = 0; iy < G.ny; ++iy)
            for (int ix = 0; ix < G.nx; ++ix)
                for (int k = 0; k < G.nu; ++k) {
                    Rec<T> R;
                    std::memset(&R, 0, sizeof R);
                    build_record<T>(G, cp, sp, ix, iy, k, R, scratch);
                    if (R.n == 0) continue;
                    const AdjRec<T> A = staged(R);
                    const double Llo = R.lc + (double)R.tab[0][0], Lhi = R.lc + (double)R.tab[MAXV - 1][0];
                    for (int j = 0; j <= G.nz; ++j) {
                        const double z = G.z0 + j * G.c;
                        const T zf = T(z);
                        int ph, pa;
                        plane_split<T>(zf, A.k4 + (zf >= T(0) ? 2 : 0), T(G.v0 / G.dv), G.nv, ph, pa);
                        for (int q = 0; q <= G.nv; ++q) {
                            const double t = G.tau[q];
                            const double lo = t >= 0 ? t * Llo : t * Lhi, hi = t >= 0 ? t * Lhi : t * Llo;
                            const bool below = q < ph, above = q >= pa;
                            const bool ok = (!below || hi <= z + tol) && (!above || lo >= z - tol) &&
                                            (!(hi < z - tol) || below) && (!(lo > z + tol) || above);
                            ++checked;
                            if (!ok) {
                                if (bad < 5)
                                    std::printf("split %s view %d pixel (%d,%d) column %d face %d plane %d: "
                                                "ph %d pa %d range [%.9g, %.9g] z %.9g\n",
                                                sizeof(T) == 4 ? "fp32" : "fp64", v, ix, iy, k, j, q, ph, pa,
                                                lo, hi, z);
                                ++bad;
                            }
                        }
                    }
                }
    }
    return bad;
}

// adj_lin against the direct per-plane sum, random detector values.
template <typename T>
static long check_lin(const DevGeom &G, long &checked, long (&runs)[4])
{
    long bad = 0;
    double2 scratch[8];
    const double tol = sizeof(T) == 4 ? 2e-5 : 1e-12;
    PlaneRow<T> pl[64];
    for (int q = 0; q <= G.nv; ++q) {
        pl[q].tau = G.tau[q];
        pl[q].tf = T(G.tau[q]);
        pl[q].inv = G.tau[q] != 0.0 ? T(1) / T(G.tau[q]) : T(0);
    }
    T ybuf[66];  // y[-1] .. y[nv], zero at both ends
    unsigned rng = 12345u;
    ybuf[0] = ybuf[G.nv + 1] = T(0);
    for (int q = 0; q < G.nv; ++q) {
        rng = rng * 1664525u + 1013904223u;
        ybuf[q + 1] = T((rng >> 8) * (1.0 / 16777216.0) - 0.25);
    }
    const T *Y = ybuf + 1;
    const double angles[3] = {0.2, 1.9, 3.6};
    for (int v = 0; v < 3; ++v) {
        const double cp = std::cos(angles[v]), sp = std::sin(angles[v]);
        for (int iy = 0; iy < G.ny; ++iy)
            for (int ix = 0; ix < G.nx; ++ix)
                for (int k = 0; k < G.nu; ++k) {
                    Rec<T> R;
                    std::memset(&R, 0, sizeof R);
                    build_record<T>(G, cp, sp, ix, iy, k, R, scratch);
                    if (R.n == 0) continue;
                    const AdjRec<T> A = staged(R);
                    const AdjTab<T> S = adj_tab<T>(A);
                    for (int iz = 0; iz < G.nz; ++iz) {
                        const double za = G.z0 + iz * G.c, zb = G.z0 + (iz + 1) * G.c;
                        int pha, paa, phb, pab;
                        T sum[1];
                        adj_lin<T, 1>(S, A.lc, A.cA, A.bA, A.k4 + (T(za) >= T(0) ? 2 : 0),
                                      A.k4 + (T(zb) >= T(0) ? 2 : 0), pl, za, zb, T(G.v0 / G.dv), G.nv, Y,
                                      0, pha, paa, phb, pab, sum);
                        double ref = (double)A.cA * (double)Y[pab - 1], scale = std::fabs(ref);
                        for (int q = paa; q < pab; ++q) {
                            const double t = (double)A.A * (G.tau[q] * A.lc - za) * ((double)Y[q - 1] - (double)Y[q]);
                            ref += t;
                            scale += std::fabs(t);
                        }
                        ++checked;
                        ++runs[pab - paa < 3 ? pab - paa : 3];
                        if (!(std::fabs((double)sum[0] - ref) <= tol * (scale + 1e-30))) {
                            if (bad < 5)
                                std::printf("lin %s view %d pixel (%d,%d) column %d voxel %d planes %d..%d: %.17g %.17g\n",
                                            sizeof(T) == 4 ? "fp32" : "fp64", v, ix, iy, k, iz, paa, pab,
                                            (double)sum[0], ref);
                            ++bad;
                        }
                    }
                }
    }
    return bad;
}

// A staged slot with a zero header adds exactly zero and reads no table row.
template <typename T>
static long check_zero(const DevGeom &G, long &checked)
{
    long bad = 0;
    PlaneRow<T> pl[64];
    for (int q = 0; q <= G.nv; ++q) {
        pl[q].tau = G.tau[q];
        pl[q].tf = T(G.tau[q]);
        pl[q].inv = G.tau[q] != 0.0 ? T(1) / T(G.tau[q]) : T(0);
    }
    T ybuf[66];
    ybuf[0] = ybuf[G.nv + 1] = T(0);
    for (int q = 0; q < G.nv; ++q) ybuf[q + 1] = T(0.5) + T(q);
    AdjRec<T> Z;
    std::memset(&Z, 0, sizeof Z);
    const T nan = std::nan("");
    for (int i = 0; i < MAXV - 1; ++i) {
        Z.g6[i] = nan;
        for (int c = 0; c < 4; ++c) Z.seg[i][c] = nan;
    }
    const AdjTab<T> S = adj_tab<T>(Z);
    for (int iz = 0; iz < G.nz; ++iz) {
        const double za = G.z0 + iz * G.c, zb = G.z0 + (iz + 1) * G.c;
        T sum[1];
        adj_terms<T, 1>(S, Z.lc, Z.cA, Z.bA, Z.k4 + (T(za) >= T(0) ? 2 : 0), Z.k4 + (T(zb) >= T(0) ? 2 : 0),
                        pl, za, zb, T(G.v0 / G.dv), G.nv, ybuf + 1, 0, sum);
        ++checked;
        if (!(sum[0] == T(0))) {
            if (bad < 5)
                std::printf("zero header %s voxel %d: %.17g\n", sizeof(T) == 4 ? "fp32" : "fp64", iz,
                            (double)sum[0]);
            ++bad;
        }
    }
    return bad;
}

int main()
{
    // an 8 x 8 x 8 grid of unit voxels, source 30 from the centre, detector 60
    // from the source, 12 columns and 8 rows of 1.5
    DevGeom G;
    std::memset(&G, 0, sizeof G);
    G.dim = 3;
    G.nx = G.ny = G.nz = 8;
    G.n_p = 1;
    G.nu = 12;
    G.nv = 8;
    G.a = G.b = G.c = 1.0;
    G.x0 = G.y0 = G.z0 = -4.0;
    G.s = 30.0;
    G.D = 60.0;
    G.du = G.dv = 1.5;
    G.u0 = -0.5 * G.nu * G.du;
    G.v0 = -0.5 * G.nv * G.dv;
    double tau[9];
    for (int q = 0; q <= G.nv; ++q) tau[q] = (G.v0 + q * G.dv) / G.D;
    G.tau = tau;
    long checked = 0, checked_splits = 0;
    const long bad = check<float>(G, checked) + check<double>(G, checked);
    const long bad_splits = check_splits<float>(G, checked_splits) + check_splits<double>(G, checked_splits);
    // the linear parts also on rows of a third of a voxel's projection, so
    // that voxels hold three or more planes (the by-parts form's loop)
    DevGeom F = G;
    F.nv = 24;
    F.dv = 0.5;
    F.v0 = -0.5 * F.nv * F.dv;
    double tauf[25];
    for (int q = 0; q <= F.nv; ++q) tauf[q] = (F.v0 + q * F.dv) / F.D;
    F.tau = tauf;
    long checked_lin = 0, runs[4] = {0, 0, 0, 0};
    const long bad_lin = check_lin<float>(G, checked_lin, runs) + check_lin<double>(G, checked_lin, runs) +
                         check_lin<float>(F, checked_lin, runs) + check_lin<double>(F, checked_lin, runs);
    std::printf("linear parts checked %ld wrong %ld (planes per voxel 0: %ld, 1: %ld, 2: %ld, 3+: %ld)\n",
                checked_lin, bad_lin, runs[0], runs[1], runs[2], runs[3]);
    for (int i = 0; i < 4; ++i)
        if (runs[i] == 0) return 1;
    long checked_zero = 0;
    const long bad_zero = check_zero<float>(G, checked_zero) + check_zero<double>(G, checked_zero) +
                          check_zero<float>(F, checked_zero) + check_zero<double>(F, checked_zero);
    std::printf("zero headers checked %ld nonzero %ld\n", checked_zero, bad_zero);
    if (bad_zero != 0 || checked_zero == 0) return 1;
    std::printf("splits checked %ld wrong %ld\n", checked_splits, bad_splits);
    std::printf("checked %ld mismatches %ld\n", checked, bad + bad_splits + bad_lin);
    return bad == 0 && bad_splits == 0 && bad_lin == 0 && checked > 0 && checked_splits > 0 && checked_lin > 0
               ? 0
               : 1;
}
