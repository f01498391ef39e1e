// Projective-geometry steps on the device, written once for any scalar type
// T with + - * / and the functions g_sqrt / g_asin / g_val below: T = double
// for the forward evaluation, T = Dual (value + one directional derivative)
// for the sources' derivatives with respect to the motion (view setup) and
// for the host check of the adjoint's reverse sweep.
//
// Method steps (arxiv 1806.02637):
//  * meet of two planes -> Pluecker line (Eq. 4);
//  * the antisymmetric 4x4 L_K of that line maps a plane to the point where
//    the line pierces it (Eq. 5; the matrix used is the one that annihilates
//    the two generating planes, i.e. Eq. 5 with the sign of its p entries
//    flipped);
//  * source = meet of two rows of P pierced by the third row (end of
//    "Optimized Algorithm");
//  * epipolar line of plane E in view P: L = meet(E, pi_inf) (Eq. 13),
//    [l]x = P L_K P^T, l = (S12, S20, S01) (Eq. 14).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace ecc {

#define ECC_HD __host__ __device__ __forceinline__

// ---- scalar types ----------------------------------------------------------
struct Dual {
    double v, d;
    ECC_HD Dual() : v(0.0), d(0.0) {}
    ECC_HD Dual(double x) : v(x), d(0.0) {}
    ECC_HD Dual(double x, double dx) : v(x), d(dx) {}
};
ECC_HD Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
ECC_HD Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
ECC_HD Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
ECC_HD Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
ECC_HD Dual operator/(Dual a, Dual b) {
    double inv = 1.0 / b.v;
    double q = a.v * inv;
    return Dual(q, (a.d - q * b.d) * inv);
}
ECC_HD double g_val(double x) { return x; }
ECC_HD double g_val(Dual x) { return x.v; }
ECC_HD double g_sqrt(double x) { return sqrt(x); }
ECC_HD Dual g_sqrt(Dual x) {
    double s = sqrt(x.v);
    return Dual(s, x.d * (0.5 / s));
}
ECC_HD double g_asin(double x) { return asin(x); }
ECC_HD Dual g_asin(Dual x) { return Dual(asin(x.v), x.d / sqrt(1.0 - x.v * x.v)); }

// ---- Eq. 4: meet of planes a and b -> (p, q, r, s, t, u) --------------------
template <class T>
ECC_HD void meet(const T a[4], const T b[4], T L[6]) {
    L[0] = a[2] * b[3] - a[3] * b[2];
    L[1] = a[1] * b[3] - a[3] * b[1];
    L[2] = a[1] * b[2] - a[2] * b[1];
    L[3] = a[0] * b[3] - a[3] * b[0];
    L[4] = a[0] * b[2] - a[2] * b[0];
    L[5] = a[0] * b[1] - a[1] * b[0];
}

// ---- Eq. 5: x = L_K p, L_K = [[0, p, -q, r], [-p, 0, s, -t], [q, -s, 0, u], [-r, t, -u, 0]]
template <class T>
ECC_HD void plucker_apply(const T L[6], const T p[4], T x[4]) {
    x[0] = L[0] * p[1] - L[1] * p[2] + L[2] * p[3];
    x[1] = -(L[0] * p[0]) + L[3] * p[2] - L[4] * p[3];
    x[2] = L[1] * p[0] - L[3] * p[1] + L[5] * p[3];
    x[3] = -(L[2] * p[0]) + L[4] * p[1] - L[5] * p[2];
}

// Source of a 3x4 projection (row-major): rows 0 and 1 meet in a line that
// pierces row 2 at the source; dehomogenised.
template <class T>
ECC_HD void source_position(const T P[12], T C[3]) {
    T L[6], X[4];
    meet(P + 0, P + 4, L);
    plucker_apply(L, P + 8, X);
    C[0] = X[0] / X[3];
    C[1] = X[1] / X[3];
    C[2] = X[2] / X[3];
}

// Eqs. 13-14: image line of plane E in view P.  Only the three entries of
// the skew matrix S = P L_K P^T that carry l are formed:
// S_ij = row_i . (L_K row_j).
template <class T>
ECC_HD void epipolar_line(const T P[12], const T E[4], T l[3]) {
    const T inf[4] = {T(0.0), T(0.0), T(0.0), T(1.0)};
    T L[6];
    meet(E, inf, L);
    T X0[4], X1[4], X2[4];
    plucker_apply(L, P + 0, X0);
    plucker_apply(L, P + 4, X1);
    plucker_apply(L, P + 8, X2);
    // l = (S12, S20, S01)
    l[0] = P[4] * X2[0] + P[5] * X2[1] + P[6] * X2[2] + P[7] * X2[3];
    l[1] = P[8] * X0[0] + P[9] * X0[1] + P[10] * X0[2] + P[11] * X0[3];
    l[2] = P[0] * X1[0] + P[1] * X1[1] + P[2] * X1[2] + P[3] * X1[3];
}

// Rigid motion: R = Rz(rz) Ry(ry) Rx(rx) from the cosines / sines of the
// three angles (the view setup applies P' = P [[R, t], [0, 1]]).
ECC_HD void rotation_zyx(const double c[3], const double s[3], double R[9]) {
    // R = Rz Ry Rx
    const double cx = c[0], sx = s[0], cy = c[1], sy = s[1], cz = c[2], sz = s[2];
    R[0] = cz * cy;
    R[1] = cz * sy * sx - sz * cx;
    R[2] = cz * sy * cx + sz * sx;
    R[3] = sz * cy;
    R[4] = sz * sy * sx + cz * cx;
    R[5] = sz * sy * cx - cz * sx;
    R[6] = -sy;
    R[7] = cy * sx;
    R[8] = cy * cx;
}

// Pencil of epipolar planes about the baseline C_a C_b: unit vectors u1, u2
// with n(kappa) = cos(kappa) u1 + sin(kappa) u2, u2 pointing from the
// baseline towards the isocentre, and kappa_max = asin(min(1, R / h)), h the
// baseline-isocentre distance (planes meeting the object sphere).
template <class T>
ECC_HD void pencil(const T Ca[3], const T Cb[3], double R_mm, T u1[3], T u2[3], T &kappa_max) {
    T b[3] = {Cb[0] - Ca[0], Cb[1] - Ca[1], Cb[2] - Ca[2]};
    T nb = g_sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    T bh[3] = {b[0] / nb, b[1] / nb, b[2] / nb};
    T cab = Ca[0] * bh[0] + Ca[1] * bh[1] + Ca[2] * bh[2];
    T w[3] = {cab * bh[0] - Ca[0], cab * bh[1] - Ca[1], cab * bh[2] - Ca[2]};
    T h = g_sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (g_val(h) < 1e-9) {
        // baseline through the isocentre: every plane of the pencil meets the
        // sphere and kappa spans the half circle; u2 is the part of the z axis
        // (the orbit's rotation axis) perpendicular to the baseline, or of the
        // x axis for a baseline within 60 degrees of z, a threshold no
        // rounding of the sources can tip
        const bool use_z = fabs(g_val(bh[2])) < 0.5;
        T e[3] = {T(use_z ? 0.0 : 1.0), T(0.0), T(use_z ? 1.0 : 0.0)};
        T eb = e[0] * bh[0] + e[1] * bh[1] + e[2] * bh[2];
        T ww[3] = {e[0] - eb * bh[0], e[1] - eb * bh[1], e[2] - eb * bh[2]};
        T nw = g_sqrt(ww[0] * ww[0] + ww[1] * ww[1] + ww[2] * ww[2]);
        u2[0] = ww[0] / nw;
        u2[1] = ww[1] / nw;
        u2[2] = ww[2] / nw;
        kappa_max = T(1.5707963267948966);
    } else {
        u2[0] = w[0] / h;
        u2[1] = w[1] / h;
        u2[2] = w[2] / h;
        T ratio = T(R_mm) / h;
        kappa_max = g_val(ratio) < 1.0 ? g_asin(ratio) : T(1.5707963267948966);
    }
    u1[0] = bh[1] * u2[2] - bh[2] * u2[1];
    u1[1] = bh[2] * u2[0] - bh[0] * u2[2];
    u1[2] = bh[0] * u2[1] - bh[1] * u2[0];
}

// Per-pair line maps: for the epipolar plane with unit normal n through C_a,
// the line in view P' is linear in n (the plane offset drops out of
// meet(E, pi_inf)), so l(kappa) = cos(kappa) l(u1) + sin(kappa) l(u2).
// H = [l(u1) l(u2)] (3x2, column-major in H[0..2], H[3..5]) with the line's
// third coordinate re-expressed about the principal point:
// l3c = l3 + l1 u0 + l2 v0.
template <class T>
ECC_HD void line_map(const T Pm[12], const T Ca[3], const T u1[3], const T u2[3], double u0, double v0, T H[6]) {
    for (int col = 0; col < 2; ++col) {
        const T *n = col == 0 ? u1 : u2;
        T E[4] = {n[0], n[1], n[2], T(0.0) - (n[0] * Ca[0] + n[1] * Ca[1] + n[2] * Ca[2])};
        T l[3];
        epipolar_line(Pm, E, l);
        H[3 * col + 0] = l[0];
        H[3 * col + 1] = l[1];
        H[3 * col + 2] = l[2] + l[0] * T(u0) + l[1] * T(v0);
    }
}

// The prior route to the same lines: the epipolar plane E maps to its image
// line through the pseudo-inverse, l = P^{+T} E (P^+ = P^T (P P^T)^{-1},
// 4x3 row-major); centred about the principal point like line_map.
template <class T>
ECC_HD void line_map_pinv(const double Pp[12], const T Ca[3], const T u1[3], const T u2[3], double u0, double v0,
                          T H[6]) {
    for (int col = 0; col < 2; ++col) {
        const T *n = col == 0 ? u1 : u2;
        T E[4] = {n[0], n[1], n[2], T(0.0) - (n[0] * Ca[0] + n[1] * Ca[1] + n[2] * Ca[2])};
        T l[3];
        for (int i = 0; i < 3; ++i)
            l[i] = T(Pp[i]) * E[0] + T(Pp[3 + i]) * E[1] + T(Pp[6 + i]) * E[2] + T(Pp[9 + i]) * E[3];
        H[3 * col + 0] = l[0];
        H[3 * col + 1] = l[1];
        H[3 * col + 2] = l[2] + l[0] * T(u0) + l[1] * T(v0);
    }
}

}  // namespace ecc
