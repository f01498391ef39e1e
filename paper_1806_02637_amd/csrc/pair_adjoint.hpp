// Reverse sweep of a pair's geometry for the adjoint (arxiv 1806.02637,
// Eqs. 4, 5, 13, 14 and the pencil of "Epipolar Consistency"; host and
// device code, FP64): the 14 per-pair sensitivities of the cost -- dE/dH_a,
// dE/dH_b for the two scaled line maps and the sampled arc's one or two
// ends -- taken back to each view's M = P'[:, 0:3] and source, then
// contracted with the 12 motion parameters' dP'/dtheta and dC/dtheta.
#pragma once

#include <math.h>

#include "arc.hpp"
#include "projective.hpp"

namespace ecc {

constexpr int kSens = 14;  // per-pair sensitivities: dE/dHa [6], dE/dHb [6], two for the arc

// Reverse sweep of a detector arc's end, the zero angle atan2(-A, B) of
// corner c = (x, y, 1) with A = H_c . c and B = H_s . c the values of the
// (unscaled) basis lines there: d end = (A dB - B dA) / (A^2 + B^2), so
// d end / d H_c = -B c / r2 and d end / d H_s = A c / r2; adds w times those
// to Hbar.
ECC_HD void arc_end_adjoint(const double H[6], int corner, double hw, double hh, double w, double Hbar[6]) {
    const double x = (corner & 2) ? hw : -hw, y = (corner & 1) ? hh : -hh;
    const double A = H[0] * x + H[1] * y + H[2], B = H[3] * x + H[4] * y + H[5];
    const double r2 = A * A + B * B;
    if (!(r2 > 0.0)) return;
    const double sa = -B * w / r2, sb = A * w / r2;
    Hbar[0] += sa * x;
    Hbar[1] += sa * y;
    Hbar[2] += sa;
    Hbar[3] += sb * x;
    Hbar[4] += sb * y;
    Hbar[5] += sb;
}

ECC_HD void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
ECC_HD double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Reverse sweep of one view's line map.  Meeting a plane with the plane at
// infinity drops its offset, and Eqs. 4, 5, 13, 14 reduce to the cofactor
// rows of M = P'[:, 0:3] (rows m_k) applied to the plane's normal n:
// l = (n . (m1 x m2), n . (m2 x m0), n . (m0 x m1)), then re-centred about
// the principal point (l3 + u0 l1 + v0 l2).  H = [l(u1), l(u2)].  Given Hbar =
// dE/dH, adds dE/du1 and dE/du2 to nbar1, nbar2 and writes dE/dM (by rows):
// with T_k = sum over columns of w_col[k] n_col (w = the re-centring's
// transpose applied to Hbar's column), E = sum_k T_k . (m_{k+1} x m_{k+2}) and
// dE/dm_j = m_{j+1} x T_{j-1} + T_{j+1} x m_{j+2} (indices mod 3).
ECC_HD void line_map_adjoint(const double P[12], double u0, double v0, const double u1[3], const double u2[3],
                                 const double Hbar[6], double nbar1[3], double nbar2[3], double Mbar[3][3]) {
    const double m[3][3] = {{P[0], P[1], P[2]}, {P[4], P[5], P[6]}, {P[8], P[9], P[10]}};
    double c[3][3];
    for (int k = 0; k < 3; ++k) cross3(m[(k + 1) % 3], m[(k + 2) % 3], c[k]);
    double T[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int col = 0; col < 2; ++col) {
        const double *n = col == 0 ? u1 : u2;
        double *nb = col == 0 ? nbar1 : nbar2;
        const double g2 = Hbar[3 * col + 2];
        const double w[3] = {Hbar[3 * col] + u0 * g2, Hbar[3 * col + 1] + v0 * g2, g2};
        for (int i = 0; i < 3; ++i) nb[i] += w[0] * c[0][i] + w[1] * c[1][i] + w[2] * c[2][i];
        for (int k = 0; k < 3; ++k)
            for (int i = 0; i < 3; ++i) T[k][i] += w[k] * n[i];
    }
    for (int j = 0; j < 3; ++j) {
        double x[3], y[3];
        cross3(m[(j + 1) % 3], T[(j + 2) % 3], x);
        cross3(T[(j + 1) % 3], m[(j + 2) % 3], y);
        for (int i = 0; i < 3; ++i) Mbar[j][i] = x[i] + y[i];
    }
}

// Reverse sweep of the pencil (the same steps and branches as pencil()):
// given dE/du1, dE/du2 and dE/dkappa_max, adds dE/dC_a and dE/dC_b.  With
// b = C_b - C_a, bh = b / |b|, w = (C_a . bh) bh - C_a, h = |w|:
//   u1 = bh x u2;   u2 = w / h, kappa_max = asin(R / h) while R < h (else
//   pi/2); through the isocentre (h < 1e-9) u2 = the unit part of a fixed
//   axis e perpendicular to bh, kappa_max = pi/2.
ECC_HD void pencil_adjoint(const double Ca[3], const double Cb[3], double R_mm, const double u1bar[3],
                               const double u2bar_in[3], double kbar, double Cabar[3], double Cbbar[3]) {
    const double b[3] = {Cb[0] - Ca[0], Cb[1] - Ca[1], Cb[2] - Ca[2]};
    const double nb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    const double bh[3] = {b[0] / nb, b[1] / nb, b[2] / nb};
    const double cab = Ca[0] * bh[0] + Ca[1] * bh[1] + Ca[2] * bh[2];
    const double w[3] = {cab * bh[0] - Ca[0], cab * bh[1] - Ca[1], cab * bh[2] - Ca[2]};
    const double h = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double bhbar[3], u2bar[3], u2[3];
    if (h < 1e-9) {
        const bool use_z = fabs(bh[2]) < 0.5;
        const double e[3] = {use_z ? 0.0 : 1.0, 0.0, use_z ? 1.0 : 0.0};
        const double eb = e[0] * bh[0] + e[1] * bh[1] + e[2] * bh[2];
        const double ww[3] = {e[0] - eb * bh[0], e[1] - eb * bh[1], e[2] - eb * bh[2]};
        const double nw = sqrt(ww[0] * ww[0] + ww[1] * ww[1] + ww[2] * ww[2]);
        for (int i = 0; i < 3; ++i) u2[i] = ww[i] / nw;
        // u1 = bh x u2
        cross3(u2, u1bar, bhbar);
        double t[3];
        cross3(u1bar, bh, t);
        for (int i = 0; i < 3; ++i) u2bar[i] = u2bar_in[i] + t[i];
        // u2 = ww / |ww|, ww = e - (e . bh) bh
        const double pu = dot3(u2bar, u2);
        double wwbar[3];
        for (int i = 0; i < 3; ++i) wwbar[i] = (u2bar[i] - pu * u2[i]) / nw;
        const double ebbar = -dot3(wwbar, bh);
        for (int i = 0; i < 3; ++i) bhbar[i] += -eb * wwbar[i] + ebbar * e[i];
    } else {
        for (int i = 0; i < 3; ++i) u2[i] = w[i] / h;
        cross3(u2, u1bar, bhbar);
        double t[3];
        cross3(u1bar, bh, t);
        for (int i = 0; i < 3; ++i) u2bar[i] = u2bar_in[i] + t[i];
        // u2 = w / h and kappa_max = asin(R / h): both through w
        const double pu = dot3(u2bar, u2);
        double wbar[3];
        for (int i = 0; i < 3; ++i) wbar[i] = (u2bar[i] - pu * u2[i]) / h;
        const double ratio = R_mm / h;
        if (ratio < 1.0) {
            const double hbar = kbar * (-ratio / h) / sqrt(1.0 - ratio * ratio);
            for (int i = 0; i < 3; ++i) wbar[i] += hbar * u2[i];
        }
        // w = cab bh - C_a, cab = C_a . bh
        const double cabbar = dot3(wbar, bh);
        for (int i = 0; i < 3; ++i) {
            bhbar[i] += cab * wbar[i] + cabbar * Ca[i];
            Cabar[i] += cabbar * bh[i] - wbar[i];
        }
    }
    // bh = b / |b|, b = C_b - C_a
    const double pb = dot3(bhbar, bh);
    for (int i = 0; i < 3; ++i) {
        const double bbar = (bhbar[i] - pb * bh[i]) / nb;
        Cbbar[i] += bbar;
        Cabar[i] -= bbar;
    }
}

// The 12 directional derivatives of the pair's cost term (6 motion
// parameters of view a, then 6 of view b) given its 14 sensitivities g: the
// geometry is formed again as pair_setup forms it (pencil, line maps, the
// power-of-two exponents of the scaled maps, the detector arc's ends), then
// swept back once.
ECC_HD void pair_gradient(const double Pa[12], const double Ca[3], double u0a, double v0a, const double Pb[12],
                          const double Cb[3], double u0b, double v0b, const double dPa[6][12], const double dCa[6][3],
                          const double dPb[6][12], const double dCb[6][3], double R_mm, bool kappa_detector, double hw,
                          double hh, const double g[kSens], double out[12]) {
    double u1[3], u2[3], km;
    pencil(Ca, Cb, R_mm, u1, u2, km);
    double Ha[6], Hb[6];
    line_map(Pa, Ca, u1, u2, u0a, v0a, Ha);
    line_map(Pb, Ca, u1, u2, u0b, v0b, Hb);
    // the forward pass scaled each map by an exact power of two (the same
    // exponent follows from the values here); the sensitivities were taken
    // with respect to the scaled maps
    double ma = 0.0, mb = 0.0;
    for (int i = 0; i < 6; ++i) {
        ma = fmax(ma, fabs(Ha[i]));
        mb = fmax(mb, fabs(Hb[i]));
    }
    const int ea = ma > 0.0 ? ilogb(ma) : 0, eb = mb > 0.0 ? ilogb(mb) : 0;
    double Hbar_a[6], Hbar_b[6];
    for (int i = 0; i < 6; ++i) {
        Hbar_a[i] = ldexp(g[i], -ea);
        Hbar_b[i] = ldexp(g[6 + i], -eb);
    }
    double kbar = 0.0;
    if (kappa_detector) {
        // an end moves with the zero angle of the corner behind it, the mean
        // of both views' corners at a tie, not at all when fixed; an empty
        // arc has zero sensitivities (no plane counts)
        double lo, hi;
        ArcEnd ends[2];
        if (pair_arc(Ha, Hb, hw, hh, lo, hi, &ends[0], &ends[1])) {
            for (int k = 0; k < 2; ++k) {
                const ArcEnd &e = ends[k];
                const double w = g[12 + k];
                const double wa = e.view == 0 ? w : (e.view == 2 ? 0.5 * w : 0.0);
                const double wb = e.view == 1 ? w : (e.view == 2 ? 0.5 * w : 0.0);
                if (wa != 0.0 && e.corner_a >= 0) arc_end_adjoint(Ha, e.corner_a, hw, hh, wa, Hbar_a);
                if (wb != 0.0 && e.corner_b >= 0) arc_end_adjoint(Hb, e.corner_b, hw, hh, wb, Hbar_b);
            }
        }
    } else {
        kbar = g[12];
    }
    double n1bar[3] = {0.0, 0.0, 0.0}, n2bar[3] = {0.0, 0.0, 0.0}, Mbar_a[3][3], Mbar_b[3][3];
    line_map_adjoint(Pa, u0a, v0a, u1, u2, Hbar_a, n1bar, n2bar, Mbar_a);
    line_map_adjoint(Pb, u0b, v0b, u1, u2, Hbar_b, n1bar, n2bar, Mbar_b);
    double Cabar[3] = {0.0, 0.0, 0.0}, Cbbar[3] = {0.0, 0.0, 0.0};
    pencil_adjoint(Ca, Cb, R_mm, n1bar, n2bar, kbar, Cabar, Cbbar);
    for (int q = 0; q < 6; ++q) {
        double sa = 0.0, sb = 0.0;
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) {
                sa += Mbar_a[j][i] * dPa[q][4 * j + i];
                sb += Mbar_b[j][i] * dPb[q][4 * j + i];
            }
        for (int i = 0; i < 3; ++i) {
            sa += Cabar[i] * dCa[q][i];
            sb += Cbbar[i] * dCb[q][i];
        }
        out[q] = sa;
        out[6 + q] = sb;
    }
}

}  // namespace ecc
