// Host check of the adjoint's reverse sweep over a pair's geometry
// (pair_gradient in pair_adjoint.hpp) against forward-mode dual numbers
// through the same pencil() / line_map() templates, one motion parameter at a
// time: for arbitrary tangents dP, dC of the two views and arbitrary
// sensitivities g, the 12 directional derivatives must agree to FP64
// rounding.  Cases: C-arm-like pairs with the object-sphere range and with
// the detector-bounded range, a baseline through the isocentre, and a
// sphere larger than the baseline's distance (kappa_max = pi/2, fixed).
#include <cstdio>
#include <cstdlib>
#include <random>

#include "../paper_1806_02637_amd/csrc/pair_adjoint.hpp"

using namespace ecc;

namespace {

std::mt19937_64 rng(12345);
double unif(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }

// P = K [R | -R C] for a source at angle phi on a circle of radius D about z,
// looking at the isocentre, detector distance f (pixels), principal point
// (u0, v0); a small random tilt keeps the case generic.
void view(double phi, double D, double f, double u0, double v0, double P[12], double C[3]) {
    C[0] = D * cos(phi) + unif(-5, 5);
    C[1] = D * sin(phi) + unif(-5, 5);
    C[2] = unif(-5, 5);
    double z[3] = {-C[0], -C[1], -C[2]};
    const double nz = sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
    for (double &v : z) v /= nz;
    double up[3] = {unif(-0.05, 0.05), unif(-0.05, 0.05), 1.0};
    double x[3], y[3];
    cross3(up, z, x);
    const double nx = sqrt(dot3(x, x));
    for (double &v : x) v /= nx;
    cross3(z, x, y);
    const double R[3][3] = {{x[0], x[1], x[2]}, {y[0], y[1], y[2]}, {z[0], z[1], z[2]}};
    const double K[3][3] = {{f, 0, u0}, {0, f, v0}, {0, 0, 1}};
    for (int i = 0; i < 3; ++i) {
        double t = 0.0;
        for (int j = 0; j < 3; ++j) {
            double kr = 0.0;
            for (int k = 0; k < 3; ++k) kr += K[i][k] * R[k][j];
            P[4 * i + j] = kr;
            t -= kr * C[j];
        }
        P[4 * i + 3] = t;
    }
}

// Forward mode, one parameter: the directional derivative of
// sum g . (scaled Ha, scaled Hb) + arc term, with the same readings as
// pair_gradient (the reference it is checked against).
double forward_dir(const double Pa[12], const double Ca[3], double u0a, double v0a, const double Pb[12],
                   const double Cb[3], double u0b, double v0b, const double dP[12], const double dC[3], bool on_a,
                   double R, bool det, double hw, double hh, const double g[kSens]) {
    Dual DPa[12], DPb[12], DCa[3], DCb[3];
    for (int e = 0; e < 12; ++e) {
        DPa[e] = Dual(Pa[e], on_a ? dP[e] : 0.0);
        DPb[e] = Dual(Pb[e], on_a ? 0.0 : dP[e]);
    }
    for (int e = 0; e < 3; ++e) {
        DCa[e] = Dual(Ca[e], on_a ? dC[e] : 0.0);
        DCb[e] = Dual(Cb[e], on_a ? 0.0 : dC[e]);
    }
    Dual u1[3], u2[3], km;
    pencil(DCa, DCb, R, u1, u2, km);
    Dual Ha[6], Hb[6];
    line_map(DPa, DCa, u1, u2, u0a, v0a, Ha);
    line_map(DPb, DCa, u1, u2, u0b, v0b, Hb);
    double ma = 0.0, mb = 0.0;
    for (int i = 0; i < 6; ++i) {
        ma = fmax(ma, fabs(Ha[i].v));
        mb = fmax(mb, fabs(Hb[i].v));
    }
    const int ea = ma > 0.0 ? ilogb(ma) : 0, eb = mb > 0.0 ? ilogb(mb) : 0;
    double ga = 0.0, gb = 0.0;
    for (int i = 0; i < 6; ++i) {
        ga += g[i] * Ha[i].d;
        gb += g[6 + i] * Hb[i].d;
    }
    double arc = 0.0;
    if (det) {
        double va[6], vb[6], lo, hi;
        for (int i = 0; i < 6; ++i) {
            va[i] = Ha[i].v;
            vb[i] = Hb[i].v;
        }
        ArcEnd ends[2];
        auto tangent = [&](const Dual H[6], int corner) {
            const double x = (corner & 2) ? hw : -hw, y = (corner & 1) ? hh : -hh;
            const double A = H[0].v * x + H[1].v * y + H[2].v, B = H[3].v * x + H[4].v * y + H[5].v;
            const double dA = H[0].d * x + H[1].d * y + H[2].d, dB = H[3].d * x + H[4].d * y + H[5].d;
            const double r2 = A * A + B * B;
            return r2 > 0.0 ? (A * dB - B * dA) / r2 : 0.0;
        };
        if (pair_arc(va, vb, hw, hh, lo, hi, &ends[0], &ends[1])) {
            for (int k = 0; k < 2; ++k) {
                const ArcEnd &e = ends[k];
                const double ta = e.corner_a >= 0 ? tangent(Ha, e.corner_a) : 0.0;
                const double tb = e.corner_b >= 0 ? tangent(Hb, e.corner_b) : 0.0;
                arc += g[12 + k] * (e.view == 0 ? ta : e.view == 1 ? tb : e.view == 2 ? 0.5 * (ta + tb) : 0.0);
            }
        }
    } else {
        arc = g[12] * km.d;
    }
    return ldexp(ga, -ea) + ldexp(gb, -eb) + arc;
}

int check(const char *name, double phi_a, double phi_b, double R, bool det, int trials, int min_corner_ends = 0) {
    int bad = 0, corner_ends = 0;
    double worst = 0.0;
    for (int t = 0; t < trials; ++t) {
        double Pa[12], Pb[12], Ca[3], Cb[3];
        const double f = 1200.0 / 0.308, u0 = 619.5, v0 = 479.5;
        view(phi_a + unif(-0.01, 0.01), 750.0, f, u0, v0, Pa, Ca);
        view(phi_b + unif(-0.01, 0.01), 750.0, f, u0, v0, Pb, Cb);
        if (phi_b - phi_a == M_PI) {  // exactly opposed sources: the baseline passes through the isocentre
            for (int i = 0; i < 3; ++i) Cb[i] = -Ca[i];
        }
        double dPa[6][12], dPb[6][12], dCa[6][3], dCb[6][3], g[kSens];
        for (int q = 0; q < 6; ++q) {
            for (int e = 0; e < 12; ++e) {
                dPa[q][e] = unif(-1, 1) * fabs(Pa[e]) * 1e-2 + unif(-1, 1);
                dPb[q][e] = unif(-1, 1) * fabs(Pb[e]) * 1e-2 + unif(-1, 1);
            }
            for (int e = 0; e < 3; ++e) {
                dCa[q][e] = unif(-1, 1);
                dCb[q][e] = unif(-1, 1);
            }
        }
        for (double &v : g) v = unif(-1, 1);
        if (det) {  // how many arc ends move with a corner (the arc-end sweep is exercised)
            double u1[3], u2[3], km, Ha[6], Hb[6], lo, hi;
            pencil(Ca, Cb, R, u1, u2, km);
            line_map(Pa, Ca, u1, u2, u0, v0, Ha);
            line_map(Pb, Ca, u1, u2, u0, v0, Hb);
            ArcEnd ends[2];
            if (pair_arc(Ha, Hb, 620.0, 480.0, lo, hi, &ends[0], &ends[1]))
                for (const ArcEnd &e : ends) corner_ends += (e.view >= 0 && (e.corner_a >= 0 || e.corner_b >= 0));
        }
        double out[12];
        pair_gradient(Pa, Ca, u0, v0, Pb, Cb, u0, v0, dPa, dCa, dPb, dCb, R, det, 620.0, 480.0, g, out);
        double ref[12], scale = 0.0;
        for (int d = 0; d < 12; ++d) {
            const bool on_a = d < 6;
            const int q = on_a ? d : d - 6;
            ref[d] = forward_dir(Pa, Ca, u0, v0, Pb, Cb, u0, v0, on_a ? dPa[q] : dPb[q], on_a ? dCa[q] : dCb[q], on_a,
                                 R, det, 620.0, 480.0, g);
            scale = fmax(scale, fabs(ref[d]));
        }
        for (int d = 0; d < 12; ++d) {
            const double err = fabs(out[d] - ref[d]) / (scale > 0.0 ? scale : 1.0);
            worst = fmax(worst, err);
            if (!(err <= 1e-9)) {
                if (bad < 5) printf("%s trial %d dir %d: reverse %.17g forward %.17g\n", name, t, d, out[d], ref[d]);
                ++bad;
            }
        }
    }
    printf("%-34s worst |reverse - forward| / max|forward| = %.2e", name, worst);
    if (det) printf(", arc ends at a corner: %d of %d", corner_ends, 2 * trials);
    printf("\n");
    if (corner_ends < min_corner_ends) {
        printf("%s: only %d arc ends at a corner (want %d)\n", name, corner_ends, min_corner_ends);
        ++bad;
    }
    return bad;
}

}  // namespace

int main() {
    int bad = 0;
    bad += check("adjacent views, object sphere", 0.3, 0.3 + 0.0127, 96.0, false, 200);
    bad += check("90 degrees apart, object sphere", 1.0, 1.0 + M_PI / 2, 96.0, false, 200);
    bad += check("near-opposed, object sphere", 0.2, 0.2 + M_PI - 0.02, 96.0, false, 200);
    bad += check("sphere wider than h (kappa fixed)", 0.5, 0.5 + 2.0, 900.0, false, 100);
    bad += check("adjacent views, detector range", 0.3, 0.3 + 0.0127, 96.0, true, 200, 200);
    bad += check("60 degrees apart, detector range", 2.0, 2.0 + M_PI / 3, 96.0, true, 200, 200);
    bad += check("opposed, detector range", 0.7, 0.7 + M_PI - 0.05, 96.0, true, 200);
    bad += check("baseline through the isocentre", 1.3, 1.3 + M_PI, 96.0, false, 50);
    if (bad) {
        printf("%d mismatches\n", bad);
        return 1;
    }
    printf("passed\n");
    return 0;
}
