// Detector-bounded plane range: the arc of a pair's pencil of epipolar
// planes whose lines meet both detectors (the reading of Eq. 15's plane
// count in which the sampled range itself is bounded by the detectors).  Host and device code, FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "projective.hpp"

namespace ecc {

// Arc of plane angles around kappa = 0 whose lines meet the closed detector
// rectangle |x| <= hw, |y| <= hh (about the principal point), from the
// centred basis lines H: the line of the plane at kappa is
// cos(kappa) H[0..2] + sin(kappa) H[3..5].  At corner c the line's value is
// A_c cos(kappa) + B_c sin(kappa), whose sign changes only at
// kappa = atan2(-A_c, B_c) mod pi; between consecutive such zeros the
// meets-the-rectangle decision (corner values not all of one strict sign) is
// constant, so the arc ends at the first zero, walking away from 0 in each
// direction, past which an interval misses.  Returns kArcNone when the plane
// at 0 misses, kArcFull with [-pi/2, pi/2] when every plane meets the
// rectangle, else kArcPart with the arc (shorter than pi, containing 0).
// c_lo / c_hi (optional) receive the corner whose zero angle each end is
// (-1 for a fixed end).  Corner c is (c & 2 ? +hw : -hw, c & 1 ? +hh : -hh).
enum ArcKind { kArcNone = 0, kArcPart = 1, kArcFull = 2 };
ECC_HD ArcKind view_arc(const double H[6], double hw, double hh, double &lo, double &hi, int *c_lo = nullptr,
                        int *c_hi = nullptr) {
    constexpr double kPi = 3.141592653589793;
    double A[4], Bc[4], z[4];
    int zc[4] = {0, 1, 2, 3};
    for (int c = 0; c < 4; ++c) {
        const double x = (c & 2) ? hw : -hw, y = (c & 1) ? hh : -hh;
        A[c] = H[0] * x + H[1] * y + H[2];
        Bc[c] = H[3] * x + H[4] * y + H[5];
    }
    auto meets = [&](double k) {
        double sn, cs;
        sincos(k, &sn, &cs);
        double mn = A[0] * cs + Bc[0] * sn, mx = mn;
        for (int c = 1; c < 4; ++c) {
            const double v = A[c] * cs + Bc[c] * sn;
            mn = fmin(mn, v);
            mx = fmax(mx, v);
        }
        return mn <= 0.0 && mx >= 0.0;
    };
    if (!meets(0.0)) return kArcNone;
    for (int c = 0; c < 4; ++c) {
        double w = atan2(-A[c], Bc[c]) + 0.5 * kPi;  // [-pi/2, 3pi/2]
        if (w >= kPi) w -= kPi;
        if (w < 0.0) w += kPi;
        z[c] = w - 0.5 * kPi;  // [-pi/2, pi/2)
    }
    // ascending (angle, corner) order (four-element sorting network)
    auto order = [&](int i, int j) {
        if (z[j] < z[i] || (z[j] == z[i] && zc[j] < zc[i])) {
            const double t = z[i];
            z[i] = z[j];
            z[j] = t;
            const int u = zc[i];
            zc[i] = zc[j];
            zc[j] = u;
        }
    };
    order(0, 1);
    order(2, 3);
    order(0, 2);
    order(1, 3);
    order(1, 2);
    int n_neg = 0, n_pos = 0;  // zeros below 0, zeros at or below 0
    for (int c = 0; c < 4; ++c) {
        n_neg += z[c] < 0.0;
        n_pos += z[c] <= 0.0;
    }
    // upward: the zeros above 0, then those at or below 0 shifted by +pi
    bool closed = false;
    double prev = 0.0;
    int src = -1;
    for (int j = 0; j < 4 && !closed; ++j) {
        const int i = n_pos + j;
        const double k = i < 4 ? z[i] : z[i - 4] + kPi;
        if (!meets(0.5 * (prev + k))) {
            closed = true;
        } else {
            prev = k;
            src = zc[i < 4 ? i : i - 4];
        }
    }
    if (!closed) {
        lo = -0.5 * kPi;
        hi = 0.5 * kPi;
        if (c_lo) *c_lo = -1;
        if (c_hi) *c_hi = -1;
        return kArcFull;
    }
    hi = prev;
    if (c_hi) *c_hi = src;
    // downward: the zeros below 0, then those at or above 0 shifted by -pi
    prev = 0.0;
    src = -1;
    for (int j = 0; j < 4; ++j) {
        const int i = n_neg - 1 - j;
        const double k = i >= 0 ? z[i] : z[i + 4] - kPi;
        if (!meets(0.5 * (prev + k))) break;
        prev = k;
        src = zc[i >= 0 ? i : i + 4];
    }
    lo = prev;
    if (c_lo) *c_lo = src;
    return kArcPart;
}

// Which view fixes each end of a pair's arc, and through which corner.
// view: -1 fixed end (+-pi/2), 0 view a, 1 view b, 2 both (the two views'
// ends agree within kArcTie rad: a circular orbit without motion makes
// them equal, and the end is then a kink between the two; its derivative is
// taken as the mean of the two, the central-difference value).
struct ArcEnd {
    int view, corner_a, corner_b;
};
constexpr double kArcTie = 1e-9;

// The pair's arc from the two views' arcs: a view that sees every plane
// leaves the other's arc whole (it may reach past +-pi/2); two partial arcs,
// each shorter than pi and containing 0, meet around 0 in [max lows, min
// highs].  Returns false when either view's arc is empty.
ECC_HD bool pair_arc(const double Ha[6], const double Hb[6], double hw, double hh, double &lo, double &hi,
                     ArcEnd *end_lo = nullptr, ArcEnd *end_hi = nullptr) {
    double la, ha, lb, hb;
    int cla, cha, clb, chb;
    const ArcKind ka = view_arc(Ha, hw, hh, la, ha, &cla, &cha);
    if (ka == kArcNone) return false;
    const ArcKind kb = view_arc(Hb, hw, hh, lb, hb, &clb, &chb);
    if (kb == kArcNone) return false;
    int v_lo, v_hi;
    if (ka == kArcFull && kb == kArcFull) {
        v_lo = v_hi = -1;
    } else if (ka == kArcFull) {
        v_lo = v_hi = 1;
    } else if (kb == kArcFull) {
        v_lo = v_hi = 0;
    } else {
        v_lo = fabs(la - lb) <= kArcTie ? 2 : (la >= lb ? 0 : 1);
        v_hi = fabs(ha - hb) <= kArcTie ? 2 : (ha <= hb ? 0 : 1);
    }
    lo = v_lo == 1 ? lb : v_lo == 0 ? la : v_lo == 2 ? fmax(la, lb) : -0.5 * 3.141592653589793;
    hi = v_hi == 1 ? hb : v_hi == 0 ? ha : v_hi == 2 ? fmin(ha, hb) : 0.5 * 3.141592653589793;
    if (end_lo) *end_lo = ArcEnd{v_lo, cla, clb};
    if (end_hi) *end_hi = ArcEnd{v_hi, cha, chb};
    return true;
}

}  // namespace ecc
