// Per-plane work of the consistency kernels: epipolar line from the pair's
// line map, its sinogram coordinates (alpha, t), the hit test and the
// weighted bilinear lookup of S_lam (Eq. 1 indexed by the line, Sec.
// "Epipolar Consistency"), in geometry precision G (float or double).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ecc_internal.hpp"
#include "poly_coeffs.hpp"

namespace ecc {

// Per-plane constants of one view pair, built in FP64 and kept in LDS.
//   ha, hb: line maps of views a and b, l = H (cos kappa, sin kappa) with the
//           line's offset about the principal point (H column-major);
//   k0, dk: kappa_k = k0 + k dk; rc, rs: cos / sin of 64 dk (one wave step);
//   inv_f2a/b: 1 / f^2 of the views (Grangeat weight 1 + t^2 / f^2);
//   sa, sb: storage scales of the two views' sinograms; va, vb: view ids.
template <class G>
struct PairConst {
    G ha[6], hb[6];
    G k0, dk, rc, rs;
    float inv_f2a, inv_f2b, sa, sb;
    int va, vb;
};

// Wave-uniform copy of a pair's constants (read from LDS by every lane) into
// scalar registers.
__device__ __forceinline__ float uniform(float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); }
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ double uniform(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <class G>
__device__ __forceinline__ PairConst<G> uniform(const PairConst<G> &p) {
    PairConst<G> u;
    for (int i = 0; i < 6; ++i) {
        u.ha[i] = uniform(p.ha[i]);
        u.hb[i] = uniform(p.hb[i]);
    }
    u.k0 = uniform(p.k0);
    u.dk = uniform(p.dk);
    u.rc = uniform(p.rc);
    u.rs = uniform(p.rs);
    u.inv_f2a = uniform(p.inv_f2a);
    u.inv_f2b = uniform(p.inv_f2b);
    u.sa = uniform(p.sa);
    u.sb = uniform(p.sb);
    u.va = uniform(p.va);
    u.vb = uniform(p.vb);
    return u;
}

// ---- storage types: one load returns the four taps of a bilinear cell ----
struct Taps {
    float s00, s10, s01, s11;  // S[m][k], S[m+1][k], S[m][k+1], S[m+1][k+1]
};

typedef float f32x4_a8 __attribute__((ext_vector_type(4), aligned(8)));
typedef uint32_t u32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));

// Each storage type loads a cell's taps as raw words (fetch) and converts
// them (unpack) separately, so that a kernel can keep the raw words of a
// plane in flight and convert them only when it combines the plane.
struct TapF32 {
    static constexpr bool kScaled = false;
    static constexpr int kAsinTerms = kAsinTermsF32;
    using Raw = f32x4_a8;
    float lo, hi;
    static __device__ __forceinline__ Raw fetch(const TapF32 *p) { return *(const f32x4_a8 *)p; }
    static __device__ __forceinline__ Taps unpack(const Raw &v) { return Taps{v.x, v.y, v.z, v.w}; }
    static __device__ __forceinline__ Taps load(const TapF32 *p) { return unpack(fetch(p)); }
};

struct TapBF16 {
    static constexpr bool kScaled = false;
    static constexpr int kAsinTerms = kAsinTerms16;
    using Raw = u32x2_a4;
    uint32_t bits;
    static __device__ __forceinline__ Raw fetch(const TapBF16 *p) { return *(const u32x2_a4 *)p; }
    static __device__ __forceinline__ Taps unpack(const Raw &v) {
        return Taps{__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xFFFF0000u), __uint_as_float(v.y << 16),
                    __uint_as_float(v.y & 0xFFFF0000u)};
    }
    static __device__ __forceinline__ Taps load(const TapBF16 *p) { return unpack(fetch(p)); }
};

struct TapF16 {
    static constexpr bool kScaled = true;  // per-view power-of-two storage scale
    static constexpr int kAsinTerms = kAsinTerms16;
    using Raw = u32x2_a4;
    uint32_t bits;
    static __device__ __forceinline__ float h2f(uint32_t h) {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
    }
    static __device__ __forceinline__ Raw fetch(const TapF16 *p) { return *(const u32x2_a4 *)p; }
    static __device__ __forceinline__ Taps unpack(const Raw &v) {
        return Taps{h2f(v.x & 0xFFFFu), h2f(v.x >> 16), h2f(v.y & 0xFFFFu), h2f(v.y >> 16)};
    }
    static __device__ __forceinline__ Taps load(const TapF16 *p) { return unpack(fetch(p)); }
};

// ---- precision-generic helpers ----------------------------------------------
// FP32: fitted polynomials (poly_coeffs.hpp) -- the plane angle only selects
// which plane of the pencil is sampled, identically for both views, and the
// line angle enters the lookup through an FP32 fraction anyway.  FP64: the
// library sincos (once per lane and pair), a 13-term fitted atan (3.5e-12
// rad) of min / max by the hardware reciprocal with two Newton steps, and a
// Newton-refined reciprocal square root.
__device__ __forceinline__ void g_sincos(float x, float *s, float *c) {
    // |x| <= pi/2 (plane angles of the pencil)
    const float x2 = x * x;
    float ps = kSin[5], pc = kCos[6];
#pragma unroll
    for (int i = 4; i >= 0; --i) ps = fmaf(ps, x2, kSin[i]);
#pragma unroll
    for (int i = 5; i >= 0; --i) pc = fmaf(pc, x2, kCos[i]);
    *s = ps * x;
    *c = pc;
}
__device__ __forceinline__ void g_sincos(double x, double *s, double *c) { sincos(x, s, c); }

// Angle in [0, pi] of a line's normal (x, y), y >= 0, given |x|, |y|,
// 1 / |(x, y)| and whether x < 0.  The base angle is the one of the smaller
// component, theta = atan(min / max) in [0, pi/4]; then
//   swap (|y| > |x|): pi/2 - theta;  xneg: pi - (...)
// combined as off + sgn theta with off in {0, pi/2, pi} and sgn = +-1.
// FP32 takes theta = asin(min / |(x, y)|) by a fitted polynomial of NT terms
// (no reciprocal: the inverse norm is shared with t) whose coefficients and
// offsets come scaled by 1 / dalpha, so the result is already in sinogram
// rows; FP64 takes atan(min / max) in radians.
template <int NT>
__device__ __forceinline__ float g_angle_rows(float ax, float ay, float rinv, bool xneg, const EvalConsts &ec) {
    const bool swap = ay > ax;
    const float s = (swap ? ax : ay) * rinv;
    const float s2 = s * s;
    float p = ec.asin_rows[NT - 1];
#pragma unroll
    for (int i = NT - 2; i >= 0; --i) p = fmaf(p, s2, ec.asin_rows[i]);
    const float off = swap ? ec.rows_half_pi : (xneg ? ec.rows_pi : 0.0f);
    return fmaf(swap != xneg ? -s : s, p, off);
}
// The same angle for a line steeper than 45 degrees (|y| > |x|) from the
// signed cosine u = x / |(x, y)|: pi/2 - asin(u).  |u| and u^2 round as s
// and s^2 above and -u carries the sign the general form selects, so the two
// give the same bits on such lines.
template <int NT>
__device__ __forceinline__ float g_angle_rows_steep(float u, const EvalConsts &ec) {
    const float u2 = u * u;
    float p = ec.asin_rows[NT - 1];
#pragma unroll
    for (int i = NT - 2; i >= 0; --i) p = fmaf(p, u2, ec.asin_rows[i]);
    return fmaf(-u, p, ec.rows_half_pi);
}
__device__ __forceinline__ double g_angle(double ax, double ay, double, bool xneg) {
    const double mx = fmax(ax, ay), mn = fmin(ax, ay);
    const bool swap = ay > ax;
    // min / max by the hardware reciprocal and two Newton steps (to the last
    // bits of FP64; a correctly rounded division is not needed here)
    double r = __builtin_amdgcn_rcp(mx);
    r = fma(r, fma(-mx, r, 1.0), r);
    r = fma(r, fma(-mx, r, 1.0), r);
    const double z = mn * r;
    const double z2 = z * z;
    constexpr int kN = sizeof(kAtan64) / sizeof(kAtan64[0]);
    double p = kAtan64[kN - 1];
#pragma unroll
    for (int i = kN - 2; i >= 0; --i) p = fma(p, z2, kAtan64[i]);
    const double off = swap ? 1.5707963267948966 : (xneg ? 3.141592653589793 : 0.0);
    return fma(swap != xneg ? -z : z, p, off);
}
__device__ __forceinline__ float g_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double g_rsqrt(double x) {
    // hardware estimate refined by two Newton steps r <- r (3 - x r^2) / 2
    double r = __builtin_amdgcn_rsq(x);
    r = r * fma(-0.5 * x, r * r, 1.5);
    r = r * fma(-0.5 * x, r * r, 1.5);
    return r;
}

// Clamp to [lo, hi]: one median-of-three in FP32; FP64 yields lo for a NaN.
__device__ __forceinline__ float g_clamp(float x, float lo, float hi) { return __builtin_amdgcn_fmed3f(x, lo, hi); }
__device__ __forceinline__ double g_clamp(double x, double lo, double hi) { return fmin(fmax(x, lo), hi); }

// Grid cell of a coordinate x: returns the fraction x - floor(x) and sets i =
// floor(x).  Lanes whose line hits a detector have x in [0, hi + 1) (rows
// alpha / dalpha <= n_alpha, columns tau in [1, n_t] since |t| <= t_max).
// FP32 leaves i unclamped -- floor and convert in one instruction, NaN -> 0,
// infinities saturate -- and tap_address bounds the byte offset instead;
// FP64 clamps i to [0, hi].
__device__ __forceinline__ float cell_split(float x, float, int &i) {
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(i) : "v"(x));
    return __builtin_amdgcn_fractf(x);
}
__device__ __forceinline__ float cell_split(double x, double hi, int &i) {
    const double fl = floor(x);
    i = (int)g_clamp(fl, 0.0, hi);
    return (float)(x - fl);
}

template <class G> struct GConst;
template <> struct GConst<float> {
    static __device__ __forceinline__ float t0_tau(const EvalConsts &e) { return e.t0_tau; }
    static __device__ __forceinline__ float inv_dt(const EvalConsts &e) { return e.inv_dt; }
    static __device__ __forceinline__ float inv_dalpha(const EvalConsts &e) { return e.inv_dalpha; }
};
template <> struct GConst<double> {
    static __device__ __forceinline__ double t0_tau(const EvalConsts &e) { return e.t0_tau_d; }
    static __device__ __forceinline__ double inv_dt(const EvalConsts &e) { return e.inv_dt_d; }
    static __device__ __forceinline__ double inv_dalpha(const EvalConsts &e) { return e.inv_dalpha_d; }
};

__device__ __forceinline__ float g_flip(float x, bool f) { return f ? -x : x; }
__device__ __forceinline__ double g_flip(double x, bool f) { return f ? -x : x; }

// Sinogram coordinates of an image line l (pixels, offset about the principal
// point).  The line's orientation is folded so that alpha = atan2(l2, l1)
// lies in [0, pi): when l2 < 0 (or l2 = 0 with l1 < 0) the line is negated,
// which maps (alpha, t) to (alpha + pi, -t), and the sinogram's odd symmetry
// contributes the sign sgn = -1.
template <class G>
struct LineCoord {
    G l1, l2, l3, rinv;  // folded line, 1/|(l1, l2)|
    G r2, edge;          // |(l1, l2)|^2, (W/2)|l1| + (H/2)|l2|
    float fa, ft, tf;    // bilinear fractions, folded t (FP32)
    int m, j;            // cell: row m, stored column j = k + 1 (in range on hitting lanes; see tap_address)
    bool hit, fold;      // fold: the line was negated (sign -1 on S)
};

// The hit test as a wave mask (inactive lanes read 0): the ballot of the
// per-lane decision reuses its compare, so masks taken before and after a
// branch cost no second comparison.
template <class G>
__device__ __forceinline__ uint64_t hit_mask(const LineCoord<G> &c) {
    return __builtin_amdgcn_ballot_w64(c.hit);
}

template <class G, int NT = 7>
__device__ __forceinline__ LineCoord<G> line_coord(const G h[6], G cs, G sn, const EvalConsts &ec) {
    LineCoord<G> c;
    const G l1 = h[0] * cs + h[3] * sn;
    const G l2 = h[1] * cs + h[4] * sn;
    const G l3 = h[2] * cs + h[5] * sn;
    // fold when l2 < 0; a line with l2 = 0 keeps alpha in {0, pi}, and
    // alpha = pi reads the pad row, which holds the folded values
    const bool fold = l2 < (G)0;
    c.fold = fold;
    c.l1 = g_flip(l1, fold);
    c.l2 = g_flip(l2, fold);
    c.l3 = g_flip(l3, fold);
    const G r2 = l1 * l1 + l2 * l2;
    c.r2 = r2;
    c.rinv = g_rsqrt(r2);
    // 1 / r with the fold's sign: t and the folded cosine without flipping
    // the line itself (negation is exact, so t = -l3_folded / r bit for bit)
    const G rinv_f = g_flip(c.rinv, fold);
    const G t = -l3 * rinv_f;
    // closed detector rectangle of pixel edges:
    // |t| <= (W/2)|cos a| + (H/2)|sin a|  <=>  |l3| <= (W/2)|l1| + (H/2)|l2|
    c.edge = (G)ec.half_w * fabs(l1) + (G)ec.half_h * fabs(l2);
    c.hit = (r2 > (G)0) & (fabs(l3) <= c.edge);
    // the folded l1 is negative iff exactly one of (l1 < 0, fold) holds; at
    // l1 = 0 both quadrant choices give pi/2
    const bool xneg = (l1 < (G)0) != fold;
    G rows;  // alpha / dalpha
    if constexpr (sizeof(G) == 4) {
        // Lanes walk consecutive planes, whose lines turn slowly: in most
        // sweeps every lane that hits has a line steeper than 45 degrees and
        // the wave takes the steep form (no quadrant selects); a wave with
        // any hitting lane at or below 45 degrees takes the general form.
        // Lanes that miss may take either: their sample is discarded.
        if (__builtin_amdgcn_ballot_w64(c.hit & (fabs(l2) <= fabs(l1))) == 0)
            rows = g_angle_rows_steep<NT>(l1 * rinv_f, ec);
        else
            rows = g_angle_rows<NT>(fabs(l1), fabs(l2), c.rinv, xneg, ec);
    } else {
        rows = g_angle(fabs(l1), fabs(l2), c.rinv, xneg) * GConst<G>::inv_dalpha(ec);
    }
    // alpha <= pi (rounded up by at most an ulp) puts row m <= n_alpha: the
    // stored cell rows run to n_alpha, whose upper row continues the
    // sinogram past pi
    c.fa = cell_split(rows, (G)ec.n_alpha, c.m);
    // stored column coordinate: column j holds t_{j-1}, so j = tau with
    // tau = (t + t_max + dt) / dt = t / dt + t0_tau
    const G tau = fma(t, GConst<G>::inv_dt(ec), GConst<G>::t0_tau(ec));
    c.ft = cell_split(tau, (G)ec.n_t, c.j);
    c.tf = (float)t;
    return c;
}


// The four taps of a line's bilinear cell: elements e and e + 1 of the view,
// e = m * row_elems + j.  A view holds < 2^28 elements of <= 8 bytes, so the
// byte offset is a 32-bit value added to the view's base address.  On lanes
// that hit a detector 0 <= m <= n_alpha and 0 <= j <= n_t, so e <= view_elems
// - 2 and the 24-bit multiply is exact.  FP32 leaves the indices of the other
// lanes unclamped (possibly negative or saturated): their offset wraps, and
// one unsigned minimum keeps the load inside the view -- a valid cell whose
// value is discarded.  FP64 indices are clamped already.
template <class Tap, class G>
__device__ __forceinline__ const Tap *tap_address(const LineCoord<G> &c, const Tap *sview, const EvalConsts &ec) {
    uint32_t off = (__umul24((uint32_t)c.m, (uint32_t)ec.row_elems) + (uint32_t)c.j) * (uint32_t)sizeof(Tap);
    if constexpr (sizeof(G) == 4) off = min(off, (uint32_t)(ec.view_elems - 2) * (uint32_t)sizeof(Tap));
    return (const Tap *)((const char *)sview + off);
}
template <class Tap, class G>
__device__ __forceinline__ Taps load_taps(const LineCoord<G> &c, const Tap *sview, const EvalConsts &ec) {
    return Tap::load(tap_address<Tap, G>(c, sview, ec));
}
template <class Tap, class G>
__device__ __forceinline__ typename Tap::Raw fetch_taps(const LineCoord<G> &c, const Tap *sview,
                                                        const EvalConsts &ec) {
    return Tap::fetch(tap_address<Tap, G>(c, sview, ec));
}

// Bilinear interpolation of a cell's taps at fractions (fa along alpha, ft
// along t).
__device__ __forceinline__ float bilerp(const Taps &tp, float fa, float ft) {
    const float r0 = fmaf(ft, tp.s01 - tp.s00, tp.s00);
    const float r1 = fmaf(ft, tp.s11 - tp.s10, tp.s10);
    return fmaf(fa, r1 - r0, r0);
}

// s1 - s0 for the FP16 values in the low (HI = false) or high halves of two
// 32-bit words, in FP32 with one rounding: v_fma_mix_f32 reads FP16 operands
// in place (op_sel picks the half), computing s1 * 1 + (-s0).
template <bool HI>
__device__ __forceinline__ float f16_sub(uint32_t w1, uint32_t w0) {
    float d;
    if constexpr (HI)
        asm("v_fma_mix_f32 %0, %1, 1.0, -%2 op_sel:[1,0,1] op_sel_hi:[1,0,1]" : "=v"(d) : "v"(w1), "v"(w0));
    else
        asm("v_fma_mix_f32 %0, %1, 1.0, -%2 op_sel_hi:[1,0,1]" : "=v"(d) : "v"(w1), "v"(w0));
    return d;
}

// Bilinear value from a cell's raw loaded words.  FP32 and BF16 convert the
// taps first.  FP16 takes the t-differences by f16_sub straight from the
// loaded words (an FP16 value converts to FP32 exactly, so these are the
// same operations and roundings as bilerp on the converted taps) and
// converts only the two taps at t: two conversions per view instead of four.
template <class Tap>
__device__ __forceinline__ float bilinear(const typename Tap::Raw &v, float fa, float ft) {
    return bilerp(Tap::unpack(v), fa, ft);
}
template <>
__device__ __forceinline__ float bilinear<TapF16>(const TapF16::Raw &v, float fa, float ft) {
    // v.x = (S[m][k], S[m+1][k]), v.y = (S[m][k+1], S[m+1][k+1]) as (low, high) halves
    const float s00 = (float)__builtin_bit_cast(_Float16, (uint16_t)(v.x & 0xFFFFu));
    const float s10 = (float)__builtin_bit_cast(_Float16, (uint16_t)(v.x >> 16));
    const float r0 = fmaf(ft, f16_sub<false>(v.y, v.x), s00);
    const float r1 = fmaf(ft, f16_sub<true>(v.y, v.x), s10);
    return fmaf(fa, r1 - r0, r0);
}

// Grangeat weight 1 + t^2 / f^2, times the storage scale of scaled types.
template <class Tap>
__device__ __forceinline__ float grangeat_weight(float t, float inv_f2, float scale) {
    const float w = fmaf(t, t * inv_f2, 1.0f);
    return Tap::kScaled ? w * scale : w;
}

// |S_lam| up to the fold sign: (1 + t^2 / f^2) * scale * bilinear(taps).
template <class Tap, class G>
__device__ __forceinline__ float sample_unsigned(const LineCoord<G> &c, const Taps &tp, float inv_f2, float scale) {
    return grangeat_weight<Tap>(c.tf, inv_f2, scale) * bilerp(tp, c.fa, c.ft);
}

// S_lam from a line's taps: sign * (1 + t^2 / f^2) * scale * bilinear(taps).
template <class Tap, class G>
__device__ __forceinline__ float sample_taps(const LineCoord<G> &c, const Taps &tp, float inv_f2, float scale) {
    const float u = sample_unsigned<Tap, G>(c, tp, inv_f2, scale);
    return c.fold ? -u : u;
}

}  // namespace ecc
