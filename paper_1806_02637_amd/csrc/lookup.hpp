// Per-plane work of the consistency kernels: epipolar line from the pair's
// line map, its sinogram coordinates (alpha, t), the hit test and the
// weighted bilinear lookup of S_lam (Eq. 1 indexed by the line, Sec.
// "Epipolar Consistency"), in geometry precision G (float or double).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ecc_internal.hpp"

namespace ecc {

// Per-plane constants of one view pair, built in FP64 and kept in LDS.
//   ha, hb: line maps of views a and b, l = H (cos kappa, sin kappa) with the
//           line's offset about the principal point (H column-major);
//   k0, dk: kappa_k = k0 + k dk;
//   inv_f2a/b: 1 / f^2 of the views (Grangeat weight 1 + t^2 / f^2);
//   sa, sb: storage scales of the two views' sinograms; va, vb: view ids.
template <class G>
struct PairConst {
    G ha[6], hb[6];
    G k0, dk;
    float inv_f2a, inv_f2b, sa, sb;
    int va, vb;
};

// ---- storage types: one load returns the four taps of a bilinear cell ----
struct Taps {
    float s00, s10, s01, s11;  // S[m][k], S[m+1][k], S[m][k+1], S[m+1][k+1]
};

typedef float f32x4_a8 __attribute__((ext_vector_type(4), aligned(8)));
typedef uint32_t u32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));

struct TapF32 {
    float lo, hi;
    static __device__ __forceinline__ Taps load(const TapF32 *p) {
        const f32x4_a8 v = *(const f32x4_a8 *)p;
        return Taps{v.x, v.y, v.z, v.w};
    }
};

struct TapBF16 {
    uint32_t bits;
    static __device__ __forceinline__ Taps load(const TapBF16 *p) {
        const u32x2_a4 v = *(const u32x2_a4 *)p;
        return Taps{__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xFFFF0000u), __uint_as_float(v.y << 16),
                    __uint_as_float(v.y & 0xFFFF0000u)};
    }
};

struct TapF16 {
    uint32_t bits;
    static __device__ __forceinline__ float h2f(uint32_t h) {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
    }
    static __device__ __forceinline__ Taps load(const TapF16 *p) {
        const u32x2_a4 v = *(const u32x2_a4 *)p;
        return Taps{h2f(v.x & 0xFFFFu), h2f(v.x >> 16), h2f(v.y & 0xFFFFu), h2f(v.y >> 16)};
    }
};

// ---- precision-generic helpers ----------------------------------------------
__device__ __forceinline__ void g_sincos(float x, float *s, float *c) { sincosf(x, s, c); }
__device__ __forceinline__ void g_sincos(double x, double *s, double *c) { sincos(x, s, c); }
__device__ __forceinline__ float g_atan2(float y, float x) { return atan2f(y, x); }
__device__ __forceinline__ double g_atan2(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ float g_rsqrt(float x) { return 1.0f / sqrtf(x); }
__device__ __forceinline__ double g_rsqrt(double x) { return 1.0 / sqrt(x); }

template <class G> struct GConst;
template <> struct GConst<float> {
    static __device__ __forceinline__ float pi() { return 3.14159265358979323846f; }
    static __device__ __forceinline__ float t_max(const EvalConsts &e) { return e.t_max; }
    static __device__ __forceinline__ float inv_dt(const EvalConsts &e) { return e.inv_dt; }
    static __device__ __forceinline__ float inv_dalpha(const EvalConsts &e) { return e.inv_dalpha; }
};
template <> struct GConst<double> {
    static __device__ __forceinline__ double pi() { return 3.14159265358979323846; }
    static __device__ __forceinline__ double t_max(const EvalConsts &e) { return e.t_max_d; }
    static __device__ __forceinline__ double inv_dt(const EvalConsts &e) { return e.inv_dt_d; }
    static __device__ __forceinline__ double inv_dalpha(const EvalConsts &e) { return e.inv_dalpha_d; }
};

// Sinogram coordinates of the image line l (pixels, offset about the
// principal point) and the lookup position.
template <class G>
struct LineCoord {
    G l1, l2, l3, r2, rinv, t;  // t after folding
    float sgn;                   // -1 when alpha was folded by pi
    float fa, ft, tf;            // bilinear fractions, folded t in FP32
    int m, k;                    // floor cell (clamped for memory safety)
    bool hit;
};

template <class G>
__device__ __forceinline__ LineCoord<G> line_coord(const G h[6], G cs, G sn, const EvalConsts &ec) {
    LineCoord<G> c;
    c.l1 = h[0] * cs + h[3] * sn;
    c.l2 = h[1] * cs + h[4] * sn;
    c.l3 = h[2] * cs + h[5] * sn;
    c.r2 = c.l1 * c.l1 + c.l2 * c.l2;
    c.rinv = g_rsqrt(c.r2);
    G alpha = g_atan2(c.l2, c.l1);
    G t = -c.l3 * c.rinv;
    c.sgn = 1.0f;
    const G pi = GConst<G>::pi();
    if (alpha < (G)0) {
        alpha += pi;
        t = -t;
        c.sgn = -1.0f;
    } else if (alpha >= pi) {
        alpha -= pi;
        t = -t;
        c.sgn = -1.0f;
    }
    c.t = t;
    // closed detector rectangle of pixel edges: |t| <= (W/2)|cos a| + (H/2)|sin a|
    const G sup = ((G)ec.half_w * fabs(c.l1) + (G)ec.half_h * fabs(c.l2)) * c.rinv;
    c.hit = (c.r2 > (G)0) && (fabs(t) <= sup);
    const G aa = alpha * GConst<G>::inv_dalpha(ec);
    const G mf = fmin(fmax(floor(aa), (G)0), (G)(ec.n_alpha - 1));
    const G tau = (t + GConst<G>::t_max(ec)) * GConst<G>::inv_dt(ec);
    const G kf = fmin(fmax(floor(tau), (G)-1), (G)(ec.n_t - 1));
    c.fa = (float)(aa - mf);
    c.ft = (float)(tau - kf);
    c.m = (int)mf;
    c.k = (int)kf;
    c.tf = (float)t;
    return c;
}

// S_lam at a line's sinogram coordinates: sign * (1 + t^2 / f^2) * scale * bilinear(taps).
template <class Tap, class G>
__device__ __forceinline__ float sample_at(const LineCoord<G> &c, const Tap *sview, const EvalConsts &ec,
                                           float inv_f2, float scale) {
    const Taps tp = Tap::load(sview + (int64_t)c.m * ec.row_elems + (c.k + 1));
    const float r0 = fmaf(c.ft, tp.s01 - tp.s00, tp.s00);
    const float r1 = fmaf(c.ft, tp.s11 - tp.s10, tp.s10);
    const float B = fmaf(c.fa, r1 - r0, r0);
    return (c.sgn * scale) * fmaf(c.tf * c.tf, inv_f2, 1.0f) * B;
}

template <class Tap, class G>
__device__ __forceinline__ float lookup(const G h[6], G cs, G sn, const Tap *sview, const EvalConsts &ec,
                                        float inv_f2, float scale, bool &hit) {
    const LineCoord<G> c = line_coord<G>(h, cs, sn, ec);
    hit = c.hit;
    return sample_at<Tap, G>(c, sview, ec, inv_f2, scale);
}

}  // namespace ecc
