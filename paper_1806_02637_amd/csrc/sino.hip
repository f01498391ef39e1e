// Radon-derivative sinograms on gfx950: Grangeat's intermediate function
// (Eq. 1) on a flat detector, precomputed once per projection and kept in HBM
// (Sec. "Epipolar Consistency").
//
//  1. sino_weight: radial (cosine) weight f / sqrt(f^2 + x^2 + y^2) on pixel
//     centres, written in two orientations (rows = image rows, and rows =
//     image columns), each with a 3-pixel zero border and with rows stored
//     in interleaved pairs: element (r, c) holds (row r, row r + 1) at
//     column c, so one 16-byte load returns a sample's 2 x 2 neighbourhood.
//  2. sino_radon: a wave sums the bilinear samples of one (view, alpha_m,
//     t_k) line, its 64 lanes taking consecutive samples, over the stretch
//     where they can be non-zero; the orientation in which the line runs
//     along the rows is used, so a wave's gather covers a few cache lines.
//  3. sino_store: central t-difference of the line integrals, the pad row
//     at alpha = pi from the odd symmetry, conversion to the storage type and
//     the row-interleaved layout the consistency kernels read.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <math.h>
#include <stdint.h>

#include "ecc_internal.hpp"

namespace ecc {

static constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Weighted pixel (x, y) of view v's image is written to both interleaved
// copies: gw2 (rows = image rows) at (y, x).x and (y - 1, x).y, gwT2 (rows =
// image columns) at (x, y).x and (x - 1, y).y, all with the 3-pixel border
// (the buffers are zeroed beforehand).  The transposed writes go through an
// LDS tile so that both copies are written along their rows.
__global__ __launch_bounds__(256) void sino_weight_kernel(const float *__restrict__ images,
                                                          const double *__restrict__ intr, int W, int H,
                                                          float *__restrict__ gw2, float *__restrict__ gwT2) {
    __shared__ float tile[32][33];
    const int v = blockIdx.z;
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    const double f = intr[3 * v + 0], u0 = intr[3 * v + 1], v0 = intr[3 * v + 2];
    const float ff = (float)(f * f);
    const float *img = images + (int64_t)v * W * H;
    const int Wp = W + 2 * kImgPad, Hp = H + 2 * kImgPad;
    // interleaved copies: (Hp - 1) x Wp pairs and (Wp - 1) x Hp pairs
    float *out = gw2 + (int64_t)v * 2 * Wp * Hp;
    float *outT = gwT2 + (int64_t)v * 2 * Wp * Hp;
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + tx, j = j0 + r;
        float val = 0.0f;
        if (i < W && j < H) {
            const float x = (float)(i - u0), y = (float)(j - v0);
            val = img[(int64_t)j * W + i] * ((float)f * rsqrtf(ff + x * x + y * y));
            const int64_t e = (int64_t)(j + kImgPad) * Wp + (i + kImgPad);  // pair index of (row, col)
            out[2 * e] = val;                 // (row j, col i).x
            out[2 * (e - Wp) + 1] = val;      // (row j - 1, col i).y
        }
        tile[r][tx] = val;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + r, j = j0 + tx;
        if (i < W && j < H) {
            const int64_t e = (int64_t)(i + kImgPad) * Hp + (j + kImgPad);
            outT[2 * e] = tile[tx][r];
            outT[2 * (e - Hp) + 1] = tile[tx][r];
        }
    }
}

hipError_t launch_sino_weight(const float *images, const double *intr, int n_views, int W, int H, float *gw,
                              float *gwT, hipStream_t s) {
    dim3 grid((W + 31) / 32, (H + 31) / 32, n_views);
    hipLaunchKernelGGL(sino_weight_kernel, grid, dim3(256), 0, s, images, intr, W, H, gw, gwT);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// s-interval where c0 + s dc stays inside (lo, hi), intersected into
// [s_lo, s_hi]; dc != 0 is given through its reciprocal.
__device__ __forceinline__ void clip_axis_r(double c0, double inv_dc, double lo, double hi, double &s_lo,
                                            double &s_hi) {
    const double a = (lo - c0) * inv_dc, b = (hi - c0) * inv_dc;
    s_lo = fmax(s_lo, fmin(a, b));
    s_hi = fmin(s_hi, fmax(a, b));
}

// FP64 value of another lane by DPP (two 32-bit moves).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

typedef float f32x4_a8 __attribute__((ext_vector_type(4), aligned(8)));

// Nonnegative position in pixels as a 32.32 fixed-point integer (a negative
// step is its two's complement).
__device__ __forceinline__ int64_t to_fixed(double x) { return (int64_t)llrint(ldexp(x, 32)); }

// Fraction of a 32.32 position from its low word: the top 23 bits become the
// mantissa of a float in [1, 2) (one funnel shift), minus 1 (exact).
__device__ __forceinline__ float fixed_fraction(uint32_t lo) {
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, lo, 9u)) - 1.0f;
}

// Block = 4 waves; each wave sums kLinesPerWave = 4 consecutive lines (t_k)
// of one alpha_m at once, 16 lanes per line: lane l takes line l / 16 and
// the samples j = j_lo + (l mod 16) + 16 i of that line's clipped stretch.
// A gather thus covers a compact patch (16 samples along, 4 lines across)
// of the image and touches few cache lines.  Positions are carried as 32.32
// fixed-point integers (one 64-bit add per sample and axis; the step is
// rounded to 2^-32 px, a drift below 1e-8 px over a line), the pad offset
// included so that they stay positive: the high word is the pixel, the low
// word's top 23 bits the bilinear weight.  Each lane sums up to 32 samples in
// FP32 before adding to its FP64 total; the 16 lane totals of a line are
// added in a fixed butterfly order.
constexpr int kLinesPerWave = 4;
constexpr int kLanesPerLine = 64 / kLinesPerWave;

// Sum over each group of LANES consecutive lanes (4, 8, 16 or 32) in a fixed
// order (pairs, quads, half rows, rows, row pairs); the total ends in the
// group's last lane (in every lane of a group of at most 16).
template <int LANES>
__device__ __forceinline__ double group_sum_f64(double x) {
    static_assert(LANES == 4 || LANES == 8 || LANES == 16 || LANES == 32, "group of 4 to 32 lanes");
    x += dpp_f64<0xB1, 0xF>(x);                        // quad_perm [1,0,3,2]
    x += dpp_f64<0x4E, 0xF>(x);                        // quad_perm [2,3,0,1]
    if (LANES >= 8) x += dpp_f64<0x141, 0xF>(x);       // row_half_mirror
    if (LANES >= 16) x += dpp_f64<0x140, 0xF>(x);      // row_mirror
    if (LANES >= 32) x += dpp_f64<0x142, 0xA>(x);      // row_bcast:15 into rows 1 and 3
    return x;
}

__global__ __launch_bounds__(256) void sino_radon_kernel(const float *__restrict__ gw2,
                                                         const float *__restrict__ gwT2,
                                                         const double *__restrict__ intr, int W, int H,
                                                         int n_alpha, int n_t, double t_max, double dt, double ds,
                                                         int n_s, double *__restrict__ G) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = blockIdx.y, v = blockIdx.z;
    const double u0 = intr[3 * v + 1], v0 = intr[3 * v + 2];
    const double alpha = m * (kPi / n_alpha);
    double sa, ca;
    sincos(alpha, &sa, &ca);
    // sample at s: (x, y) = (u0 + t ca - s sa, v0 + t sa + s ca); use the copy
    // whose rows run closer to the line direction (-sa, ca)
    const bool trans = fabs(sa) <= fabs(ca);  // uniform over the block
    const int Wp = W + 2 * kImgPad, Hp = H + 2 * kImgPad;
    const int P_ext = trans ? H : W, Q_ext = trans ? W : H;
    const int pitch = trans ? Hp : Wp;  // pairs per row
    const double dp = trans ? ca : -sa, dq = trans ? -sa : ca;
    const float *img = (trans ? gwT2 : gw2) + (int64_t)v * 2 * Wp * Hp;
    const double c = 0.5 * (n_s - 1);
    const int64_t fx_step_p = to_fixed(kLanesPerLine * ds * dp), fx_step_q = to_fixed(kLanesPerLine * ds * dq);
    // reciprocals for the clip: |dp| >= 1/sqrt(2) by the choice of copy, dq
    // may vanish (lines along an image axis)
    const double inv_dp = 1.0 / dp, inv_ds = 1.0 / ds;
    const bool q_flat = fabs(dq) < 1e-12;
    const double inv_dq = q_flat ? 0.0 : 1.0 / dq;
    // this lane's line and place in it
    const int li = lane / kLanesPerLine, sl = lane % kLanesPerLine;
    const int k = (blockIdx.x * 4 + wave) * kLinesPerWave + li;
    const double t = -t_max + k * dt;
    const double p0 = trans ? v0 + t * sa : u0 + t * ca;
    const double q0 = trans ? u0 + t * ca : v0 + t * sa;
    double s_lo = -1e300, s_hi = 1e300;
    clip_axis_r(p0, inv_dp, -1.0, (double)P_ext, s_lo, s_hi);
    if (q_flat) {
        if (!(q0 > -1.0 && q0 < (double)Q_ext)) {
            s_lo = 1.0;
            s_hi = -1.0;
        }
    } else {
        clip_axis_r(q0, inv_dq, -1.0, (double)Q_ext, s_lo, s_hi);
    }
    int n = 0, j_lo = 0;  // the same on the line's 16 lanes
    if (k < n_t && s_lo <= s_hi) {
        // one extra sample (ds <= 1 px) on each side absorbs rounding of the
        // clip: samples stay within 2 px of the image, inside the zero border
        j_lo = max(0, (int)ceil(s_lo * inv_ds + c) - 1);
        n = max(0, min(n_s - 1, (int)floor(s_hi * inv_ds + c) + 1) - j_lo + 1);
    }
    // sweeps in which every lane of the wave has a sample, and in which some do
    int n_min = n, n_max = n;
    for (int o = kLanesPerLine; o < 64; o <<= 1) {
        n_min = min(n_min, __shfl_xor(n_min, o, 64));
        n_max = max(n_max, __shfl_xor(n_max, o, 64));
    }
    const int full = __builtin_amdgcn_readfirstlane(n_min / kLanesPerLine);
    const int sweeps = __builtin_amdgcn_readfirstlane((n_max + kLanesPerLine - 1) / kLanesPerLine);
    const double s = (j_lo + sl - c) * ds;
    int64_t pp = to_fixed(p0 + s * dp + kImgPad), qq = to_fixed(q0 + s * dq + kImgPad);
    auto sample = [&]() {
        const int ip = (int)(pp >> 32), iq = (int)(qq >> 32);
        const float fp = fixed_fraction((uint32_t)pp), fq = fixed_fraction((uint32_t)qq);
        const uint32_t e = __umul24((uint32_t)iq, (uint32_t)pitch) + (uint32_t)ip;
        const f32x4_a8 g = *(const f32x4_a8 *)((const char *)img + e * 8u);
        // g = (row iq, row iq + 1) at column ip, then at column ip + 1
        const float a = fmaf(fp, g.z - g.x, g.x);
        const float b = fmaf(fp, g.w - g.y, g.y);
        return fmaf(fq, b - a, a);
    };
    double acc = 0.0;
    for (int i0 = 0; i0 < full; i0 += 32) {
        const int i1 = min(i0 + 32, full);
        float part = 0.0f;
#pragma unroll 4
        for (int i = i0; i < i1; ++i) {
            part += sample();
            pp += fx_step_p;
            qq += fx_step_q;
        }
        acc += (double)part;
    }
    // the lines' ragged ends (adjacent lines differ by a few samples)
    for (int i = full; i < sweeps; ++i) {
        if (sl + kLanesPerLine * i < n) acc += (double)sample();
        pp += fx_step_p;
        qq += fx_step_q;
    }
    acc = group_sum_f64<kLanesPerLine>(acc);
    if (sl == kLanesPerLine - 1 && k < n_t) G[((int64_t)v * n_alpha + m) * n_t + k] = acc * ds;
}

hipError_t launch_sino_radon(const float *gw, const float *gwT, const double *intr, int n_views, int W, int H,
                             int n_alpha, int n_t, double ds, double *G, hipStream_t s) {
    const double t_max = 0.5 * sqrt((double)W * W + (double)H * H);
    const double dt = 2.0 * t_max / (n_t - 1);
    const int n_s = 2 * (int)ceil(t_max / ds) + 1;
    dim3 grid((n_t + 4 * kLinesPerWave - 1) / (4 * kLinesPerWave), n_alpha, n_views);
    hipLaunchKernelGGL(sino_radon_kernel, grid, dim3(256), 0, s, gw, gwT, intr, W, H, n_alpha, n_t, t_max, dt, ds,
                       n_s, G);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stored value at (m, k), m = 0..n_alpha + 1, from either the line integrals
// G (central difference) or an external sinogram [n_alpha + 1][n_t].  Rows
// past pi follow from the odd symmetry S(alpha + pi, t) = -S(alpha, -t); an
// external sinogram supplies its own row n_alpha (alpha = pi).
__device__ __forceinline__ double drho_at(const double *G, const float *ext, int v, int m, int k, int n_alpha,
                                          int n_t, double inv_2dt) {
    double sign = 1.0;
    if (m >= n_alpha && !(ext && m == n_alpha)) {
        m -= n_alpha;
        k = n_t - 1 - k;
        sign = -1.0;
    }
    if (ext) return sign * (double)ext[((int64_t)v * (n_alpha + 1) + m) * n_t + k];
    const double *row = G + ((int64_t)v * n_alpha + m) * n_t;
    const double hi = k + 1 < n_t ? row[k + 1] : 0.0;
    const double lo = k - 1 >= 0 ? row[k - 1] : 0.0;
    return sign * (hi - lo) * inv_2dt;
}

// Largest |value| per view (for the FP16 scale): a workgroup scans 32 rows
// of one view and issues one atomic max (order-independent, so the result is
// deterministic).
__global__ __launch_bounds__(256) void sino_absmax_kernel(const double *G, const float *ext, int n_alpha, int n_t,
                                                          double inv_2dt, uint32_t *absmax) {
    __shared__ float red[4];
    const int v = blockIdx.y;
    const int m0 = blockIdx.x * 32;
    const int m1 = min(m0 + 32, n_alpha + 1);
    float a = 0.0f;
    for (int m = m0; m < m1; ++m)
        for (int k = threadIdx.x; k < n_t; k += 256)
            a = fmaxf(a, fabsf((float)drho_at(G, ext, v, m, k, n_alpha, n_t, inv_2dt)));
    for (int off = 32; off > 0; off >>= 1) a = fmaxf(a, __shfl_xor(a, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        if (mx > 0.0f) atomicMax(absmax + v, __float_as_uint(mx));
    }
}

__device__ __forceinline__ uint16_t to_bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint16_t to_f16_rne(float x) {
    _Float16 h = (_Float16)x;
    return __builtin_bit_cast(uint16_t, h);
}

__global__ __launch_bounds__(256) void sino_store_kernel(const double *G, const float *ext, int n_alpha, int n_t,
                                                         double inv_2dt, int dtype, void *sino,
                                                         float *view_scale, const uint32_t *absmax) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;  // column 0..n_t+1
    const int m = blockIdx.y, v = blockIdx.z;
    const int row_elems = n_t + 2;
    if (j >= row_elems) return;
    // FP16: exact power-of-two scale so that the view's largest magnitude
    // lands in (2^13, 2^14]
    float scale = 1.0f;
    if (dtype == 2) {
        const float mx = __uint_as_float(absmax[v]);
        int e = 0;
        if (mx > 0.0f) {
            int ex;
            frexpf(mx, &ex);  // mx = f * 2^ex, f in [0.5, 1)
            e = ex - 14;
        }
        scale = ldexpf(1.0f, e);
    }
    if (m == 0 && j == 0) view_scale[v] = scale;
    const int k = j - 1;
    float lo = 0.0f, hi = 0.0f;
    if (k >= 0 && k < n_t) {
        lo = (float)drho_at(G, ext, v, m, k, n_alpha, n_t, inv_2dt);
        hi = (float)drho_at(G, ext, v, m + 1, k, n_alpha, n_t, inv_2dt);
    }
    const int64_t e = ((int64_t)v * (n_alpha + 1) + m) * row_elems + j;
    if (dtype == 0) {
        float2 *out = (float2 *)sino;
        out[e] = make_float2(lo, hi);
    } else {
        const float inv = 1.0f / scale;
        uint32_t packed;
        if (dtype == 1)
            packed = (uint32_t)to_bf16_rne(lo) | ((uint32_t)to_bf16_rne(hi) << 16);
        else
            packed = (uint32_t)to_f16_rne(lo * inv) | ((uint32_t)to_f16_rne(hi * inv) << 16);
        ((uint32_t *)sino)[e] = packed;
    }
}

hipError_t launch_sino_store(const double *G, const float *ext, int n_views, int n_alpha, int n_t, double dt,
                             int dtype, void *sino, float *view_scale, uint32_t *view_absmax, hipStream_t s) {
    const double inv_2dt = 0.5 / dt;
    if (dtype == 2) {
        hipError_t err = hipMemsetAsync(view_absmax, 0, sizeof(uint32_t) * n_views, s);
        if (err != hipSuccess) return err;
        dim3 g1((n_alpha + 1 + 31) / 32, n_views);
        hipLaunchKernelGGL(sino_absmax_kernel, g1, dim3(256), 0, s, G, ext, n_alpha, n_t, inv_2dt, view_absmax);
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    dim3 g2((n_t + 2 + 255) / 256, n_alpha + 1, n_views);
    hipLaunchKernelGGL(sino_store_kernel, g2, dim3(256), 0, s, G, ext, n_alpha, n_t, inv_2dt, dtype, sino,
                       view_scale, view_absmax);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sino_read_kernel(const void *sino, const float *view_scale, SinoLayout L,
                                                        int v, float *out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;  // 0..n_alpha
    if (k >= L.n_t) return;
    const int mr = m < L.n_alpha ? m : L.n_alpha - 1;
    const int half = m < L.n_alpha ? 0 : 1;
    const int64_t e = (int64_t)v * L.view_elems + (int64_t)mr * L.row_elems + (k + 1);
    float val;
    if (L.dtype == 0) {
        const float2 p = ((const float2 *)sino)[e];
        val = half ? p.y : p.x;
    } else {
        const uint32_t p = ((const uint32_t *)sino)[e];
        const uint16_t h = (uint16_t)(half ? (p >> 16) : (p & 0xFFFFu));
        if (L.dtype == 1)
            val = __uint_as_float((uint32_t)h << 16);
        else
            val = (float)__builtin_bit_cast(_Float16, h);
    }
    out[(int64_t)m * L.n_t + k] = val * view_scale[v];
}

hipError_t launch_sino_read(const void *sino, const float *view_scale, SinoLayout L, int view, float *out,
                            hipStream_t s) {
    dim3 grid((L.n_t + 255) / 256, L.n_alpha + 1, 1);
    hipLaunchKernelGGL(sino_read_kernel, grid, dim3(256), 0, s, sino, view_scale, L, view, out);
    return hipGetLastError();
}

}  // namespace ecc
