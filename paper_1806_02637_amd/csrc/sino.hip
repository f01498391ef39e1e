// Radon-derivative sinograms on gfx950: Grangeat's intermediate function
// (Eq. 1) on a flat detector, precomputed once per projection and kept in HBM
// (Sec. "Epipolar Consistency").
//
//  1. sino_weight: radial (cosine) weight f / sqrt(f^2 + x^2 + y^2) on pixel
//     centres, written twice: row-major and transposed, both with a 3-pixel
//     zero border so that line samples need no bounds checks.
//  2. sino_radon: 16 lanes per (view, alpha_m, t_k) cell sum bilinear
//     samples along its line, only over the stretch where they can be
//     non-zero; a wave covers 4 neighbouring lines x 16 consecutive samples so
//     its gathers stay within a small image patch (see the kernel).
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
__global__ __launch_bounds__(256) void sino_weight_kernel(const float *__restrict__ images,
                                                          const double *__restrict__ intr, int W, int H,
                                                          float *__restrict__ gw, float *__restrict__ gwT) {
    __shared__ float tile[32][33];
    const int v = blockIdx.z;
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    const double f = intr[3 * v + 0], u0 = intr[3 * v + 1], v0 = intr[3 * v + 2];
    const float ff = (float)(f * f);
    const float *img = images + (int64_t)v * W * H;
    const int Wp = W + 2 * kImgPad, Hp = H + 2 * kImgPad;
    float *out = gw + (int64_t)v * Wp * Hp;
    float *outT = gwT + (int64_t)v * Wp * Hp;
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + tx, j = j0 + r;
        float val = 0.0f;
        if (i < W && j < H) {
            const float x = (float)(i - u0), y = (float)(j - v0);
            val = img[(int64_t)j * W + i] * ((float)f * rsqrtf(ff + x * x + y * y));
            out[(int64_t)(j + kImgPad) * Wp + (i + kImgPad)] = val;
        }
        tile[r][tx] = val;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + r, j = j0 + tx;
        if (i < W && j < H) outT[(int64_t)(i + kImgPad) * Hp + (j + kImgPad)] = tile[tx][r];
    }
}

hipError_t launch_sino_weight(const float *images, const double *intr, int n_views, int W, int H, float *gw,
                              float *gwT, hipStream_t s) {
    dim3 grid((W + 31) / 32, (H + 31) / 32, n_views);
    hipLaunchKernelGGL(sino_weight_kernel, grid, dim3(256), 0, s, images, intr, W, H, gw, gwT);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// s-interval where c0 + s dc stays inside (lo, hi)
__device__ __forceinline__ void clip_axis(double c0, double dc, double lo, double hi, double &s_lo, double &s_hi) {
    if (fabs(dc) < 1e-12) {
        if (!(c0 > lo && c0 < hi)) {
            s_lo = 1.0;
            s_hi = -1.0;
        }
        return;
    }
    double a = (lo - c0) / dc, b = (hi - c0) / dc;
    if (a > b) {
        double tmp = a;
        a = b;
        b = tmp;
    }
    s_lo = fmax(s_lo, a);
    s_hi = fmin(s_hi, b);
}

typedef float float2_a4 __attribute__((ext_vector_type(2), aligned(4)));

// Block = 4 waves; wave = 4 detector lines (consecutive t) x 16 lanes along
// each line.  Lane (ti, si) takes samples j = j0 + si + 16 i of line ti, so
// one gather of the wave touches a compact patch of about 6 x 8 pixels
// whatever the angle; the image copy is chosen so that the lines run along
// its contiguous axis.  Per lane the sample position is kept as an integer
// pixel plus an FP32 fraction renormalised every step (drift < 1e-4 px over
// a line); per-lane sums are flushed from FP32 to FP64 every 32 steps and the
// 16 lane sums of a line are added in a fixed butterfly order.
__global__ __launch_bounds__(256) void sino_radon_kernel(const float *__restrict__ gw, const float *__restrict__ gwT,
                                                         const double *__restrict__ intr, int W, int H,
                                                         int n_alpha, int n_t, double t_max, double dt, double ds,
                                                         int n_s, double *__restrict__ G) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ti = lane >> 4, si = lane & 15;
    const int k = (blockIdx.x * 4 + wave) * 4 + ti;
    const int m = blockIdx.y, v = blockIdx.z;
    const double u0 = intr[3 * v + 1], v0 = intr[3 * v + 2];
    const double alpha = m * (kPi / n_alpha);
    double sa, ca;
    sincos(alpha, &sa, &ca);
    const double t = -t_max + (k < n_t ? k : 0) * dt;
    // sample at s: (x, y) = (u0 + t ca - s sa, v0 + t sa + s ca); the line
    // direction (-sa, ca) is closer to the x axis when |sa| > |ca|
    const bool trans = fabs(sa) <= fabs(ca);  // uniform over the block
    double p0, q0, dp, dq;
    int P_ext, Q_ext;
    const float *img;
    if (!trans) {
        p0 = u0 + t * ca;
        q0 = v0 + t * sa;
        dp = -sa;
        dq = ca;
        P_ext = W;
        Q_ext = H;
        img = gw + (int64_t)v * (W + 2 * kImgPad) * (H + 2 * kImgPad);
    } else {
        p0 = v0 + t * sa;
        q0 = u0 + t * ca;
        dp = ca;
        dq = -sa;
        P_ext = H;
        Q_ext = W;
        img = gwT + (int64_t)v * (W + 2 * kImgPad) * (H + 2 * kImgPad);
    }
    const int pitch = P_ext + 2 * kImgPad;
    double s_lo = -1e300, s_hi = 1e300;
    clip_axis(p0, dp, -1.0, (double)P_ext, s_lo, s_hi);
    clip_axis(q0, dq, -1.0, (double)Q_ext, s_lo, s_hi);
    const double c = 0.5 * (n_s - 1);
    int j_lo = 1, j_hi = 0;  // empty
    if (k < n_t && s_lo <= s_hi) {
        // one extra sample (ds <= 1 px) on each side absorbs rounding of the
        // clip: samples stay within 2 px of the image, inside the zero border
        j_lo = max(0, (int)ceil(s_lo / ds + c) - 1);
        j_hi = min(n_s - 1, (int)floor(s_hi / ds + c) + 1);
    }
    // wave-uniform sweep over the union of the four lines' ranges
    int w_lo = j_lo <= j_hi ? j_lo : 0x7fffffff, w_hi = j_lo <= j_hi ? j_hi : -1;
    for (int off = 16; off < 64; off <<= 1) {
        w_lo = min(w_lo, __shfl_xor(w_lo, off, 64));
        w_hi = max(w_hi, __shfl_xor(w_hi, off, 64));
    }
    double acc = 0.0;
    if (w_lo <= w_hi) {
        const int j_first = w_lo + si;
        const double s = (j_first - c) * ds;
        const double pp = p0 + s * dp, qq = q0 + s * dq;
        const double pfl = floor(pp), qfl = floor(qq);
        float fp = (float)(pp - pfl), fq = (float)(qq - qfl);
        int ip = (int)pfl + kImgPad, iq = (int)qfl + kImgPad;
        const float sp = (float)(16.0 * ds * dp), sq = (float)(16.0 * ds * dq);
        float part = 0.0f;
        int n_in_part = 0;
        for (int j = j_first; j - si <= w_hi; j += 16) {
            if (j >= j_lo && j <= j_hi) {
                const float *ptr = img + (int64_t)iq * pitch + ip;
                const float2_a4 top = *(const float2_a4 *)ptr;
                const float2_a4 bot = *(const float2_a4 *)(ptr + pitch);
                const float a = fmaf(fp, top.y - top.x, top.x);
                const float b = fmaf(fp, bot.y - bot.x, bot.x);
                part += fmaf(fq, b - a, a);
            }
            fp += sp;
            fq += sq;
            const float flp = floorf(fp), flq = floorf(fq);
            fp -= flp;
            fq -= flq;
            ip += (int)flp;
            iq += (int)flq;
            if (++n_in_part == 32) {
                acc += (double)part;
                part = 0.0f;
                n_in_part = 0;
            }
        }
        acc += (double)part;
    }
    for (int off = 1; off < 16; off <<= 1) acc += __shfl_xor(acc, off, 64);
    if (si == 0 && k < n_t) G[((int64_t)v * n_alpha + m) * n_t + k] = acc * ds;
}

hipError_t launch_sino_radon(const float *gw, const float *gwT, const double *intr, int n_views, int W, int H,
                             int n_alpha, int n_t, double ds, double *G, hipStream_t s) {
    const double t_max = 0.5 * sqrt((double)W * W + (double)H * H);
    const double dt = 2.0 * t_max / (n_t - 1);
    const int n_s = 2 * (int)ceil(t_max / ds) + 1;
    dim3 grid((n_t + 15) / 16, n_alpha, n_views);  // 16 lines per block
    hipLaunchKernelGGL(sino_radon_kernel, grid, dim3(256), 0, s, gw, gwT, intr, W, H, n_alpha, n_t, t_max, dt, ds,
                       n_s, G);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stored value at (m, k), m = 0..n_alpha (row n_alpha = alpha = pi), from
// either the line integrals G (central difference) or an external sinogram.
__device__ __forceinline__ double drho_at(const double *G, const float *ext, int v, int m, int k, int n_alpha,
                                          int n_t, double inv_2dt) {
    if (ext) return (double)ext[((int64_t)v * (n_alpha + 1) + m) * n_t + k];
    double sign = 1.0;
    if (m == n_alpha) {
        m = 0;
        k = n_t - 1 - k;
        sign = -1.0;
    }
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
    const int64_t e = ((int64_t)v * n_alpha + m) * row_elems + j;
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
    dim3 g2((n_t + 2 + 255) / 256, n_alpha, n_views);
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
