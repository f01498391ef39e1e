// FDK reconstruction (Feldkamp, Davis and Kress 1984) of a circular short
// scan with per-view projection matrices: the check of a motion-compensated
// scan ("Experiments"), where the estimated motion enters only through
// P'_lam = P_lam T(theta_lam) in the back-projection.
//
// fdk_view       one thread per view: orbit angle from the nominal source,
//                angular step, source distance D, and the moved P' in FP32.
// fdk_filter     one workgroup per (view, detector row): Parker's short-scan
//                weight (Parker 1982) and the cosine weight applied while the
//                row is staged in LDS, then the sampled ramp filter (Kak and
//                Slaney, ch. 3: h(0) = 1/4, h(n) = -1/(pi n)^2 for odd n) as a
//                direct sum over the odd taps, written as interleaved row pairs
//                so one 16-byte load returns a bilinear cell.
// fdk_backproject  16 x 16 voxel columns x 16 slices per workgroup; each
//                thread walks one column's 16 voxels through every view:
//                (a, b, c) = P' (x, 1) with rows 0-1 about the principal
//                point, (u, v) = (u0, v0) + (a, b) / c, weight dbeta D^2 / c^2,
//                bilinear read of the filtered view.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ecc_internal.hpp"

namespace ecc {

constexpr double kPiD = 3.14159265358979323846;
constexpr float kPiF = 3.14159265358979f;

// four floats at an 8-byte aligned address (a float2 pair and its neighbour)
typedef float fdk_f32x4_a8 __attribute__((ext_vector_type(4), aligned(8)));

__device__ __forceinline__ double orbit_angle(const ViewGeom &g) { return atan2(g.C[1], g.C[0]); }

__device__ __forceinline__ double wrap_2pi(double a) {
    a = fmod(a, 2.0 * kPiD);
    return a < 0.0 ? a + 2.0 * kPiD : a;
}

__global__ __launch_bounds__(256) void fdk_view_kernel(const ViewGeom *__restrict__ nominal,
                                                       const ViewGeom *__restrict__ moved, int n_views,
                                                       FdkView *__restrict__ out) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_views) return;
    const double b0 = orbit_angle(nominal[0]);
    const double arc = wrap_2pi(orbit_angle(nominal[n_views - 1]) - b0);
    const ViewGeom &g = nominal[v];
    const double D = sqrt(g.C[0] * g.C[0] + g.C[1] * g.C[1] + g.C[2] * g.C[2]);
    const double dbeta = arc / (n_views - 1);
    FdkView o;
    // P' with its image rows taken about the principal point (u - u0, v - v0):
    // keeps the FP32 products near the size of the detector offsets
    const double *Pm = moved[v].P;
    for (int i = 0; i < 4; ++i) {
        o.P[i] = (float)(Pm[i] - g.u0 * Pm[8 + i]);
        o.P[4 + i] = (float)(Pm[4 + i] - g.v0 * Pm[8 + i]);
        o.P[8 + i] = (float)Pm[8 + i];
    }
    o.beta = (float)wrap_2pi(orbit_angle(g) - b0);
    o.delta = (float)(0.5 * (arc - kPiD));
    o.f = (float)g.f;
    o.u0 = (float)g.u0;
    o.v0 = (float)g.v0;
    o.scale = (float)(dbeta * D * D);
    o.inv_tau = (float)(g.f / D);
    o.pad = 0.0f;
    out[v] = o;
}

// Parker's weight at orbit angle beta (from the first view) for fan angle
// gamma, scan range [0, pi + 2 delta].
__device__ __forceinline__ float parker(float beta, float gamma, float delta) {
    if (beta < 2.0f * (delta - gamma)) {
        const float s = sinf(0.25f * kPiF * beta / (delta - gamma));
        return s * s;
    }
    if (beta > kPiF - 2.0f * gamma) {
        const float s = sinf(0.25f * kPiF * (kPiF + 2.0f * delta - beta) / (delta + gamma));
        return s * s;
    }
    return 1.0f;
}

// Dynamic LDS: xs[3W] (the weighted row between two W-long zero margins) and
// hs[W/2 + 1] (the odd ramp taps h(2m + 1)).
__global__ __launch_bounds__(256) void fdk_filter_kernel(const float *__restrict__ images,
                                                         const FdkView *__restrict__ views, int W, int H,
                                                         float2 *__restrict__ Qi) {
    extern __shared__ float sm[];
    float *xs = sm;
    float *hs = sm + 3 * W;
    const int v = blockIdx.x, view = blockIdx.y;
    const FdkView vw = views[view];
    const float *row = images + ((int64_t)view * H + v) * W;
    const float dv = (float)v - vw.v0;
    const float f2 = vw.f * vw.f + dv * dv;
    for (int k = threadIdx.x; k < W; k += blockDim.x) {
        const float du = (float)k - vw.u0;
        const float cosw = vw.f * rsqrtf(f2 + du * du);
        const float gamma = -atanf(du / vw.f);
        xs[W + k] = row[k] * cosw * parker(vw.beta, gamma, vw.delta);
        xs[k] = 0.0f;
        xs[2 * W + k] = 0.0f;
    }
    const int M = W / 2;  // odd taps n = 2m + 1 <= W - 1
    for (int m = threadIdx.x; m < M; m += blockDim.x) {
        const float n = (float)(2 * m + 1);
        hs[m] = -1.0f / (kPiF * kPiF * n * n);
    }
    __syncthreads();
    // interleaved row pairs: Qi[r][c] = (Q[r - 1][c - 1], Q[r][c - 1]) for
    // r = 0..H, c = 0..W + 1, zero beyond the detector
    float2 *pair_lo = Qi + ((int64_t)view * (H + 1) + (v + 1)) * (W + 2);  // .x of row pair (v, v + 1)
    float2 *pair_hi = Qi + ((int64_t)view * (H + 1) + v) * (W + 2);        // .y of row pair (v - 1, v)
    for (int c = threadIdx.x; c < W + 2; c += blockDim.x) {
        float q = 0.0f;
        const int u = c - 1;
        if (u >= 0 && u < W) {
            const float *xu = xs + W + u;
            float acc = 0.25f * xu[0];
#pragma unroll 4
            for (int m = 0; m < M; ++m) {
                const int n = 2 * m + 1;
                acc = fmaf(hs[m], xu[-n] + xu[n], acc);
            }
            q = acc * vw.inv_tau;
        }
        pair_lo[c].x = q;
        pair_hi[c].y = q;
        if (v == 0) (pair_lo - (W + 2))[c].x = 0.0f;  // row pair (-1, 0)
        if (v == H - 1) (pair_lo)[c].y = 0.0f;        // row pair (H - 1, H)
    }
}

constexpr int kBpTile = 16;   // voxel columns per workgroup side
constexpr int kBpSlab = 16;   // slices per thread
constexpr int kBpStage = 128;  // views staged in LDS at a time

__global__ __launch_bounds__(256) void fdk_backproject_kernel(const float2 *__restrict__ Qi,
                                                              const FdkView *__restrict__ views, int n_views,
                                                              int W, int H, FdkVolume vol, float *__restrict__ out) {
    __shared__ FdkView sv[kBpStage];
    const int ix = blockIdx.x * kBpTile + (threadIdx.x % kBpTile);
    const int iy = blockIdx.y * kBpTile + (threadIdx.x / kBpTile);
    const int iz0 = blockIdx.z * kBpSlab;
    const float s = vol.voxel_mm;
    const float x = ((float)ix - 0.5f * (float)(vol.nx - 1)) * s;
    const float y = ((float)iy - 0.5f * (float)(vol.ny - 1)) * s;
    const float z0 = ((float)iz0 - 0.5f * (float)(vol.nz - 1)) * s;
    const int64_t view_elems = (int64_t)(H + 1) * (W + 2);
    float acc[kBpSlab];
#pragma unroll
    for (int k = 0; k < kBpSlab; ++k) acc[k] = 0.0f;
    for (int v0 = 0; v0 < n_views; v0 += kBpStage) {
        const int nv = min(kBpStage, n_views - v0);
        __syncthreads();
        for (int i = threadIdx.x; i < nv; i += blockDim.x) sv[i] = views[v0 + i];
        __syncthreads();
        for (int j = 0; j < nv; ++j) {
            const FdkView &w = sv[j];
            const float a0 = fmaf(w.P[0], x, fmaf(w.P[1], y, fmaf(w.P[2], z0, w.P[3])));
            const float b0 = fmaf(w.P[4], x, fmaf(w.P[5], y, fmaf(w.P[6], z0, w.P[7])));
            const float c0 = fmaf(w.P[8], x, fmaf(w.P[9], y, fmaf(w.P[10], z0, w.P[11])));
            const float da = w.P[2] * s, db = w.P[6] * s, dc = w.P[10] * s;
            const float2 *q = Qi + (int64_t)(v0 + j) * view_elems;
#pragma unroll
            for (int k = 0; k < kBpSlab; ++k) {
                const float a = fmaf((float)k, da, a0);
                const float b = fmaf((float)k, db, b0);
                const float c = fmaf((float)k, dc, c0);
                const float rc = __builtin_amdgcn_rcpf(c);
                const float u = fmaf(a, rc, w.u0), vv = fmaf(b, rc, w.v0);
                const float uf = floorf(u), vf = floorf(vv);
                const float fu = u - uf, fv = vv - vf;
                // cells with a corner on the detector; others read a clamped
                // cell and count zero
                const bool ok = (c > 0.0f) & (uf >= -1.0f) & (uf <= (float)(W - 1)) & (vf >= -1.0f) &
                                (vf <= (float)(H - 1));
                const int iu = (int)fminf(fmaxf(uf, -1.0f), (float)(W - 1));
                const int iv = (int)fminf(fmaxf(vf, -1.0f), (float)(H - 1));
                const fdk_f32x4_a8 t = *(const fdk_f32x4_a8 *)(q + (int64_t)(iv + 1) * (W + 2) + (iu + 1));
                const float top = fmaf(fu, t.z - t.x, t.x);
                const float bot = fmaf(fu, t.w - t.y, t.y);
                const float val = fmaf(fv, bot - top, top);
                acc[k] = ok ? fmaf(w.scale * rc * rc, val, acc[k]) : acc[k];
            }
        }
    }
    if (ix >= vol.nx || iy >= vol.ny) return;
#pragma unroll
    for (int k = 0; k < kBpSlab; ++k) {
        const int iz = iz0 + k;
        if (iz < vol.nz) out[((int64_t)iz * vol.ny + iy) * vol.nx + ix] = acc[k];
    }
}

hipError_t launch_fdk(const float *images, const ViewGeom *nominal, const ViewGeom *moved, int n_views, int W,
                      int H, FdkVolume vol, FdkView *views, float2 *Qi, float *out, hipStream_t s) {
    hipLaunchKernelGGL(fdk_view_kernel, dim3((n_views + 255) / 256), dim3(256), 0, s, nominal, moved, n_views,
                       views);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds = sizeof(float) * (3 * (size_t)W + W / 2 + 1);
    hipLaunchKernelGGL(fdk_filter_kernel, dim3(H, n_views), dim3(256), lds, s, images, (const FdkView *)views, W, H,
                       Qi);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const dim3 grid((vol.nx + kBpTile - 1) / kBpTile, (vol.ny + kBpTile - 1) / kBpTile,
                    (vol.nz + kBpSlab - 1) / kBpSlab);
    hipLaunchKernelGGL(fdk_backproject_kernel, grid, dim3(kBpTile * kBpTile), 0, s, (const float2 *)Qi,
                       (const FdkView *)views, n_views, W, H, vol, out);
    return hipGetLastError();
}

}  // namespace ecc
