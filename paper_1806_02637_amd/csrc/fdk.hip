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
//                direct sum over the odd taps (8 outputs per thread sharing
//                sliding register windows), scaled by dbeta D^2 and written
//                as interleaved row pairs inside a two-wide zero border, so one
//                16-byte load returns a bilinear cell.
// fdk_backproject  16 x 16 voxel columns x 16 slices per workgroup; each
//                thread walks one column's 16 voxels through every view:
//                (a, b, c) = P' (x, 1) with rows 0-1 about the principal
//                point, (u, v) = (u0, v0) + (a, b) / c, weight 1 / c^2,
//                bilinear read of the filtered view (clamped into its zero
//                border off the detector).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ecc_internal.hpp"
#include "fdk.hpp"

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

// Ramp filter of one thread's outputs: the 8 outputs u0, u0 + 2, ..., u0 + 14
// (one parity), Q(u) = x(u) / 4 + sum_m h_m (x(u - n_m) + x(u + n_m)) over the
// odd taps n_m = 2m + 1.  With L_i = x(u0 - 1 - 2i) and R_i = x(u0 + 1 + 2i),
// output j takes L_{m - j} and R_{m + j} at tap m, so two windows of 15
// values slide by 8 taps per chunk: 16 new reads feed 64 tap pairs.  xc: the
// row with zero margins of at least W + 64 on both sides; hs: M8 taps (a
// multiple of 8, zero past the last odd tap).
constexpr int kFiltOut = 8;
__host__ __device__ inline void filter_group(const float *xc, const float *hs, int M8, int u0, float acc[kFiltOut]) {
    float Lw[15], Rw[15];
#pragma unroll
    for (int t = 0; t < 15; ++t) {
        Lw[t] = xc[u0 - 1 - 2 * (t - 7)];  // L_{t - 7}
        Rw[t] = xc[u0 + 1 + 2 * t];        // R_t
    }
#pragma unroll
    for (int j = 0; j < kFiltOut; ++j) acc[j] = 0.25f * xc[u0 + 2 * j];
    for (int c = 0; c < M8; c += 8) {
        float h[8], nL[8], nR[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) h[i] = hs[c + i];
        // the next chunk's new window values, read before this chunk's sums
        // so that the reads overlap them
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            nL[t] = xc[u0 - 1 - 2 * (c + 8 + t)];   // L_{c + 8 + t}
            nR[t] = xc[u0 + 1 + 2 * (c + 15 + t)];  // R_{c + 15 + t}
        }
        // Lw[t] = L_{c - 7 + t}, Rw[t] = R_{c + t}
#pragma unroll
        for (int mm = 0; mm < 8; ++mm) {
#pragma unroll
            for (int j = 0; j < kFiltOut; ++j) acc[j] = fmaf(h[mm], Lw[mm - j + 7] + Rw[mm + j], acc[j]);
        }
#pragma unroll
        for (int t = 0; t < 7; ++t) {
            Lw[t] = Lw[t + 8];
            Rw[t] = Rw[t + 8];
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            Lw[7 + t] = nL[t];
            Rw[7 + t] = nR[t];
        }
    }
}

// Filter workgroups: `rows` (1 or 2) consecutive detector rows of one view
// per workgroup (two rows give more active lanes per wave than one row of
// ceil(W / 8) work items), 2 ceil(W / 16) threads per row (rounded up to
// whole waves over the workgroup), thread 2g + p of a row taking outputs
// 16 g + p + 2 j.  Dynamic LDS per row: the weighted row with W + 64 zeros
// on each side; then the taps, padded to a multiple of 8.
__host__ __device__ inline int filter_margin(int W) { return W + 64; }
__host__ __device__ inline int filter_taps8(int W) { return ((W / 2 + 7) / 8) * 8; }
__host__ __device__ inline int filter_row_floats(int W) { return 2 * filter_margin(W) + W; }
__host__ __device__ inline int filter_items(int W) { return 2 * ((W + 15) / 16); }

__global__ __launch_bounds__(1024) void fdk_filter_kernel(const float *__restrict__ images,
                                                          const FdkView *__restrict__ views, int W, int H, int rows,
                                                          float2 *__restrict__ Qi) {
    extern __shared__ float sm[];
    const int pad = filter_margin(W), M8 = filter_taps8(W), RF = filter_row_floats(W);
    float *hs = sm + rows * RF;  // [M8]
    const int view = blockIdx.y, v_first = blockIdx.x * rows;
    const int n_rows = min(rows, H - v_first);
    const FdkView vw = views[view];
    for (int r = 0; r < n_rows; ++r) {
        float *xs = sm + r * RF;
        const int v = v_first + r;
        const float *row = images + ((int64_t)view * H + v) * W;
        const float dv = (float)v - vw.v0;
        const float f2 = vw.f * vw.f + dv * dv;
        for (int k = threadIdx.x; k < W; k += blockDim.x) {
            const float du = (float)k - vw.u0;
            const float cosw = vw.f * rsqrtf(f2 + du * du);
            const float gamma = -atanf(du / vw.f);
            xs[pad + k] = row[k] * cosw * parker(vw.beta, gamma, vw.delta);
        }
        for (int k = threadIdx.x; k < pad; k += blockDim.x) {
            xs[k] = 0.0f;
            xs[pad + W + k] = 0.0f;
        }
    }
    const int M = W / 2;  // odd taps n = 2m + 1 <= W - 1
    for (int m = threadIdx.x; m < M8; m += blockDim.x) {
        const float n = (float)(2 * m + 1);
        hs[m] = m < M ? -1.0f / (kPiF * kPiF * n * n) : 0.0f;
    }
    __syncthreads();
    // padded grid Qp[v + 2][u + 2] = dbeta D^2 Q[v][u], two zero rows and
    // columns on every side, stored as interleaved row pairs
    // Qi[r][c] = (Qp[r][c], Qp[r + 1][c]), r = 0..H + 2, c = 0..W + 3
    const int WP = W + 4, items = filter_items(W);
    const float out_scale = vw.inv_tau * vw.scale;
    const int r = threadIdx.x / items, item = threadIdx.x % items;
    const int v = v_first + r;
    if (r < n_rows) {
        float2 *row_x = Qi + ((int64_t)view * (H + 3) + (v + 2)) * WP;  // .x of pair r = v + 2
        float2 *row_y = Qi + ((int64_t)view * (H + 3) + (v + 1)) * WP;  // .y of pair r = v + 1
        const int g = item >> 1, u0 = 16 * g + (item & 1);
        if (16 * g < W) {
            float acc[kFiltOut];
            filter_group(sm + r * RF + pad, hs, M8, u0, acc);
#pragma unroll
            for (int j = 0; j < kFiltOut; ++j) {
                const int u = u0 + 2 * j;
                if (u < W) {
                    row_x[u + 2].x = acc[j] * out_scale;
                    row_y[u + 2].y = acc[j] * out_scale;
                }
            }
        }
        if (item < 4) {  // zero columns 0, 1, W + 2, W + 3
            const int c = item < 2 ? item : W + item;
            row_x[c].x = 0.0f;
            row_y[c].y = 0.0f;
        }
    }
    for (int c = threadIdx.x; c < WP; c += blockDim.x) {
        float2 *first = Qi + ((int64_t)view * (H + 3)) * WP;
        if (v_first == 0) {  // zero rows Qp[0], Qp[1]
            first[c].x = 0.0f;
            first[c].y = 0.0f;
            first[WP + c].x = 0.0f;
        }
        if (v_first + n_rows == H) {  // zero rows Qp[H + 2], Qp[H + 3]
            first[(int64_t)(H + 1) * WP + c].y = 0.0f;
            first[(int64_t)(H + 2) * WP + c].x = 0.0f;
            first[(int64_t)(H + 2) * WP + c].y = 0.0f;
        }
    }
}

constexpr int kBpTile = 16;   // voxel columns per workgroup side
constexpr int kBpSlab = 16;   // slices per thread
constexpr int kBpStage = 128;  // views staged in LDS at a time

// Workgroups are numbered so that each XCD (8 per chip, blocks dealt to them
// round-robin) takes one contiguous range of tiles, x fastest then y then z:
// a z-slab of the volume, whose footprint in every view is a band of rows
// that fits the XCD's L2.
__global__ __launch_bounds__(256) void fdk_backproject_kernel(const float2 *__restrict__ Qi,
                                                              const FdkView *__restrict__ views, int n_views,
                                                              int W, int H, FdkVolume vol, int tiles_x, int tiles_y,
                                                              int n_tiles, float *__restrict__ out) {
    __shared__ FdkView sv[kBpStage];
    const int per = (n_tiles + 7) / 8;
    const int tile = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (tile >= n_tiles) return;  // no barrier has been reached yet
    const int tx = tile % tiles_x, ty = (tile / tiles_x) % tiles_y, tz = tile / (tiles_x * tiles_y);
    // each wave takes an 8 x 8 quarter of the 16 x 16 tile: its 64 voxel
    // columns project onto a compact detector patch (few cache lines per gather)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ix = tx * kBpTile + (wave & 1) * 8 + (lane & 7);
    const int iy = ty * kBpTile + (wave >> 1) * 8 + (lane >> 3);
    const int iz0 = tz * kBpSlab;
    const float s = vol.voxel_mm;
    const float x = ((float)ix - 0.5f * (float)(vol.nx - 1)) * s;
    const float y = ((float)iy - 0.5f * (float)(vol.ny - 1)) * s;
    const float z0 = ((float)iz0 - 0.5f * (float)(vol.nz - 1)) * s;
    const uint32_t WP = (uint32_t)W + 4;
    const int64_t view_bytes = (int64_t)(H + 3) * WP * sizeof(float2);
    const float u_hi = (float)W, v_hi = (float)H;
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
            const char *q = (const char *)Qi + (int64_t)(v0 + j) * view_bytes;
#pragma unroll
            for (int k = 0; k < kBpSlab; ++k) {
                const float a = fmaf((float)k, da, a0);
                const float b = fmaf((float)k, db, b0);
                const float c = fmaf((float)k, dc, c0);
                // a point behind the source counts zero (rc = 0 also keeps
                // its coordinates finite)
                const float rc = c > 0.0f ? __builtin_amdgcn_rcpf(c) : 0.0f;
                const float u = fmaf(a, rc, w.u0), vv = fmaf(b, rc, w.v0);
                // cells off the detector are clamped into the two-wide zero
                // border: any point outside reads four zeros
                const float uf = __builtin_amdgcn_fmed3f(floorf(u), -2.0f, u_hi);
                const float vf = __builtin_amdgcn_fmed3f(floorf(vv), -2.0f, v_hi);
                const float fu = u - uf, fv = vv - vf;
                const uint32_t e = __umul24((uint32_t)((int)vf + 2), WP) + (uint32_t)((int)uf + 2);
                const fdk_f32x4_a8 t = *(const fdk_f32x4_a8 *)(q + e * (uint32_t)sizeof(float2));
                const float top = fmaf(fu, t.z - t.x, t.x);
                const float bot = fmaf(fu, t.w - t.y, t.y);
                const float val = fmaf(fv, bot - top, top);
                acc[k] = fmaf(rc * rc, val, acc[k]);
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
    // two rows per workgroup while they fit 64 KB of LDS
    const size_t row_bytes = sizeof(float) * filter_row_floats(W), tap_bytes = sizeof(float) * filter_taps8(W);
    const int rows = 2 * row_bytes + tap_bytes <= 65536 ? 2 : 1;
    const int threads = 64 * ((rows * filter_items(W) + 63) / 64);
    hipLaunchKernelGGL(fdk_filter_kernel, dim3((H + rows - 1) / rows, n_views), dim3(threads), rows * row_bytes + tap_bytes,
                       s, images, (const FdkView *)views, W, H, rows, Qi);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int tiles_x = (vol.nx + kBpTile - 1) / kBpTile, tiles_y = (vol.ny + kBpTile - 1) / kBpTile;
    const int n_tiles = tiles_x * tiles_y * ((vol.nz + kBpSlab - 1) / kBpSlab);
    const int blocks = 8 * ((n_tiles + 7) / 8);
    hipLaunchKernelGGL(fdk_backproject_kernel, dim3(blocks), dim3(kBpTile * kBpTile), 0, s, (const float2 *)Qi,
                       (const FdkView *)views, n_views, W, H, vol, tiles_x, tiles_y, n_tiles, out);
    return hipGetLastError();
}

}  // namespace ecc
