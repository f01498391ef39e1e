// FDK reconstruction (Feldkamp, Davis and Kress 1984) of a circular short
// scan with per-view projection matrices: the check of a motion-compensated
// scan ("Experiments"), where the estimated motion enters only through
// P'_lam = P_lam T(theta_lam) in the back-projection.
//
// fdk_view       one thread per view: orbit angle from the nominal source,
//                angular step, source distance D, and the moved P' in FP32.
// fdk_parker     Parker's short-scan weight (Parker 1982) of every (view,
//                column).
// fdk_weight     cosine- and Parker-weighted detector rows, split by column
//                parity.
// fdk_filter_mfma  the sampled ramp filter (Kak and Slaney, ch. 3: h(0) = 1/4,
//                h(n) = -1/(pi n)^2 for odd n) of every weighted detector
//                row, as two Toeplitz matrix products
//                on the matrix cores (one per output-column parity), scaled by
//                dbeta D^2 and written as interleaved row pairs inside a
//                two-wide zero border (fdk_border writes the border), so one
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

#include <type_traits>

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

// ---------------------------------------------------------------------------
// The ramp filter as a matrix product on the matrix cores.  Split the outputs
// by column parity p, u = 2i + p.  The filter's off-diagonal taps are odd,
// so they pair each output with the inputs of the other parity,
// k = 2j + 1 - p, and u - k = 2(i - j) + 2p - 1: per parity
// Q_p = X_q G_p + X_p / 4 with the Toeplitz G_p[j][i] = h(2(i - j) + 2p - 1).
// The rows of X are all detector rows of all views, so each parity is one
// (N H) x (W / 2) x (W / 2) FP32 product (v_mfma_f32_32x32x2f32), half the
// multiply-adds of the plain convolution.  A (weighted inputs) is staged in
// LDS per 32-input step; B is read from the 1-D table of G_p's diagonals.

typedef float fdk_v16f __attribute__((ext_vector_type(16)));

constexpr int kMmRows = 64;   // detector rows per workgroup (2 waves of 32)
constexpr int kMmCols = 128;  // outputs of one parity per workgroup (2 waves of 2 x 32)
constexpr int kMmK = 32;      // inputs staged per step

// Parker weight of every (view, column).
__global__ __launch_bounds__(256) void fdk_parker_kernel(const FdkView *__restrict__ views, int n_views, int W,
                                                         float *__restrict__ pw) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_views * W) return;
    const FdkView vw = views[idx / W];
    const float du = (float)(idx % W) - vw.u0;
    pw[idx] = parker(vw.beta, -atanf(du / vw.f), vw.delta);
}

// Weighted inputs x(r, k) = p(r, k) * cosine weight * Parker weight, split by
// column parity: X_even[r][j] = x(r, 2j) ([N H][ceil(W / 2)]) and
// X_odd[r][j] = x(r, 2j + 1) ([N H][floor(W / 2)]), so the products read
// contiguous rows.
__global__ __launch_bounds__(256) void fdk_weight_kernel(const float *__restrict__ images,
                                                         const FdkView *__restrict__ views,
                                                         const float *__restrict__ pw, int W, int H,
                                                         float *__restrict__ x_even, float *__restrict__ x_odd) {
    const int k = blockIdx.y * blockDim.x + threadIdx.x;
    const int64_t r = blockIdx.x;  // view * H + v
    if (k >= W) return;
    const int view = (int)(r / H), v = (int)(r % H);
    const FdkView vw = views[view];
    const float du = (float)k - vw.u0, dv = (float)v - vw.v0;
    const float cosw = vw.f * rsqrtf(vw.f * vw.f + du * du + dv * dv);
    const float x = images[r * W + k] * cosw * pw[(int64_t)view * W + k];
    if (k & 1) x_odd[r * (W / 2) + (k >> 1)] = x;
    else x_even[r * ((W + 1) / 2) + (k >> 1)] = x;
}

// Workgroups: (parity, row tile, column tile), numbered with the column tile
// fastest and dealt so that each XCD takes a contiguous range: the column
// tiles of one row tile share its inputs in the XCD's L2.  Dynamic LDS: the
// diagonals of G_p, W - 1 floats.
__global__ __launch_bounds__(256) void fdk_filter_mfma_kernel(const float *__restrict__ x_even,
                                                              const float *__restrict__ x_odd,
                                                              const FdkView *__restrict__ views, int n_views, int W,
                                                              int H, int row_tiles, int col_tiles,
                                                              float2 *__restrict__ Qi) {
    __shared__ float As[kMmRows][kMmK + 1];
    extern __shared__ float gs[];
    const int total = 2 * row_tiles * col_tiles;
    const int per = (total + 7) / 8;
    const int t = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (t >= total) return;  // before any barrier
    const int p = t / (row_tiles * col_tiles), rem = t % (row_tiles * col_tiles);
    const int row_tile = rem / col_tiles, col_tile = rem % col_tiles;
    const int q = 1 - p;
    const int Wp = (W + 1 - p) / 2, Wq = (W + 1 - q) / 2;  // outputs of parity p, inputs of parity q
    const int64_t n_rows = (int64_t)n_views * H;
    const float *xq = q ? x_odd : x_even;  // [n_rows][Wq]
    const float *xp = p ? x_odd : x_even;  // [n_rows][Wp]
    // g[d + Wq - 1] = h(2d + 2p - 1), d = i - j in [-(Wq - 1), Wp - 1]
    for (int e = threadIdx.x; e < Wp + Wq - 1; e += blockDim.x) {
        const float n = (float)(2 * (e - (Wq - 1)) + 2 * p - 1);
        gs[e] = -1.0f / (kPiF * kPiF * n * n);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int64_t r_base = (int64_t)row_tile * kMmRows;
    const int i_base = col_tile * kMmCols + 64 * wc;
    fdk_v16f acc0 = {0}, acc1 = {0};
    // each thread stages 8 inputs of a step; the next step's are loaded into
    // registers while this step's products run
    constexpr int kPer = kMmRows * kMmK / 256;
    float pre[kPer];
    auto load_step = [&](int j0) {
#pragma unroll
        for (int e8 = 0; e8 < kPer; ++e8) {
            const int e = threadIdx.x + 256 * e8;
            const int64_t r = r_base + e / kMmK;
            const int j = j0 + e % kMmK;
            pre[e8] = (r < n_rows && j < Wq) ? xq[r * Wq + j] : 0.0f;
        }
    };
    load_step(0);
    for (int j0 = 0; j0 < Wq; j0 += kMmK) {
        __syncthreads();  // the previous step's reads of As are done (and gs is written)
#pragma unroll
        for (int e8 = 0; e8 < kPer; ++e8) {
            const int e = threadIdx.x + 256 * e8;
            As[e / kMmK][e % kMmK] = pre[e8];
        }
        __syncthreads();
        if (j0 + kMmK < Wq) load_step(j0 + kMmK);
#pragma unroll 4
        for (int kk = 0; kk < kMmK; kk += 2) {
            const float a = As[32 * wr + (lane & 31)][kk + (lane >> 5)];
            const int j = j0 + kk + (lane >> 5);
            const int i0 = i_base + (lane & 31), i1 = i0 + 32;
            const bool jok = j < Wq;
            const float b0 = (jok && i0 < Wp) ? gs[i0 - j + Wq - 1] : 0.0f;
            const float b1 = (jok && i1 < Wp) ? gs[i1 - j + Wq - 1] : 0.0f;
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b1, acc1, 0, 0, 0);
        }
    }
    // outputs: register e of lane l holds row 8 (e / 4) + 4 (l / 32) + e % 4,
    // column l % 32 of the wave's 32 x 32 block
    const int WP = W + 4;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int64_t r = r_base + 32 * wr + 8 * (e / 4) + 4 * (lane >> 5) + (e % 4);
        if (r >= n_rows) continue;
        const int view = (int)(r / H), v = (int)(r % H);
        const FdkView &vw = views[view];
        const float out_scale = vw.inv_tau * vw.scale;
        float2 *row_x = Qi + ((int64_t)view * (H + 3) + (v + 2)) * WP;
        float2 *row_y = Qi + ((int64_t)view * (H + 3) + (v + 1)) * WP;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = (h == 0 ? i_base : i_base + 32) + (lane & 31);
            if (i >= Wp) continue;
            const int u = 2 * i + p;
            const float acc = h == 0 ? acc0[e] : acc1[e];
            const float qv = fmaf(0.25f, xp[r * Wp + i], acc) * out_scale;
            row_x[u + 2].x = qv;
            row_y[u + 2].y = qv;
        }
    }
}

// The zero border of the interleaved filtered views: columns 0, 1, W + 2,
// W + 3 of every row pair, and the pair halves that hold rows Qp[0], Qp[1],
// Qp[H + 2], Qp[H + 3].
__global__ __launch_bounds__(256) void fdk_border_kernel(int n_views, int W, int H, float2 *__restrict__ Qi) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int WP = W + 4;
    const int64_t n_cols = (int64_t)n_views * (H + 3) * 4;
    if (idx < n_cols) {
        const int64_t vr = idx / 4;  // view * (H + 3) + r
        const int c = (int)(idx % 4);
        Qi[vr * WP + (c < 2 ? c : W + c)] = make_float2(0.0f, 0.0f);
        return;
    }
    const int64_t k = idx - n_cols;
    if (k >= (int64_t)n_views * W) return;
    const int64_t view = k / W;
    const int c = (int)(k % W) + 2;
    float2 *base = Qi + view * (H + 3) * WP;
    base[c] = make_float2(0.0f, 0.0f);                        // pair 0: Qp[0], Qp[1]
    base[WP + c].x = 0.0f;                                     // pair 1: Qp[1]
    base[(int64_t)(H + 1) * WP + c].y = 0.0f;                  // pair H + 1: Qp[H + 2]
    base[(int64_t)(H + 2) * WP + c] = make_float2(0.0f, 0.0f);  // pair H + 2: Qp[H + 2], Qp[H + 3]
}

constexpr int kBpTile = 16;   // voxel columns per workgroup side
constexpr int kBpSlab = 16;   // slices per thread
// LDS window of one view: up to kBpRows pair rows x kBpCols pair elements,
// wave w staging rows w, w + 4, ... (one element per lane).  Rows are
// kBpPitch elements apart, so that the rows of a gather start on different
// LDS banks.
constexpr int kBpCols = 64;
constexpr int kBpRows = 56;
constexpr int kBpPitch = 66;
constexpr int kBpPer = kBpRows / 4;  // rows each wave stages per view
constexpr int kBpWinChunk = 256;     // views whose windows are computed together

// Cell of a padded-view coordinate x: returns the fraction x - floor(x) and
// sets i = floor(x) clamped to [0, hi] (one floor-and-convert instruction on
// the clamped value).  Coordinates are finite: the voxel's projection with
// the reciprocal depth set to 0 behind the source.
__device__ __forceinline__ float bp_cell(float x, float hi, int &i) {
    const float xc = __builtin_amdgcn_fmed3f(x, 0.0f, hi);
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(i) : "v"(xc));
    return __builtin_amdgcn_fractf(x);
}

// The part of one padded filtered view that a workgroup's 16 x 16 x 16 voxel
// box reads: element rows [v_lo, v_lo + rows) x columns [u_lo, u_lo + cols), returned as
// (u_lo, v_lo, rows, cols).
// The box lies in front of the source, so its projection is the convex hull
// of its 8 corner voxels' projections.  One cell of margin on each side
// covers the rounding of the per-voxel coordinates; the cell indices are
// clamped as the per-voxel ones, and the window takes one more column for a
// cell's second column (also when the whole box projects past the
// detector's edge).  cols = 0 when a corner is not in front of the source or
// the window exceeds the LDS tile (the view is then read directly).
__device__ __forceinline__ int4 bp_window(const FdkView &w, float xb, float yb, float zb, float ext, int W,
                                            int H) {
    float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY, cmin = INFINITY;
#pragma unroll
    for (int corner = 0; corner < 8; ++corner) {
        const float X = (corner & 1) ? xb + ext : xb, Y = (corner & 2) ? yb + ext : yb;
        const float Z = (corner & 4) ? zb + ext : zb;
        const float a = fmaf(w.P[0], X, fmaf(w.P[1], Y, fmaf(w.P[2], Z, w.P[3])));
        const float b = fmaf(w.P[4], X, fmaf(w.P[5], Y, fmaf(w.P[6], Z, w.P[7])));
        const float c = fmaf(w.P[8], X, fmaf(w.P[9], Y, fmaf(w.P[10], Z, w.P[11])));
        const float rc = c > 0.0f ? __builtin_amdgcn_rcpf(c) : 0.0f;
        const float u = fmaf(a, rc, w.u0 + 2.0f), v = fmaf(b, rc, w.v0 + 2.0f);
        umin = fminf(umin, u);
        umax = fmaxf(umax, u);
        vmin = fminf(vmin, v);
        vmax = fmaxf(vmax, v);
        cmin = fminf(cmin, c);
    }
    const float ulo = __builtin_amdgcn_fmed3f(floorf(umin) - 1.0f, 0.0f, (float)(W + 2));
    const float uhi = __builtin_amdgcn_fmed3f(floorf(umax) + 1.0f, 0.0f, (float)(W + 2)) + 1.0f;
    const float vlo = __builtin_amdgcn_fmed3f(floorf(vmin) - 1.0f, 0.0f, (float)(H + 2));
    const float vhi = __builtin_amdgcn_fmed3f(floorf(vmax) + 1.0f, 0.0f, (float)(H + 2));
    const bool fits = cmin > 0.0f && uhi - ulo < (float)kBpCols && vhi - vlo < (float)kBpRows;
    if (!fits) return make_int4(0, 0, 0, 0);
    return make_int4((int)ulo, (int)vlo, (int)(vhi - vlo + 1.0f), (int)(uhi - ulo + 1.0f));
}

// Workgroups are numbered so that each XCD (8 per chip, blocks dealt to them
// round-robin) takes one contiguous range of tiles, x fastest then y then z:
// a z-slab of the volume, whose footprint in every view is a band of rows.
//
// Each view's window is loaded once per workgroup into LDS (loads for view
// j + 1 in flight in registers while view j is computed) and every voxel
// reads its cells there: a window element serves about five updates, which
// otherwise each fetch a cache line of their own from L2.  Views whose
// window does not fit read the filtered view directly.
__global__ __launch_bounds__(256) void fdk_backproject_kernel(const float2 *__restrict__ Qi,
                                                              const FdkView *__restrict__ views, int n_views,
                                                              int W, int H, FdkVolume vol, int tiles_x, int tiles_y,
                                                              int n_tiles, float *__restrict__ out) {
    __shared__ float2 win_lds[kBpRows * kBpPitch];
    __shared__ int4 wins[2][kBpWinChunk];  // windows of two chunks of views
    const int per = (n_tiles + 7) / 8;
    const int tile = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (tile >= n_tiles) return;  // no barrier has been reached yet
    const int tx = tile % tiles_x, ty = (tile / tiles_x) % tiles_y, tz = tile / (tiles_x * tiles_y);
    // each wave takes an 8 x 8 quarter of the 16 x 16 tile: its 64 voxel
    // columns project onto a compact detector patch
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ix = tx * kBpTile + (wave & 1) * 8 + (lane & 7);
    const int iy = ty * kBpTile + (wave >> 1) * 8 + (lane >> 3);
    const int iz0 = tz * kBpSlab;
    const float s = vol.voxel_mm;
    const float hx = 0.5f * (float)(vol.nx - 1), hy = 0.5f * (float)(vol.ny - 1), hz = 0.5f * (float)(vol.nz - 1);
    const float x = ((float)ix - hx) * s;
    const float y = ((float)iy - hy) * s;
    const float z0 = ((float)iz0 - hz) * s;
    // the workgroup's voxel box (centres of its corner voxels)
    const float xb = ((float)(tx * kBpTile) - hx) * s, yb = ((float)(ty * kBpTile) - hy) * s;
    const float ext = (float)(kBpTile - 1) * s;
    static_assert(kBpTile == kBpSlab, "the window's box is a cube");
    const uint32_t WP = (uint32_t)W + 4;
    const int64_t view_elems = (int64_t)(H + 3) * WP;
    // cell coordinates in the padded view (detector column u at u + 2, row v
    // at pair row v + 2): cells past the detector are clamped into the
    // two-wide zero border, where all four taps read zero
    const float u_hi = (float)(W + 2), v_hi = (float)(H + 2);
    float acc[kBpSlab];
#pragma unroll
    for (int k = 0; k < kBpSlab; ++k) acc[k] = 0.0f;
    // staging: wave w moves window rows w + 4 i, lane l their column l
    const int sw = __builtin_amdgcn_readfirstlane(wave);
    float2 pre[kBpPer];
    auto prefetch = [&](const int4 &wn, int view) {
        const float2 *src = Qi + view * view_elems + (int64_t)(wn.y + sw) * WP + wn.x;
        if (lane < wn.w) {
#pragma unroll
            for (int i = 0; i < kBpPer; ++i)
                if (sw + 4 * i < wn.z) pre[i] = src[(uint32_t)(4 * i) * WP + lane];
        }
    };
    auto stage = [&](const int4 &wn) {
        if (lane < wn.w) {
#pragma unroll
            for (int i = 0; i < kBpPer; ++i)
                if (sw + 4 * i < wn.z) win_lds[(sw + 4 * i) * kBpPitch + lane] = pre[i];
        }
    };
    // windows of views [c kBpWinChunk, (c + 1) kBpWinChunk), one per thread
    auto chunk_windows = [&](int c) {
        const int v = c * kBpWinChunk + (int)threadIdx.x;
        if (v < n_views) wins[c & 1][threadIdx.x] = bp_window(views[v], xb, yb, z0, ext, W, H);
    };
    auto window_of = [&](int v) {
        const int4 r = wins[(v / kBpWinChunk) & 1][v % kBpWinChunk];
        return make_int4(__builtin_amdgcn_readfirstlane(r.x), __builtin_amdgcn_readfirstlane(r.y),
                         __builtin_amdgcn_readfirstlane(r.z), __builtin_amdgcn_readfirstlane(r.w));
    };
    // bilinear value of cell (iu, iv) at fractions (fu, fv), from the window
    // (FROM_LDS) or from the view
    auto bilerp = [](const fdk_f32x4_a8 &t, float fu, float fv) {
        const float top = fmaf(fu, t.z - t.x, t.x);
        const float bot = fmaf(fu, t.w - t.y, t.y);
        return fmaf(fv, bot - top, top);
    };
    // the updates of one view; FROM_LDS is the same for the whole workgroup
    auto view_updates = [&](const FdkView &w, const float2 *q, const int4 &wn, auto from_lds) {
        constexpr bool FROM_LDS = decltype(from_lds)::value;
        auto cell = [&](int iu, int iv, float fu, float fv) {
            fdk_f32x4_a8 t;
            if (FROM_LDS) {
                t = *(const fdk_f32x4_a8 *)(win_lds + ((iv - wn.y) * kBpPitch + (iu - wn.x)));
            } else {
                const uint32_t e = __umul24((uint32_t)iv, WP) + (uint32_t)iu;
                t = *(const fdk_f32x4_a8 *)((const char *)q + e * (uint32_t)sizeof(float2));
            }
            return bilerp(t, fu, fv);
        };
        const float a0 = fmaf(w.P[0], x, fmaf(w.P[1], y, fmaf(w.P[2], z0, w.P[3])));
        const float b0 = fmaf(w.P[4], x, fmaf(w.P[5], y, fmaf(w.P[6], z0, w.P[7])));
        const float c0 = fmaf(w.P[8], x, fmaf(w.P[9], y, fmaf(w.P[10], z0, w.P[11])));
        const float db = w.P[6] * s;
        const float u0p = w.u0 + 2.0f, v0p = w.v0 + 2.0f;
        if (w.P[2] == 0.0f && w.P[10] == 0.0f) {
            // the view's column and depth do not change along z (a circular
            // orbit about z, moved by translations and rotations about z):
            // column, weight and reciprocal once per voxel column, only the
            // row moves.  The values equal the general branch's, whose z
            // terms vanish exactly.
            const float rc = c0 > 0.0f ? __builtin_amdgcn_rcpf(c0) : 0.0f;
            const float wgt = rc * rc;
            int iu;
            const float fu = bp_cell(fmaf(a0, rc, u0p), u_hi, iu);
#pragma unroll
            for (int k = 0; k < kBpSlab; ++k) {
                int iv;
                const float fv = bp_cell(fmaf(fmaf((float)k, db, b0), rc, v0p), v_hi, iv);
                acc[k] = fmaf(wgt, cell(iu, iv, fu, fv), acc[k]);
            }
        } else {
            const float da = w.P[2] * s, dc = w.P[10] * s;
#pragma unroll
            for (int k = 0; k < kBpSlab; ++k) {
                const float a = fmaf((float)k, da, a0);
                const float b = fmaf((float)k, db, b0);
                const float c = fmaf((float)k, dc, c0);
                // a point behind the source counts zero (rc = 0 also keeps
                // its coordinates finite)
                const float rc = c > 0.0f ? __builtin_amdgcn_rcpf(c) : 0.0f;
                int iu, iv;
                const float fu = bp_cell(fmaf(a, rc, u0p), u_hi, iu);
                const float fv = bp_cell(fmaf(b, rc, v0p), v_hi, iv);
                acc[k] = fmaf(rc * rc, cell(iu, iv, fu, fv), acc[k]);
            }
        }
    };
    chunk_windows(0);
    __syncthreads();
    int4 next = window_of(0);
    if (next.w) prefetch(next, 0);
    for (int j = 0; j < n_views; ++j) {
        const FdkView &w = views[j];
        const int4 cur = next;
        // the next chunk's windows, written to the buffer whose last reads
        // (views of the chunk before this one) ended two barriers ago; the
        // barrier below orders them before their first read
        if (j % kBpWinChunk == 0) chunk_windows(j / kBpWinChunk + 1);
        __syncthreads();  // every wave is done with the previous window
        if (cur.w) stage(cur);
        __syncthreads();
        if (j + 1 < n_views) {
            next = window_of(j + 1);
            if (next.w) prefetch(next, j + 1);
        }
        const float2 *q = Qi + j * view_elems;
        if (cur.w)
            view_updates(w, q, cur, std::true_type{});
        else
            view_updates(w, q, cur, std::false_type{});
    }
    if (ix >= vol.nx || iy >= vol.ny) return;
#pragma unroll
    for (int k = 0; k < kBpSlab; ++k) {
        const int iz = iz0 + k;
        if (iz < vol.nz) out[((int64_t)iz * vol.ny + iy) * vol.nx + ix] = acc[k];
    }
}

hipError_t launch_fdk(const float *images, const ViewGeom *nominal, const ViewGeom *moved, int n_views, int W,
                      int H, FdkVolume vol, FdkView *views, float *pw, float *xw, float2 *Qi, float *out,
                      hipStream_t s) {
    hipLaunchKernelGGL(fdk_view_kernel, dim3((n_views + 255) / 256), dim3(256), 0, s, nominal, moved, n_views,
                       views);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n_pw = (int64_t)n_views * W;
    hipLaunchKernelGGL(fdk_parker_kernel, dim3((unsigned)((n_pw + 255) / 256)), dim3(256), 0, s,
                       (const FdkView *)views, n_views, W, pw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t n_border = (int64_t)n_views * (H + 3) * 4 + n_pw;
    hipLaunchKernelGGL(fdk_border_kernel, dim3((unsigned)((n_border + 255) / 256)), dim3(256), 0, s, n_views, W, H,
                       Qi);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    float *x_even = xw, *x_odd = xw + (int64_t)n_views * H * ((W + 1) / 2);
    hipLaunchKernelGGL(fdk_weight_kernel, dim3((unsigned)((int64_t)n_views * H), (W + 255) / 256), dim3(256), 0, s,
                       images,
                       (const FdkView *)views, (const float *)pw, W, H, x_even, x_odd);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int row_tiles = (int)(((int64_t)n_views * H + kMmRows - 1) / kMmRows);
    const int col_tiles = ((W + 1) / 2 + kMmCols - 1) / kMmCols;
    const int total = 2 * row_tiles * col_tiles;
    hipLaunchKernelGGL(fdk_filter_mfma_kernel, dim3((unsigned)(8 * ((total + 7) / 8))), dim3(256),
                       sizeof(float) * W, s, (const float *)x_even, (const float *)x_odd, (const FdkView *)views,
                       n_views, W, H, row_tiles, col_tiles, Qi);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int tiles_x = (vol.nx + kBpTile - 1) / kBpTile, tiles_y = (vol.ny + kBpTile - 1) / kBpTile;
    const int n_tiles = tiles_x * tiles_y * ((vol.nz + kBpSlab - 1) / kBpSlab);
    const int blocks = 8 * ((n_tiles + 7) / 8);
    hipLaunchKernelGGL(fdk_backproject_kernel, dim3(blocks), dim3(kBpTile * kBpTile), 0, s, (const float2 *)Qi,
                       (const FdkView *)views, n_views, W, H, vol, tiles_x, tiles_y, n_tiles, out);
    return hipGetLastError();
}

}  // namespace ecc
