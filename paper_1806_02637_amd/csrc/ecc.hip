// Epipolar-consistency cost on gfx950 (arxiv 1806.02637, Eqs. 13-17).
//
// view_setup   one thread per (hypothesis, view): P' = P T(theta) and its
//              source (Eqs. 4-5), FP64; optionally dP'/dtheta for the adjoint.
// ecc_fwd      a workgroup = 4 waves = 4 hypotheses of one tile of 64 view
//              pairs.  Lane j of a wave first builds pair j's geometry in FP64
//              (baseline, pencil of planes, the two line maps of Eq. 14) into
//              LDS; the wave then walks its 64 pairs with lanes along the plane
//              angle kappa: line -> (alpha, t) -> four bilinear taps per view
//              in one load -> (S_a - S_b)^2 -> wave-shuffle sum (Eq. 15) ->
//              Cauchy norm (Eq. 16).  No atomics; per-tile FP64 partials.
// reduce_cost  fixed-order sum of the tile partials per hypothesis (Eq. 17).
//
// Blocks are numbered so that each of the 8 XCDs (which receive workgroups
// round-robin) walks a contiguous run of tiles with the hypotheses of a tile
// back to back, keeping a tile's sinogram rows in that XCD's L2.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ecc_internal.hpp"
#include "lookup.hpp"
#include "pair.hpp"
#include "projective.hpp"

namespace ecc {

// ---------------------------------------------------------------------------
__device__ __forceinline__ void mat3_mul(const double A[9], const double B[9], double C[9]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

__global__ __launch_bounds__(256) void view_setup_kernel(const double *__restrict__ P, const double *__restrict__ intr,
                                                         const double *__restrict__ theta, int B, int n_views,
                                                         ViewGeom *__restrict__ vt, ViewGeomGrad *__restrict__ vg) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * n_views) return;
    const int v = idx % n_views;
    const double *th = theta + (int64_t)idx * 6;
    const double deg = 3.14159265358979323846 / 180.0;
    double c[3], s[3];
    for (int i = 0; i < 3; ++i) sincos(th[i] * deg, &s[i], &c[i]);
    // R = Rz Ry Rx and the three partial derivatives
    const double Rx[9] = {1, 0, 0, 0, c[0], -s[0], 0, s[0], c[0]};
    const double Ry[9] = {c[1], 0, s[1], 0, 1, 0, -s[1], 0, c[1]};
    const double Rz[9] = {c[2], -s[2], 0, s[2], c[2], 0, 0, 0, 1};
    double RyRx[9], R[9];
    mat3_mul(Ry, Rx, RyRx);
    mat3_mul(Rz, RyRx, R);
    const double *Pv = P + (int64_t)v * 12;
    ViewGeom g;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            g.P[4 * i + j] = Pv[4 * i] * R[j] + Pv[4 * i + 1] * R[3 + j] + Pv[4 * i + 2] * R[6 + j];
        g.P[4 * i + 3] = Pv[4 * i] * th[3] + Pv[4 * i + 1] * th[4] + Pv[4 * i + 2] * th[5] + Pv[4 * i + 3];
    }
    source_position(g.P, g.C);
    g.f = intr[3 * v];
    g.u0 = intr[3 * v + 1];
    g.v0 = intr[3 * v + 2];
    g.pad[0] = g.pad[1] = 0.0;
    vt[idx] = g;
    if (vg) {
        const double dRx[9] = {0, 0, 0, 0, -s[0] * deg, -c[0] * deg, 0, c[0] * deg, -s[0] * deg};
        const double dRy[9] = {-s[1] * deg, 0, c[1] * deg, 0, 0, 0, -c[1] * deg, 0, -s[1] * deg};
        const double dRz[9] = {-s[2] * deg, -c[2] * deg, 0, c[2] * deg, -s[2] * deg, 0, 0, 0, 0};
        double dR[3][9], tmp[9];
        mat3_mul(Ry, dRx, tmp);
        mat3_mul(Rz, tmp, dR[0]);
        mat3_mul(dRy, Rx, tmp);
        mat3_mul(Rz, tmp, dR[1]);
        mat3_mul(dRz, RyRx, dR[2]);
        ViewGeomGrad gg;
        for (int q = 0; q < 6; ++q) {
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j)
                    gg.dP[q][4 * i + j] =
                        q < 3 ? Pv[4 * i] * dR[q][j] + Pv[4 * i + 1] * dR[q][3 + j] + Pv[4 * i + 2] * dR[q][6 + j] : 0.0;
                gg.dP[q][4 * i + 3] = q < 3 ? 0.0 : Pv[4 * i + (q - 3)];
            }
            Dual Pd[12], Cd[3];
            for (int e = 0; e < 12; ++e) Pd[e] = Dual(g.P[e], gg.dP[q][e]);
            source_position(Pd, Cd);
            for (int e = 0; e < 3; ++e) gg.dC[q][e] = Cd[e].d;
        }
        vg[idx] = gg;
    }
}

hipError_t launch_view_setup(const double *P, const double *intr, const double *theta, int B, int n_views,
                             ViewGeom *vt, ViewGeomGrad *vg, hipStream_t s) {
    const int n = B * n_views;
    hipLaunchKernelGGL(view_setup_kernel, dim3((n + 255) / 256), dim3(256), 0, s, P, intr, theta, B, n_views, vt, vg);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <class Tap, class G>
__global__ __launch_bounds__(256) void ecc_fwd_kernel(const void *__restrict__ sino, const float *__restrict__ vscale,
                                                      const ViewGeom *__restrict__ vt, EvalConsts ec,
                                                      float *__restrict__ out_pair, double *__restrict__ partials,
                                                      int n_tiles) {
    __shared__ PairConst<G> lds[kWavesPerBlock][kPairsPerWave];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int hyp_groups = (ec.B + kWavesPerBlock - 1) / kWavesPerBlock;
    const int64_t total = (int64_t)n_tiles * hyp_groups;
    const int64_t w = xcd_work_item(total);
    if (w >= total) return;  // whole block
    const int tile = (int)(w / hyp_groups);
    const int hyp = (int)(w % hyp_groups) * kWavesPerBlock + wave;
    const bool active = hyp < ec.B;
    const int64_t p0 = (int64_t)tile * kPairsPerWave;
    const int np = (int)min((int64_t)kPairsPerWave, (int64_t)ec.n_pairs - p0);

    if (active && lane < np) {
        int a, b;
        pair_from_index(p0 + lane, ec.n_views, a, b);
        PairConst<G> pc;
        pair_setup<G>(vt[(int64_t)hyp * ec.n_views + a], vt[(int64_t)hyp * ec.n_views + b], ec.R_mm, ec.K, pc);
        pc.va = a;
        pc.vb = b;
        pc.sa = vscale[a];
        pc.sb = vscale[b];
        lds[wave][lane] = pc;
    }
    __syncthreads();
    if (!active) return;

    const Tap *base = (const Tap *)sino;
    double wave_acc = 0.0;
    for (int q = 0; q < np; ++q) {
        const PairConst<G> &pc = lds[wave][q];
        const Tap *sa = base + (int64_t)pc.va * ec.view_elems;
        const Tap *sb = base + (int64_t)pc.vb * ec.view_elems;
        float acc = 0.0f;
        int cnt = 0;
        for (int k = lane; k < ec.K; k += 64) {
            G sn, cs;
            g_sincos(pc.k0 + (G)k * pc.dk, &sn, &cs);
            bool hit_a, hit_b;
            const float Sa = lookup<Tap, G>(pc.ha, cs, sn, sa, ec, pc.inv_f2a, pc.sa, hit_a);
            const float Sb = lookup<Tap, G>(pc.hb, cs, sn, sb, ec, pc.inv_f2b, pc.sb, hit_b);
            if (hit_a && hit_b) {
                const float diff = Sa - Sb;
                acc = fmaf(diff, diff, acc);
                ++cnt;
            }
        }
        acc = wave_sum(acc);
        cnt = wave_sum_i(cnt);
        const float d = cnt > 0 ? acc / (float)cnt : 0.0f;
        const float e = ec.inv_c > 0.0f ? d / (1.0f + d * ec.inv_c) : d;
        if (out_pair && lane == 0) out_pair[(int64_t)hyp * ec.n_pairs + p0 + q] = e;
        wave_acc += (double)e;
    }
    if (lane == 0) partials[(int64_t)hyp * n_tiles + tile] = wave_acc;
}

template <class Tap, class G>
static hipError_t launch_fwd_t(const void *sino, const float *vscale, const ViewGeom *vt, EvalConsts ec,
                               float *out_pair, double *partials, int n_tiles, hipStream_t s) {
    const int64_t total = (int64_t)n_tiles * ((ec.B + kWavesPerBlock - 1) / kWavesPerBlock);
    const int64_t blocks = 8 * ((total + 7) / 8);
    hipLaunchKernelGGL((ecc_fwd_kernel<Tap, G>), dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0, s, sino,
                       vscale, vt, ec, out_pair, partials, n_tiles);
    return hipGetLastError();
}

hipError_t launch_ecc_fwd(const void *sino, const float *view_scale, const ViewGeom *vt, EvalConsts ec, int dtype,
                          float *out_pair, double *partials, int n_tiles, hipStream_t s) {
    if (ec.geom64) {
        if (dtype == 0) return launch_fwd_t<TapF32, double>(sino, view_scale, vt, ec, out_pair, partials, n_tiles, s);
        if (dtype == 1) return launch_fwd_t<TapBF16, double>(sino, view_scale, vt, ec, out_pair, partials, n_tiles, s);
        return launch_fwd_t<TapF16, double>(sino, view_scale, vt, ec, out_pair, partials, n_tiles, s);
    }
    if (dtype == 0) return launch_fwd_t<TapF32, float>(sino, view_scale, vt, ec, out_pair, partials, n_tiles, s);
    if (dtype == 1) return launch_fwd_t<TapBF16, float>(sino, view_scale, vt, ec, out_pair, partials, n_tiles, s);
    return launch_fwd_t<TapF16, float>(sino, view_scale, vt, ec, out_pair, partials, n_tiles, s);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void reduce_cost_kernel(const double *__restrict__ partials, int n_tiles,
                                                          double *__restrict__ out_cost) {
    __shared__ double red[256];
    const int hyp = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n_tiles; i += 256) acc += partials[(int64_t)hyp * n_tiles + i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out_cost[hyp] = red[0];
}

hipError_t launch_reduce_cost(const double *partials, int n_tiles, int B, double *out_cost, hipStream_t s) {
    hipLaunchKernelGGL(reduce_cost_kernel, dim3(B), dim3(256), 0, s, partials, n_tiles, out_cost);
    return hipGetLastError();
}

}  // namespace ecc
