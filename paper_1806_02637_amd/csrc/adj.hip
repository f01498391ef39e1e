// Adjoint of the consistency cost: d cost / d theta for every view's six
// motion parameters, with the line geometry recomputed rather than stored.
//
// ecc_adj       same work split as the forward kernel (one hypothesis x one
//               work tile per workgroup, its pairs shared by the four
//               waves).  Per pair:
//                 1. forward sweep over the K planes -> d, N (Eq. 15), e (Eq. 16);
//                 2. reverse sweep over the planes: dE/dS_a = +g, dE/dS_b = -g with
//                    g = de/dd * 2 (S_a - S_b) / N on planes hitting both
//                    detectors; through the weighted bilinear lookup to
//                    (alpha, t), through atan2 / offset to the line l, through
//                    l = H (cos k, sin k) to the 6 + 6 line-map entries and to
//                    the sampled arc: kappa_max for the object-sphere range
//                    (k = kappa_max ((2k+1)/K - 1)), or its two ends lo, hi for
//                    the detector-bounded range (k = lo + (k+1/2)(hi - lo)/K);
//                    fixed-order wave sums of those 14 sensitivities, written
//                    per pair.
// pair_grad     one thread per (hypothesis, pair): the 14 sensitivities taken
//               back through the pair's geometry in FP64 (one reverse sweep:
//               line maps -> rows of M = P'[:, 0:3] and the pencil's u1, u2,
//               kappa_max -> the two sources), then contracted with each of
//               the 12 motion parameters' dP'/dtheta and dC/dtheta.  A
//               detector arc's end moves as the zero angle of the corner that
//               fixes it, atan2(-A_c, B_c) with (A_c, B_c) the two basis
//               lines' values at the corner.
// reduce_grad   fixed-order sum of the per-pair 12-vectors into grad[B][N][6].
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ecc_internal.hpp"
#include "lookup.hpp"
#include "pair.hpp"
#include "pair_adjoint.hpp"
#include "projective.hpp"

namespace ecc {

// Reverse sweep through one view's lookup: accumulates dE/dH (6) given
// gS = dE/dS, and the same terms weighted by u (the plane's position in its
// range), from which the plane-angle sensitivities follow once per pair.
// With the folded line l' (the fold sign cancels in dS/dl), r = |(l1', l2')|,
// n = (l1', l2') / r, alpha = atan2(l2', l1') and t = -l3' / r:
//   dalpha/dl' = (-n2, n1, 0) / r,   dt/dl' = -(t n1, t n2, 1) / r,
// so with A = gS dS/dalpha / r and T = gS dS/dt / r:
//   dE/dl' = (-(A n2 + T t n1), A n1 - T t n2, -T).
template <class Tap, class G>
__device__ __forceinline__ void lookup_adjoint(G cs, G sn, const Taps &tp, const EvalConsts &ec, float inv_f2,
                                               float scale, float gS, const LineCoord<G> &c, float u, float gH[6],
                                               float gHu[6]) {
    const float d0 = tp.s01 - tp.s00, d1 = tp.s11 - tp.s10;
    const float r0 = fmaf(c.ft, d0, tp.s00);
    const float r1 = fmaf(c.ft, d1, tp.s10);
    const float Bv = fmaf(c.fa, r1 - r0, r0);
    const float x = c.tf * inv_f2;
    const float w = fmaf(c.tf, x, 1.0f);
    // S = sgn * scale * w(t) * B(alpha, t): dS/dalpha, dS/dt (without scale)
    const float dS_dalpha = w * (r1 - r0) * ec.inv_dalpha;
    const float dS_dt = fmaf(2.0f * x, Bv, w * ec.inv_dt * fmaf(c.fa, d1 - d0, d0));
    const float rinv = (float)c.rinv;
    const float gr = Tap::kScaled ? gS * scale * rinv : gS * rinv;
    const float A = gr * dS_dalpha, T = gr * dS_dt;
    const float Tt = T * c.tf;
    const float n1 = (float)c.l1 * rinv, n2 = (float)c.l2 * rinv;
    const float gl1 = -fmaf(A, n2, Tt * n1);
    const float gl2 = fmaf(A, n1, -(Tt * n2));
    const float gl3 = -T;
    const float fc = (float)cs, fs = (float)sn;
    gH[0] = fmaf(gl1, fc, gH[0]);
    gH[1] = fmaf(gl2, fc, gH[1]);
    gH[2] = fmaf(gl3, fc, gH[2]);
    gH[3] = fmaf(gl1, fs, gH[3]);
    gH[4] = fmaf(gl2, fs, gH[4]);
    gH[5] = fmaf(gl3, fs, gH[5]);
    const float uc = u * fc, us = u * fs;
    gHu[0] = fmaf(gl1, uc, gHu[0]);
    gHu[1] = fmaf(gl2, uc, gHu[1]);
    gHu[2] = fmaf(gl3, uc, gHu[2]);
    gHu[3] = fmaf(gl1, us, gHu[3]);
    gHu[4] = fmaf(gl2, us, gHu[4]);
    gHu[5] = fmaf(gl3, us, gHu[5]);
}

// Sum over planes of gk dl/dkappa . dE/dl with dl/dkappa = H (-sin, cos):
// from the accumulated sums G_c = sum gl cos, G_s = sum gl sin,
//   sum gk = H_s . G_c - H_c . G_s   (H_c = h[0..2], H_s = h[3..5]).
template <class G>
__device__ __forceinline__ float kappa_sum(const G h[6], const float gH[6]) {
    float r = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) r = fmaf((float)h[3 + i], gH[i], fmaf(-(float)h[i], gH[3 + i], r));
    return r;
}


// Sums of 16 per-lane values over the wave at once, in a fixed order:
// swap-and-add across the wave's halves (v_permlane32_swap: a value's lanes
// 32-63 trade places with another's lanes 0-31, so one add leaves value i in
// lanes 0-31 and value i + 8 in lanes 32-63, each summed over lanes l and
// l + 32), the same within each half (v_permlane16_swap), then across 8 and
// 4 lanes of a row (DPP rotate by 8, half-row mirror, the lane's bit choosing
// which value it keeps) and over each quad.  Every lane ends with the total
// of value ((l >> 2) & 1) + 2 ((l >> 3) & 1) + 4 (l >> 4): 35 instructions
// for 16 totals where 16 separate wave sums take about 110.  All 64 lanes
// must be active (the adjoint calls it after the plane loop, outside any
// lane-dependent branch).
__device__ __forceinline__ float swap_add32(float a, float b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap_add16(float a, float b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float wave_sum16(const float v[16], int lane) {
    float w[8], x[4], y[2];
#pragma unroll
    for (int i = 0; i < 8; ++i) w[i] = swap_add32(v[i], v[i + 8]);
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = swap_add16(w[i], w[i + 4]);
    const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float keep = b3 ? x[i + 2] : x[i], give = b3 ? x[i] : x[i + 2];
        y[i] = keep + __int_as_float(dpp_i<0x128, 0xF>(__float_as_int(give)));  // row_ror:8
    }
    const float keep = b2 ? y[1] : y[0], give = b2 ? y[0] : y[1];
    float z = keep + __int_as_float(dpp_i<0x141, 0xF>(__float_as_int(give)));  // row_half_mirror
    z += __int_as_float(dpp_i<0xB1, 0xF>(__float_as_int(z)));                  // quad_perm [1,0,3,2]
    z += __int_as_float(dpp_i<0x4E, 0xF>(__float_as_int(z)));                  // quad_perm [2,3,0,1]
    return z;
}
__device__ __forceinline__ int wave_sum16_index(int lane) {
    return ((lane >> 2) & 1) | (((lane >> 3) & 1) << 1) | ((lane >> 4) << 2);
}

// Cost and the pair sensitivities in one sweep over the planes.  With
// d = sum (S_a - S_b)^2 / N, e = d / (1 + d / c), every plane's gradient
// term is (2 / (N den^2)) (S_a - S_b) d(S_a - S_b), den = 1 + d / c: the
// factor in front is one number per pair, so the sweep accumulates
// (S_a - S_b) d(S_a - S_b) alongside the cost and the factor is applied
// after the wave sums (no second sweep re-deriving the lines).
template <class Tap, class G>
__global__ __launch_bounds__(256) void ecc_adj_kernel(const void *__restrict__ sino,
                                                      const PairConst<G> *__restrict__ table, EvalConsts ec,
                                                      float *__restrict__ sens, double *__restrict__ partials,
                                                      int n_tiles) {
    // the plane angle's row offsets stay in vector registers (a select
    // cannot take two scalar operands)
    asm volatile("" : "+v"(ec.rows_half_pi), "+v"(ec.rows_pi));
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int Q = pair_split(ec.B), hpb = kWavesPerBlock / Q;
    const int hyp_groups = (ec.B + hpb - 1) / hpb;
    const int64_t total = plane_work_items(ec.B, n_tiles);
    const int64_t w = xcd_work_item(total);
    if (w >= total) return;  // whole workgroups
    const int S = pair_subtiles(ec.B);
    const int tile_w = (int)(w / hyp_groups);  // work tile: sub-tile sub of pair tile tile
    const int tile = tile_w / S, sub = tile_w % S;
    const int hyp = (int)(w % hyp_groups) * hpb + wave % hpb;
    const int part = wave / hpb, q_per = kPairsPerWave / (Q * S);
    const int q0 = sub * (kPairsPerWave / S) + part * q_per;  // this wave's pairs: q0 .. q0 + q_per - 1
    // a wave without a hypothesis exists only when Q = 1, where no barrier
    // follows; with Q > 1 every wave has one (hpb <= B)
    if (hyp >= ec.B) return;
    __shared__ double part_acc[kWavesPerBlock];
    __shared__ PairConst<G> slots[kWavesPerBlock][kPairsPerWave];
    stage_tile(slots[wave], table + (int64_t)hyp * ec.n_pairs, tile, q0, q_per, lane, ec.n_views);

    const Tap *base = (const Tap *)sino;
    const float kinv = 1.0f / (float)ec.K;
    const bool detector = ec.kappa_detector != 0;
    const bool has_tail = (ec.K & 63) != 0;
    const int n_sweeps = (ec.K >> 6) + (has_tail ? 1 : 0);
    const bool in_tail = lane < (ec.K & 63);
    const uint64_t tail_mask = (1ull << (ec.K & 63)) - 1;
    double wave_acc = 0.0;
    for (int q = 0; q < q_per; ++q) {
        const PairConst<G> pc = uniform(slots[wave][q]);
        if (pc.va < 0) continue;
        const int64_t p = pair_index(pc.va, pc.vb, ec.n_views);
        const Tap *sa = base + (int64_t)pc.va * ec.view_elems;
        const Tap *sb = base + (int64_t)pc.vb * ec.view_elems;
        float acc = 0.0f;
        int cnt = 0;
        float g[kSens];
        for (int i = 0; i < kSens; ++i) g[i] = 0.0f;
        float gu[12];  // dE/dHa, dE/dHb terms weighted by the plane position u
        for (int i = 0; i < 12; ++i) gu[i] = 0.0f;
        G sn, cs;
        g_sincos(pc.k0 + (G)lane * pc.dk, &sn, &cs);
        for (int i = 0; i < n_sweeps; ++i) {
            const bool last = has_tail & (i == n_sweeps - 1);
            const LineCoord<G> ca = line_coord<G, Tap::kAsinTerms>(pc.ha, cs, sn, ec);
            const LineCoord<G> cb = line_coord<G, Tap::kAsinTerms>(pc.hb, cs, sn, ec);
            const Taps ta = load_taps<Tap, G>(ca, sa, ec);
            const Taps tb = load_taps<Tap, G>(cb, sb, ec);
            const bool hit = (!last | in_tail) & ca.hit & cb.hit;
            cnt += __popcll(hit_mask(ca) & hit_mask(cb) & (last ? tail_mask : ~0ull));
            if (hit) {
                const float diff = sample_taps<Tap, G>(ca, ta, pc.inv_f2a, pc.sa) -
                                   sample_taps<Tap, G>(cb, tb, pc.inv_f2b, pc.sb);
                acc = fmaf(diff, diff, acc);
                // object sphere: kappa_k = kappa_max ((2k + 1) / K - 1);
                // detector arc: kappa_k = lo + u (hi - lo), u = (k + 1/2) / K
                const float u = ((float)(lane + 64 * i) + 0.5f) * kinv;
                lookup_adjoint<Tap, G>(cs, sn, ta, ec, pc.inv_f2a, pc.sa, diff, ca, u, g, gu);
                lookup_adjoint<Tap, G>(cs, sn, tb, ec, pc.inv_f2b, pc.sb, -diff, cb, u, g + 6, gu + 6);
            }
            const G c2 = cs * pc.rc - sn * pc.rs;
            sn = sn * pc.rc + cs * pc.rs;
            cs = c2;
        }
        {
            // dE/dkappa_k summed with the weights of the range's parameters:
            // object sphere, kappa_max: 2u - 1; detector arc, lo: 1 - u, hi: u
            const float s0 = kappa_sum(pc.ha, g) + kappa_sum(pc.hb, g + 6);
            const float s1 = kappa_sum(pc.ha, gu) + kappa_sum(pc.hb, gu + 6);
            g[12] = detector ? s0 - s1 : fmaf(2.0f, s1, -s0);
            g[13] = detector ? s1 : 0.0f;
        }
        acc = wave_sum(acc);
        // d and e through the hardware reciprocal, as in the forward kernel
        const float d = cnt > 0 ? acc * __builtin_amdgcn_rcpf((float)cnt) : 0.0f;
        const float den = 1.0f + d * ec.inv_c;
        const float e = ec.inv_c > 0.0f ? d * __builtin_amdgcn_rcpf(den) : d;
        wave_acc += (double)e;
        const float coef = cnt > 0 ? 2.0f * __builtin_amdgcn_rcpf((float)cnt * den * den) : 0.0f;
        float g16[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) g16[i] = i < kSens ? g[i] : 0.0f;
        const float gs = coef * wave_sum16(g16, lane);
        const int j = wave_sum16_index(lane);
        if ((lane & 3) == 0 && j < kSens) sens[((int64_t)hyp * ec.n_pairs + p) * kSens + j] = gs;
    }
    if (Q == 1) {
        if (lane == 0) partials[(int64_t)hyp * n_tiles + tile_w] = wave_acc;
    } else {
        if (lane == 0) part_acc[wave] = wave_acc;
        __syncthreads();
        if (part == 0 && lane == 0) {
            double sum = 0.0;
            for (int k = 0; k < Q; ++k) sum += part_acc[k * hpb + wave];
            partials[(int64_t)hyp * n_tiles + tile_w] = sum;
        }
    }
}

// One thread per (hypothesis, pair): pair_gradient (pair_adjoint.hpp).
__global__ __launch_bounds__(256) void pair_grad_kernel(const ViewGeom *__restrict__ vt,
                                                        const ViewGeomGrad *__restrict__ vg,
                                                        const float *__restrict__ sens, EvalConsts ec,
                                                        float *__restrict__ pair_grad) {
    const int64_t hp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // hyp * n_pairs + pair
    if (hp >= (int64_t)ec.B * ec.n_pairs) return;
    const int hyp = (int)(hp / ec.n_pairs);
    int a, b;
    pair_from_index(hp % ec.n_pairs, ec.n_views, a, b);
    const int64_t ga = (int64_t)hyp * ec.n_views + a, gb = (int64_t)hyp * ec.n_views + b;
    const ViewGeom &A = vt[ga], &Bv = vt[gb];
    double g[kSens], out[12];
    for (int i = 0; i < kSens; ++i) g[i] = (double)sens[hp * kSens + i];
    const ViewGeomGrad &dA = vg[ga], &dB = vg[gb];
    pair_gradient(A.P, A.C, A.u0, A.v0, Bv.P, Bv.C, Bv.u0, Bv.v0, dA.dP, dA.dC, dB.dP, dB.dC, ec.R_mm,
                  ec.kappa_detector != 0, (double)ec.half_w, (double)ec.half_h, g, out);
    for (int q = 0; q < 12; ++q) pair_grad[hp * 12 + q] = (float)out[q];
}

template <class Tap, class G>
static hipError_t launch_adj_t(const void *sino, const void *table, EvalConsts ec, float *sens, double *partials,
                               int n_tiles, hipStream_t s) {
    const int64_t total = plane_work_items(ec.B, n_tiles);
    const int64_t blocks = 8 * ((total + 7) / 8);
    hipLaunchKernelGGL((ecc_adj_kernel<Tap, G>), dim3((unsigned)blocks), dim3(64 * kWavesPerBlock),
                       occupancy_lds_bytes(plane_kernel_lds<G>(), kAdjBlocksPerCU), s, sino,
                       (const PairConst<G> *)table, ec, sens, partials, n_tiles);
    return hipGetLastError();
}

hipError_t launch_ecc_adj(const void *sino, const void *table, const ViewGeom *vt, const ViewGeomGrad *vg,
                          EvalConsts ec, int dtype, float *sens, float *pair_grad, double *partials, int n_tiles,
                          hipStream_t s) {
    hipError_t e;
    if (ec.geom64) {
        if (dtype == 0) e = launch_adj_t<TapF32, double>(sino, table, ec, sens, partials, n_tiles, s);
        else if (dtype == 1) e = launch_adj_t<TapBF16, double>(sino, table, ec, sens, partials, n_tiles, s);
        else e = launch_adj_t<TapF16, double>(sino, table, ec, sens, partials, n_tiles, s);
    } else {
        if (dtype == 0) e = launch_adj_t<TapF32, float>(sino, table, ec, sens, partials, n_tiles, s);
        else if (dtype == 1) e = launch_adj_t<TapBF16, float>(sino, table, ec, sens, partials, n_tiles, s);
        else e = launch_adj_t<TapF16, float>(sino, table, ec, sens, partials, n_tiles, s);
    }
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)ec.B * ec.n_pairs;
    hipLaunchKernelGGL(pair_grad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, vt, vg, sens, ec,
                       pair_grad);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// grad[b][v][0..5] = sum over partners u of the pair (min, max)'s 12-vector:
// entries 0..5 when v is the first view of the pair, 6..11 else.  One wave
// per (hypothesis, view): lane l adds the partners u = l, l + 64, ... in
// FP64, then the 64 lane sums are added in a fixed butterfly order.
__global__ __launch_bounds__(256) void reduce_grad_kernel(const float *__restrict__ pair_grad, int B, int n_views,
                                                          float *__restrict__ grad) {
    const int64_t wid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (wid >= (int64_t)B * n_views) return;  // whole waves; no barriers
    const int b = (int)(wid / n_views), v = (int)(wid % n_views);
    const int64_t n_pairs = (int64_t)n_views * (n_views - 1) / 2;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const float *pg = pair_grad + (int64_t)b * n_pairs * 12;
    for (int u = lane; u < n_views; u += 64) {
        if (u == v) continue;
        const float *src = u < v ? pg + pair_index(u, v, n_views) * 12 + 6 : pg + pair_index(v, u, n_views) * 12;
        for (int q = 0; q < 6; ++q) acc[q] += (double)src[q];
    }
    for (int q = 0; q < 6; ++q)
        for (int o = 32; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, 64);
    if (lane == 0)
        for (int q = 0; q < 6; ++q) grad[wid * 6 + q] = (float)acc[q];
}

hipError_t launch_reduce_grad(const float *pair_grad, int B, int n_views, float *grad, hipStream_t s) {
    const int64_t waves = (int64_t)B * n_views;
    hipLaunchKernelGGL(reduce_grad_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, pair_grad, B, n_views,
                       grad);
    return hipGetLastError();
}

}  // namespace ecc
