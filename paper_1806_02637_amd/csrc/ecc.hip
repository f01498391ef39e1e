// Epipolar-consistency cost on gfx950 (arxiv 1806.02637, Eqs. 13-17).
//
// view_setup   one thread per (hypothesis, view): P' = P T(theta) and its
//              source (Eqs. 4-5), FP64; optionally dP'/dtheta for the adjoint.
// pair_setup   one thread per (hypothesis, pair): the pair's geometry in FP64
//              (baseline, pencil of planes, the two line maps of Eq. 14) ->
//              a table of per-plane constants.
// ecc_fwd      a workgroup = one hypothesis x one sub-tile of a tile of up
//              to 64 view pairs (8 x 8 view blocks); a wave walks its
//              pairs (constants staged in LDS) with lanes along the plane angle kappa: line ->
//              (alpha, t) -> four bilinear taps per view in one load ->
//              (S_a - S_b)^2 -> wave-shuffle sum (Eq. 15) -> Cauchy norm
//              (Eq. 16).  No atomics; per-tile FP64 partials.
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
size_t pair_const_bytes(bool geom64) { return geom64 ? sizeof(PairConst<double>) : sizeof(PairConst<float>); }

// One thread per (hypothesis, pair): the FP64 per-pair geometry -> the pair's
// per-plane constants, written to a table the plane kernels read with
// wave-uniform (scalar) loads.
template <class G>
__global__ __launch_bounds__(256) void pair_setup_kernel(const float *__restrict__ vscale,
                                                         const ViewGeom *__restrict__ vt,
                                                         const double *__restrict__ pinv, EvalConsts ec,
                                                         PairConst<G> *__restrict__ table) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)ec.B * ec.n_pairs) return;
    const int hyp = (int)(idx / ec.n_pairs);
    const int64_t p = idx % ec.n_pairs;
    int a, b;
    pair_from_index(p, ec.n_views, a, b);
    PairConst<G> pc;
    const int64_t ga = (int64_t)hyp * ec.n_views + a, gb = (int64_t)hyp * ec.n_views + b;
    pair_setup<G>(vt[ga], vt[gb], ec, pc, pinv ? pinv + 12 * ga : nullptr,
                  pinv ? pinv + 12 * gb : nullptr);
    pc.va = a;
    pc.vb = b;
    pc.sa = vscale[a];
    pc.sb = vscale[b];
    table[idx] = pc;
}

template <class G>
static hipError_t launch_pair_setup_t(const float *vscale, const ViewGeom *vt, const double *pinv, EvalConsts ec,
                                      void *table, hipStream_t s) {
    const int64_t n = (int64_t)ec.B * ec.n_pairs;
    hipLaunchKernelGGL(pair_setup_kernel<G>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, vscale, vt, pinv,
                       ec, (PairConst<G> *)table);
    return hipGetLastError();
}

hipError_t launch_pair_setup(const float *view_scale, const ViewGeom *vt, EvalConsts ec, void *table, hipStream_t s,
                             const double *pinv) {
    return ec.geom64 ? launch_pair_setup_t<double>(view_scale, vt, pinv, ec, table, s)
                     : launch_pair_setup_t<float>(view_scale, vt, pinv, ec, table, s);
}

// One plane of one pair between issuing its gathers and combining them: the
// raw taps in flight (converted only in the combine) plus everything the
// combine needs (bilinear fractions, Grangeat weights with the storage scale,
// hit test, relative fold sign).
template <class Tap>
struct PlaneInFlight {
    typename Tap::Raw ta, tb;
    float fa_a, ft_a, w_a, fa_b, ft_b, w_b;
    bool hit, flip;
    uint64_t mask;  // wave mask of `hit`
};

template <class Tap, class G>
__device__ __forceinline__ void issue_plane(PlaneInFlight<Tap> &P, const PairConst<G> &pc, G cs, G sn,
                                            const Tap *sa, const Tap *sb, const EvalConsts &ec) {
    const LineCoord<G> ca = line_coord<G, Tap::kAsinTerms>(pc.ha, cs, sn, ec);
    const LineCoord<G> cb = line_coord<G, Tap::kAsinTerms>(pc.hb, cs, sn, ec);
    P.ta = fetch_taps<Tap, G>(ca, sa, ec);
    P.tb = fetch_taps<Tap, G>(cb, sb, ec);
    P.fa_a = ca.fa;
    P.ft_a = ca.ft;
    P.fa_b = cb.fa;
    P.ft_b = cb.ft;
    P.w_a = grangeat_weight<Tap>(ca.tf, pc.inv_f2a, pc.sa);
    P.w_b = grangeat_weight<Tap>(cb.tf, pc.inv_f2b, pc.sb);
    P.hit = ca.hit & cb.hit;
    P.flip = ca.fold != cb.fold;
    P.mask = hit_mask(ca) & hit_mask(cb);
}

// Adds (S_a - S_b)^2 of a plane whose taps have arrived.  (S_a - S_b)^2 =
// (U_a -+ U_b)^2 with U the unsigned samples: only the relative fold sign
// matters.  `valid` masks the lanes past K in the last sweep, `count_mask`
// the same lanes in the hit count.
template <class Tap>
__device__ __forceinline__ void combine_plane(const PlaneInFlight<Tap> &P, bool valid, uint64_t count_mask,
                                              float &acc, int &cnt) {
    const float Ua = P.w_a * bilinear<Tap>(P.ta, P.fa_a, P.ft_a);
    const float Ub = P.w_b * bilinear<Tap>(P.tb, P.fa_b, P.ft_b);
    const float d = (P.hit & valid) ? Ua - (P.flip ? -Ub : Ub) : 0.0f;
    acc = fmaf(d, d, acc);
    cnt += __popcll(P.mask & count_mask);
}

// A workgroup = one hypothesis x one work tile (a sub-tile of a pair tile,
// pair_subtiles), its pairs split into 4 parts over its waves (pair_split);
// consecutive workgroups are the same work tile's other hypotheses, which
// read nearly the same sinogram cells.  Lanes
// walk the planes k = lane + 64 i; the trip count is wave-uniform (K / 64
// full sweeps plus a masked tail) and the hit count is a population count of
// the hit mask.  The gathers of sweep i + 1 are issued before sweep i is
// combined, so each wave keeps two planes' gathers in flight.  out_pair and
// out_count (e and N_kappa per pair) are optional.
template <class Tap, class G>
__global__ __launch_bounds__(256) void ecc_fwd_kernel(const void *__restrict__ sino,
                                                      const PairConst<G> *__restrict__ table, EvalConsts ec,
                                                      float *__restrict__ out_pair, int32_t *__restrict__ out_count,
                                                      double *__restrict__ partials, int n_tiles) {
    // the column offset joins an FMA with two other scalar operands: keep it
    // in a vector register for the whole kernel rather than copy it per plane
    asm volatile("" : "+v"(ec.t0_tau));
    // so are the plane angle's two row offsets (a select cannot take two
    // scalar operands)
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
    const bool has_tail = (ec.K & 63) != 0;
    const int n_sweeps = (ec.K >> 6) + (has_tail ? 1 : 0);
    const bool in_tail = lane < (ec.K & 63);
    const uint64_t tail_mask = (1ull << (ec.K & 63)) - 1;
    double wave_acc = 0.0;
    for (int q = 0; q < q_per; ++q) {
        const PairConst<G> pc = slots[wave][q];
        // view ids (and so the two sinogram bases) in scalar registers
        const int a = uniform(pc.va), b = uniform(pc.vb);
        if (a < 0) continue;
        const int64_t p = pair_index(a, b, ec.n_views);
        const Tap *sa = base + (int64_t)a * ec.view_elems;
        const Tap *sb = base + (int64_t)b * ec.view_elems;
        float acc = 0.0f;
        int cnt = 0;
        // plane angle of this lane, advanced by one wave step (64 dk) per
        // sweep through the rotation (rc, rs)
        G sn, cs;
        g_sincos(pc.k0 + (G)lane * pc.dk, &sn, &cs);
        auto rotate = [&]() {
            const G c2 = cs * pc.rc - sn * pc.rs;
            sn = sn * pc.rc + cs * pc.rs;
            cs = c2;
        };
        // sweep i is the partial last one when has_tail and i = n_sweeps - 1
        auto combine = [&](const PlaneInFlight<Tap> &P, int i) {
            const bool last = has_tail & (i == n_sweeps - 1);
            combine_plane(P, !last | in_tail, last ? tail_mask : ~0ull, acc, cnt);
        };
        {
            // two buffers, swapped by unrolling (no register copies); the
            // steady state issues unconditionally so that each combine waits
            // only for its own gathers (three planes in flight measured no
            // faster at B = 32 on the 496-view scan, with any storage form)
            PlaneInFlight<Tap> P0, P1;
            issue_plane<Tap, G>(P0, pc, cs, sn, sa, sb, ec);
            rotate();
            int i = 0;
            // (the scheduling barriers keep the compiler from hoisting a
            // combine above the issue that is meant to cover its latency)
            for (; i + 2 < n_sweeps; i += 2) {
                issue_plane<Tap, G>(P1, pc, cs, sn, sa, sb, ec);
                rotate();
                __builtin_amdgcn_sched_barrier(0);
                combine(P0, i);
                issue_plane<Tap, G>(P0, pc, cs, sn, sa, sb, ec);
                rotate();
                __builtin_amdgcn_sched_barrier(0);
                combine(P1, i + 1);
            }
            if (i + 1 < n_sweeps) {
                issue_plane<Tap, G>(P1, pc, cs, sn, sa, sb, ec);
                __builtin_amdgcn_sched_barrier(0);
                combine(P0, i);
                combine(P1, i + 1);
            } else {
                combine(P0, i);
            }
        }
        acc = wave_sum(acc);
        // d and e through the hardware reciprocal (1 ulp; cnt >= 1 and the
        // Cauchy denominator >= 1), as in the adjoint
        const float d = cnt > 0 ? acc * __builtin_amdgcn_rcpf((float)cnt) : 0.0f;
        const float e = ec.inv_c > 0.0f ? d * __builtin_amdgcn_rcpf(1.0f + d * ec.inv_c) : d;
        if (out_pair && lane == 0) out_pair[(int64_t)hyp * ec.n_pairs + p] = e;
        if (out_count && lane == 0) out_count[(int64_t)hyp * ec.n_pairs + p] = cnt;
        wave_acc += (double)e;
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

// Occupancy cap of the plane kernels: workgroups per CU, enforced through an
// unused dynamic LDS allocation (160 KB per CU).  More resident waves than
// this widen the set of pair tiles in flight per XCD, and L2 misses grow
// faster than latency hiding gains.
size_t occupancy_lds_bytes(size_t static_bytes, int cap) {
    if (cap <= 0) return 0;
    size_t b = (160u * 1024u) / (size_t)cap;
    b = (b / 1024) * 1024;
    if (b > 65536) b = 65536;
    return b > static_bytes ? b - static_bytes : 0;
}

template <class Tap, class G>
static hipError_t launch_fwd_t(const void *sino, const void *table, EvalConsts ec, float *out_pair,
                               int32_t *out_count, double *partials, int n_tiles, hipStream_t s) {
    const int64_t total = plane_work_items(ec.B, n_tiles);
    const int64_t blocks = 8 * ((total + 7) / 8);
    hipLaunchKernelGGL((ecc_fwd_kernel<Tap, G>), dim3((unsigned)blocks), dim3(64 * kWavesPerBlock),
                       occupancy_lds_bytes(plane_kernel_lds<G>(), kFwdBlocksPerCU),
                       s, sino, (const PairConst<G> *)table, ec, out_pair, out_count, partials, n_tiles);
    return hipGetLastError();
}

hipError_t launch_ecc_fwd(const void *sino, const void *table, EvalConsts ec, int dtype, float *out_pair,
                          int32_t *out_count, double *partials, int n_tiles, hipStream_t s) {
    if (ec.geom64) {
        if (dtype == 0) return launch_fwd_t<TapF32, double>(sino, table, ec, out_pair, out_count, partials, n_tiles, s);
        if (dtype == 1) return launch_fwd_t<TapBF16, double>(sino, table, ec, out_pair, out_count, partials, n_tiles, s);
        return launch_fwd_t<TapF16, double>(sino, table, ec, out_pair, out_count, partials, n_tiles, s);
    }
    if (dtype == 0) return launch_fwd_t<TapF32, float>(sino, table, ec, out_pair, out_count, partials, n_tiles, s);
    if (dtype == 1) return launch_fwd_t<TapBF16, float>(sino, table, ec, out_pair, out_count, partials, n_tiles, s);
    return launch_fwd_t<TapF16, float>(sino, table, ec, out_pair, out_count, partials, n_tiles, s);
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
