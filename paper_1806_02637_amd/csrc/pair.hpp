// Per-pair device helpers shared by the forward and adjoint kernels: pair
// indexing, the FP64 per-pair geometry, wave reductions and the XCD-aware
// block numbering.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "arc.hpp"
#include "ecc_internal.hpp"
#include "lookup.hpp"
#include "projective.hpp"

namespace ecc {

// Pair (a, b) from its row-major triangle index.
__device__ __forceinline__ void pair_from_index(int64_t p, int n, int &a, int &b) {
    const double m = 2.0 * n - 1.0;
    int aa = (int)floor(0.5 * (m - sqrt(m * m - 8.0 * (double)p)));
    if (aa < 0) aa = 0;
    if (aa > n - 2) aa = n - 2;
    while (aa > 0 && pair_index(aa, aa + 1, n) > p) --aa;
    while (aa < n - 2 && pair_index(aa + 1, aa + 2, n) <= p) ++aa;
    a = aa;
    b = (int)(p - pair_index(aa, aa + 1, n)) + aa + 1;
}

// FP64 per-pair geometry -> the per-plane constants of one pair.  The line
// maps come from Eqs. 13-14 (the moved P' of each view), or, when pinv_a /
// pinv_b are given, from the caller's pseudo-inverses of P' (the route the
// method replaces; same lines up to a positive scale).  The K planes sample
// the pencil's arc that meets the object sphere of radius R_mm, or, with
// kappa_detector, the arc around kappa = 0 whose lines meet both detectors;
// a pair whose detector arc is empty gets lines that miss every detector
// (N = 0, e = 0).
template <class G>
__device__ __forceinline__ void pair_setup(const ViewGeom &A, const ViewGeom &Bv, const EvalConsts &ec,
                                           PairConst<G> &pc, const double *pinv_a = nullptr,
                                           const double *pinv_b = nullptr) {
    double u1[3], u2[3], km;
    pencil(A.C, Bv.C, ec.R_mm, u1, u2, km);
    double Ha[6], Hb[6];
    if (pinv_a) {
        line_map_pinv(pinv_a, A.C, u1, u2, A.u0, A.v0, Ha);
        line_map_pinv(pinv_b, A.C, u1, u2, Bv.u0, Bv.v0, Hb);
    } else {
        line_map(A.P, A.C, u1, u2, A.u0, A.v0, Ha);
        line_map(Bv.P, A.C, u1, u2, Bv.u0, Bv.v0, Hb);
    }
    double lo = -km, hi = km;
    if (ec.kappa_detector) {
        if (!pair_arc(Ha, Hb, (double)ec.half_w, (double)ec.half_h, lo, hi)) {
            // every sample at kappa = 0 on the line x = -2^20 px: off every
            // detector, finite coordinates (cell indices outside the
            // sinogram, whose loads tap_address keeps inside the view)
            for (int i = 0; i < 6; ++i) Ha[i] = Hb[i] = 0.0;
            Ha[0] = Hb[0] = 1.0;
            Ha[2] = Hb[2] = 1048576.0;
            lo = hi = 0.0;
        }
    }
    // (alpha, t) of a line do not change under a positive scale: bring both
    // maps to unit magnitude with an exact power of two
    double ma = 0.0, mb = 0.0;
    for (int i = 0; i < 6; ++i) {
        ma = fmax(ma, fabs(Ha[i]));
        mb = fmax(mb, fabs(Hb[i]));
    }
    const int ea = ma > 0.0 ? ilogb(ma) : 0, eb = mb > 0.0 ? ilogb(mb) : 0;
    for (int i = 0; i < 6; ++i) {
        pc.ha[i] = (G)ldexp(Ha[i], -ea);
        pc.hb[i] = (G)ldexp(Hb[i], -eb);
    }
    const double dk = (hi - lo) / ec.K;
    pc.k0 = (G)(lo + 0.5 * dk);
    pc.dk = (G)dk;
    double rs, rc;
    sincos(64.0 * dk, &rs, &rc);
    pc.rc = (G)rc;
    pc.rs = (G)rs;
    pc.inv_f2a = (float)(1.0 / (A.f * A.f));
    pc.inv_f2b = (float)(1.0 / (Bv.f * Bv.f));
}

// Wave-wide sums with DPP in a fixed order: pairs, quads, half rows and rows
// of 16 lanes, then row 0 + row 1 into row 1 and rows 0-1 + rows 2-3 into
// row 3; lane 63 ends with the total, broadcast through a scalar register.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_i(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, ROW_MASK, 0xF, false);
}
__device__ __forceinline__ float wave_sum(float x) {
    x += __int_as_float(dpp_i<0xB1, 0xF>(__float_as_int(x)));   // quad_perm [1,0,3,2]
    x += __int_as_float(dpp_i<0x4E, 0xF>(__float_as_int(x)));   // quad_perm [2,3,0,1]
    x += __int_as_float(dpp_i<0x141, 0xF>(__float_as_int(x)));  // row_half_mirror
    x += __int_as_float(dpp_i<0x140, 0xF>(__float_as_int(x)));  // row_mirror
    x += __int_as_float(dpp_i<0x142, 0xA>(__float_as_int(x)));  // row_bcast:15
    x += __int_as_float(dpp_i<0x143, 0xC>(__float_as_int(x)));  // row_bcast:31
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Pair tiles: the views are cut into blocks of kViewBlock consecutive views and
// a tile is one (block I, block J >= I) product -- up to 8 x 8 pairs (I < J)
// or the 28 pairs inside one block (I == J).  The 8 neighbouring sources of a
// block give similar pencils in each view of the other block, so a tile
// touches 16 views' sinograms with high reuse.  Tiles run row by row
// (I fixed, J increasing), so the tiles in flight on one XCD share block I.
// Inside a tile a wave walks the pairs with the block-J view b fixed for 8
// consecutive pairs while the block-I view a changes: the block-I views'
// lines are largely common to all tiles in flight and stay in L2 until a view
// comes back 8 pairs later, while each tile's own view b is reused at once.
// (With a fixed and b walking, every tile's b comes back only after 8 pairs,
// by when the other tiles' lines have evicted it: at B = 32 on the 496-view
// scan, with four hypotheses of a tile per workgroup, that order measured an
// L2 hit rate of 0.754 against 0.860 and 9.7 against 9.3 ms per evaluation.)
constexpr int kViewBlock = 8;

__host__ __device__ inline int n_view_blocks(int n_views) { return (n_views + kViewBlock - 1) / kViewBlock; }
__host__ __device__ inline int n_pair_tiles(int n_views) {
    const int nb = n_view_blocks(n_views);
    return nb * (nb + 1) / 2;
}

// Pair q (0..63) of tile `tile`; false when the slot is empty.
__device__ __forceinline__ bool tile_pair(int tile, int q, int n_views, int &a, int &b) {
    const int nb = n_view_blocks(n_views);
    // block row I of the upper triangle (diagonal included)
    const double m = 2.0 * nb + 1.0;
    int I = (int)floor(0.5 * (m - sqrt(m * m - 8.0 * (double)tile)));
    if (I < 0) I = 0;
    if (I > nb - 1) I = nb - 1;
    while (I > 0 && I * nb - I * (I - 1) / 2 > tile) --I;
    while (I < nb - 1 && (I + 1) * nb - (I + 1) * I / 2 <= tile) ++I;
    const int J = tile - (I * nb - I * (I - 1) / 2) + I;
    if (I < J) {
        a = I * kViewBlock + q % kViewBlock;
        b = J * kViewBlock + q / kViewBlock;
    } else {
        if (q >= kViewBlock * (kViewBlock - 1) / 2) return false;
        int i, j;
        pair_from_index(q, kViewBlock, i, j);
        a = I * kViewBlock + i;
        b = I * kViewBlock + j;
    }
    return a < n_views && b < n_views;
}

// Stages the constants of pairs q0 .. q0 + n - 1 of a tile into this wave's
// LDS slots (lane i < n loads pair q0 + i into slot i); empty slots get
// va = -1.  Wave-scope fences make the slots written by one lane visible to
// the whole wave.
template <class G>
__device__ __forceinline__ void stage_tile(PairConst<G> *slots, const PairConst<G> *tab, int tile, int q0, int n,
                                           int lane, int n_views) {
    if (lane < n) {
        int a, b;
        if (tile_pair(tile, q0 + lane, n_views, a, b)) {
            slots[lane] = tab[pair_index(a, b, n_views)];
        } else {
            slots[lane].va = -1;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Waves of a workgroup: kWavesPerBlock / Q hypotheses of one work tile (a
// pair tile's sub-tile, pair_subtiles), its pairs split into Q parts,
// Q = pair_split(B); the parts' sums are added in a fixed order.
// Q = kWavesPerBlock for every B: a workgroup is one hypothesis of one work
// tile, its waves sharing the work tile's pairs, and consecutive workgroups
// on an XCD are the same work tile's next hypotheses.  The XCD then
// holds all hypotheses of a few tiles rather than four hypotheses of many, a
// smaller set of sinogram lines in flight (at B = 32 on the 496-view scan the
// forward kernel ran 2-4 % and the adjoint 7 % faster than with four
// hypotheses of a tile per workgroup), and a B = 1 evaluation (one L-BFGS
// step) has four times the waves in flight it would have with one wave per
// tile.
__host__ __device__ inline int pair_split(int) { return kWavesPerBlock; }
__host__ __device__ inline int64_t plane_work_items(int B, int n_work_tiles) {
    const int hpb = kWavesPerBlock / pair_split(B);
    return (int64_t)n_work_tiles * ((B + hpb - 1) / hpb);
}

// Static LDS of the plane kernels: the pair constants of each wave's tile and
// the per-wave partial sums.
template <class G>
constexpr size_t plane_kernel_lds() {
    return sizeof(PairConst<G>) * kPairsPerWave * kWavesPerBlock + sizeof(double) * kWavesPerBlock;
}

// Logical work item of a block under the XCD-aware numbering.
__device__ __forceinline__ int64_t xcd_work_item(int64_t total) {
    const int64_t per = (total + 7) / 8;
    const int64_t i = blockIdx.x;
    return (i % 8) * per + i / 8;
}

}  // namespace ecc
