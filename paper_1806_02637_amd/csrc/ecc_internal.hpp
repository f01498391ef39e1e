// Internal declarations of the ECC engine: data layouts shared by the host
// engine and the kernels, and the host-side launchers of each kernel file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct ecc_ctx;

namespace ecc {

// ---------------------------------------------------------------------------
// Resident sinogram layout.
//
// Row-interleaved: element (view, m, j) holds the pair (S[m][k], S[m+1][k])
// with k = j - 1, for m = 0..n_alpha and j = 0..n_t+1.  Columns j = 0 and
// j = n_t + 1 are zero (t beyond the grid reads as 0).  Rows n_alpha and
// n_alpha + 1 continue the sinogram past pi by its odd symmetry,
// S(alpha + pi, t_k) = -S(alpha, t_{n_t-1-k}): row n_alpha is the pad row at
// alpha = pi, row n_alpha + 1 the one a step beyond it.  One 2-element load
// at (m, k + 1) therefore returns all four bilinear taps of cell (m, k).
// FP32 storage: 8-byte elements; BF16 / FP16: 4-byte elements.
// ---------------------------------------------------------------------------
struct SinoLayout {
    int32_t n_views, n_alpha, n_t;
    int32_t row_elems;      // n_t + 2
    int64_t view_elems;     // (n_alpha + 1) * row_elems
    int32_t dtype;          // ECC_F32 / ECC_BF16 / ECC_F16
    int32_t elem_bytes;     // 8 or 4
};

inline SinoLayout make_layout(int n_views, int n_alpha, int n_t, int dtype) {
    SinoLayout L;
    L.n_views = n_views;
    L.n_alpha = n_alpha;
    L.n_t = n_t;
    L.row_elems = n_t + 2;
    L.view_elems = (int64_t)(n_alpha + 1) * L.row_elems;
    L.dtype = dtype;
    L.elem_bytes = dtype == 0 ? 8 : 4;
    return L;
}

// Per (hypothesis, view) geometry, FP64: moved projection P' = P T(theta)
// (row-major 3x4), its source, and the view's intrinsics.
struct ViewGeom {
    double P[12];
    double C[3];
    double f, u0, v0;
    double pad[2];
};
static_assert(sizeof(ViewGeom) == 160, "ViewGeom layout");

// Derivatives of a ViewGeom with respect to the view's 6 motion parameters.
struct ViewGeomGrad {
    double dP[6][12];
    double dC[6][3];
};

// Terms of the plane-angle polynomial (in sinogram rows, FP32 plane geometry)
// per storage form: 7 with FP32 storage (1.6e-7 rad, the rounding of an FP32
// angle near pi), 6 with 16-bit storage (3.9e-7 rad, 1e-4 of a row at 768 rows,
// far below the rounding of the stored values).  The host fills
// EvalConsts::asin_rows for the same count.
constexpr int kAsinTermsF32 = 7;
constexpr int kAsinTerms16 = 6;

// Scan-wide constants of an evaluation.
struct EvalConsts {
    int32_t n_views, n_pairs, K, B;
    int32_t n_alpha, n_t, row_elems, geom64;
    int64_t view_elems;
    double R_mm;
    float inv_c;       // 1/c, 0 for c = inf
    float half_w, half_h;
    // t / dt + t0_tau, t0_tau = (t_max + dt) / dt, is the stored column
    // coordinate of t
    float t0_tau, inv_dt, inv_dalpha;
    int32_t kappa_detector;  // 1: planes sample the arc both detectors see (else the object sphere's)
    double t0_tau_d, inv_dt_d, inv_dalpha_d;
    // FP32 plane angle in sinogram rows (alpha / dalpha): the asin
    // coefficients of the storage type's fit times 1 / dalpha, and the
    // offsets pi/2 and pi in rows
    float asin_rows[7];
    float rows_half_pi, rows_pi;
};

// Pair index <-> (a, b), a < b, row-major triangle.
__host__ __device__ inline int64_t pair_index(int a, int b, int n) {
    return (int64_t)a * n - (int64_t)a * (a + 1) / 2 + (b - a - 1);
}

// Launchers (each returns hipError_t of the launch).
hipError_t launch_sino_weight(const float *images, const double *intr, int n_views, int W, int H, float *gw,
                              float *gwT, hipStream_t s);
hipError_t launch_sino_radon(const float *gw, const float *gwT, const double *intr, int n_views, int W, int H,
                             int n_alpha, int n_t, double ds, double *G, hipStream_t s);
hipError_t launch_sino_store(const double *G, const float *ext, int n_views, int n_alpha, int n_t, double dt,
                             int dtype, void *sino, float *view_scale, uint32_t *view_absmax, hipStream_t s);
hipError_t launch_sino_read(const void *sino, const float *view_scale, SinoLayout L, int view, float *out,
                            hipStream_t s);

hipError_t launch_view_setup(const double *P, const double *intr, const double *theta, int B, int n_views,
                             ViewGeom *vt, ViewGeomGrad *vg, hipStream_t s);
// per-pair constant table: [B][n_pairs] PairConst<float> or PairConst<double>
size_t pair_const_bytes(bool geom64);
// pinv (optional): [B][n_views][4][3] pseudo-inverses of the moved P' (the
// line route the method replaces)
hipError_t launch_pair_setup(const float *view_scale, const ViewGeom *vt, EvalConsts ec, void *table, hipStream_t s,
                             const double *pinv = nullptr);
// out_pair [B][n_pairs] e and out_count [B][n_pairs] N_kappa, each optional
hipError_t launch_ecc_fwd(const void *sino, const void *table, EvalConsts ec, int dtype, float *out_pair,
                          int32_t *out_count, double *partials, int n_tiles, hipStream_t s);
// adjoint: plane kernel -> per-pair sensitivities sens [B][n_pairs][13], then
// per-pair tangent sweeps -> pair_grad [B][n_pairs][12]
hipError_t launch_ecc_adj(const void *sino, const void *table, const ViewGeom *vt, const ViewGeomGrad *vg,
                          EvalConsts ec, int dtype, float *sens, float *pair_grad, double *partials, int n_tiles,
                          hipStream_t s);
hipError_t launch_reduce_cost(const double *partials, int n_tiles, int B, double *out_cost, hipStream_t s);
hipError_t launch_reduce_grad(const float *pair_grad, int B, int n_views, float *grad, hipStream_t s);

// Akima spline motion model (spline.hip): node positions along the view
// index, strictly ascending, covering [0, n_views - 1].
constexpr int kMaxSplineNodes = 64;
struct SplineKnots {
    int32_t n;
    double x[kMaxSplineNodes];
};
// nodes [B][6][n] -> theta [B][n_views][6]
hipError_t launch_spline_motion(const SplineKnots &kn, int B, int n_views, const double *nodes, double *theta,
                                hipStream_t s);
// grad_theta [B][n_views][6] -> grad_nodes [B][6][n]
hipError_t launch_spline_grad(const SplineKnots &kn, int B, int n_views, const double *nodes,
                              const float *grad_theta, double *grad_nodes, hipStream_t s);

// Engine services shared with the server (engine.hip).
int ctx_device(struct ::ecc_ctx *ctx);
int32_t set_error(int32_t code, const char *fmt, ...);

constexpr int kPairsPerWave = 64;
// zero border (pixels) around the weighted projections read by the line sums
constexpr int kImgPad = 3;
constexpr int kWavesPerBlock = 4;
// Sub-tiles per pair tile: a tile's 64 pairs are spread over 8 consecutive
// workgroups with one hypothesis (8 pairs each), 4 with two, 2 otherwise (32
// pairs each), so that an XCD keeps few tiles' lines in flight.  At B = 1 on
// the 496-view scan 1953 whole tiles put about 1000 different tiles' lines
// in flight and the L2 hit 40 % of requests; 4 sub-tiles per tile cut a
// B = 1 cost from 0.64 to 0.49 ms, 8 to 0.45 ms; at B = 32, 2 sub-tiles
// take 1 % off the forward step and 2 % off cost + gradient (4 are no
// better).  The plane kernels take the number of work tiles, pair tiles *
// pair_subtiles(B), and write one partial sum per hypothesis and work tile.
__host__ __device__ inline int pair_subtiles(int B) { return B == 1 ? 8 : (B == 2 ? 4 : 2); }
// caps on resident plane-kernel workgroups per CU (0 = no cap), 4 for the
// forward kernel with every storage form and for the adjoint (at B = 32 on
// the 496-view scan: the FP32 forward kernel at 3 is 2 % slower, the 16-bit
// forms at 5 or 6 no faster; the adjoint at 3 is 17 % slower)
constexpr int kFwdBlocksPerCU = 4;
constexpr int kAdjBlocksPerCU = 4;
// dynamic LDS that, added to a kernel's static LDS, caps resident
// workgroups per CU at `cap` (0 = no cap)
size_t occupancy_lds_bytes(size_t static_bytes, int cap);

}  // namespace ecc
