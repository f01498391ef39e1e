/*
 * ecc.h -- C ABI of the MI355X engine for Grangeat-based epipolar consistency
 * (ECC) of C-arm cone-beam projections (arxiv 1806.02637, "Fast Epipolar
 * Consistency without the Need for Pseudo Matrix Inverses").
 *
 * The engine holds scans (views + 3x4 projection matrices), builds each view's
 * Radon-derivative sinogram once and keeps it in HBM, and evaluates the
 * consistency cost (and its gradient) for batches of per-view rigid-motion
 * hypotheses.  All compute runs in HIP kernels for gfx950.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns ecc_status: ECC_OK (0) or a negative code.  No
 *   function aborts.  The message of the last failure on the calling thread
 *   is available from ecc_last_error().
 * - Argument checks (shapes, ranges, NULLs, unknown ids) are synchronous and
 *   leave no partial state.  HIP failures are reported as ECC_E_HIP.
 * - Pointers named *_dev are device pointers on the context's device; the
 *   caller keeps ownership and must keep them alive until the work queued on
 *   `stream` has completed.  Host pointers are only read during the call.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   Evaluation entry points are asynchronous on that stream.
 * - A context may be used from several host threads; scan loading/freeing is
 *   serialised internally.  Evaluations on different streams may overlap on
 *   the device as long as each has its own workspace.
 * - Pairs are the N(N-1)/2 view pairs a < b in row-major triangle order:
 *   pair index p(a, b) = a N - a (a + 1) / 2 + (b - a - 1).
 */
#ifndef ECC_H
#define ECC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ecc_status;
typedef struct ecc_ctx ecc_ctx;

enum {
    ECC_OK = 0,
    ECC_E_ARG = -1,     /* invalid argument, shape or value */
    ECC_E_BUDGET = -2,  /* the request would exceed the context's HBM budget */
    ECC_E_HIP = -3,     /* a HIP runtime call failed */
    ECC_E_STATE = -4,   /* call out of order (e.g. cost before sinograms are built) */
    ECC_E_NOSCAN = -5   /* unknown or freed scan id */
};

/* Storage type of the resident sinograms. */
enum { ECC_F32 = 0, ECC_BF16 = 1, ECC_F16 = 2 };

/* Precision of the per-plane geometry (epipolar line, its angle and offset).
 * The per-view and per-pair geometry (moved projection, sources, baseline,
 * pencil of planes) is always FP64. */
enum { ECC_GEOM_F32 = 0, ECC_GEOM_F64 = 1 };
/* Which arc of the pencil of epipolar planes an evaluation samples. */
enum { ECC_KAPPA_OBJECT = 0, ECC_KAPPA_DETECTOR = 1 };

/* Message of the last failed call on this thread ("" if none). */
const char *ecc_last_error(void);

/* Creates a context on HIP device `hip_device`.  `hbm_budget_bytes` bounds
 * the device memory the context itself allocates (resident scans); 0 means
 * no bound. */
ecc_status ecc_create(ecc_ctx **out, int hip_device, uint64_t hbm_budget_bytes);

/* Frees every scan and the context.  Waits for the device to go idle. */
ecc_status ecc_destroy(ecc_ctx *ctx);

/* Loads one scan: a set of projections, each with its 3x4 projection
 * matrix (Sec. "Epipolar Consistency").
 *   P      [n_views][3][4] FP64, row-major, maps world mm to detector pixels
 *          (pixel centres at integer (u, v), u = column, v = row).  All views
 *          must share the sign of det(P[:, :3]) (one detector handedness).
 *   intr   [n_views][3] FP64 = {f_px, u0, v0}: focal length in pixels and the
 *          principal point, used for the cosine weight of Eq. 1 and to centre
 *          detector lines.  The principal point must be the detector centre,
 *          (u0, v0) = ((W - 1) / 2, (H - 1) / 2) within 1e-6 px: the hit test
 *          behind Eq. 15's plane count and the sinogram's t range are taken
 *          about it.  Rigid motion does not change them.
 *   images [n_views][H][W] FP32 line integrals (row v, column u); host memory
 *          if images_on_device == 0, else a device pointer.  Copied.
 * The projections are held (FP32, in HBM) until sinograms are built.
 * Errors: ECC_E_ARG (sizes < 2, NULLs, non-finite or mixed-handedness P,
 * a principal point off the detector centre),
 * ECC_E_BUDGET, ECC_E_HIP. */
ecc_status ecc_scan_load(ecc_ctx *ctx, int32_t *scan_id, int32_t n_views, int32_t W, int32_t H,
                         const double *P, const double *intr, const float *images, int32_t images_on_device);

/* Builds every view's Radon-derivative sinogram: Grangeat's intermediate
 * function (Eq. 1) on a flat detector, precomputed once per projection
 * (Sec. "Epipolar Consistency").  Grid: alpha_m = m pi / n_alpha,
 * t_k = -t_max + k 2 t_max / (n_t - 1), t_max = sqrt(W^2 + H^2) / 2 px; line
 * integrals of the cosine-weighted image sampled every ds_px pixels with
 * bilinear interpolation; stored value = central t-difference of the line
 * integrals.  dtype selects the storage (ECC_F32 / ECC_BF16 / ECC_F16; FP16
 * is stored with an exact per-view power-of-two scale).  Runs on `stream`
 * and synchronises it before returning; the projections are then released.
 * Errors: ECC_E_ARG (n_alpha outside [2, 65536], n_t outside [3, 65536],
 * (n_alpha + 1)(n_t + 2) >= 2^28 stored elements per view, ds_px outside
 * (0, 1], bad dtype), ECC_E_STATE (already built), ECC_E_NOSCAN,
 * ECC_E_BUDGET, ECC_E_HIP. */
ecc_status ecc_scan_build_sinograms(ecc_ctx *ctx, int32_t scan_id, int32_t n_alpha, int32_t n_t,
                                    double ds_px, int32_t dtype, void *stream);

/* Installs sinograms computed elsewhere instead of building them (same grid
 * as above).  sino: [n_views][n_alpha + 1][n_t] FP32, row n_alpha holding
 * the values at alpha = pi, host memory (sino_on_device == 0) or device.
 * Converted to `dtype` on the device.  Errors as ecc_scan_build_sinograms. */
ecc_status ecc_scan_set_sinograms(ecc_ctx *ctx, int32_t scan_id, int32_t n_alpha, int32_t n_t,
                                  const float *sino, int32_t sino_on_device, int32_t dtype);

/* Copies one view's resident sinogram back, decoded to FP32, as
 * [n_alpha + 1][n_t] into host memory `out` (synchronous). */
ecc_status ecc_scan_read_sinogram(ecc_ctx *ctx, int32_t scan_id, int32_t view, float *out);

/* Releases a scan and its device memory (after the device is idle). */
ecc_status ecc_scan_free(ecc_ctx *ctx, int32_t scan_id);

/* Device bytes the scan holds now. */
ecc_status ecc_scan_bytes(ecc_ctx *ctx, int32_t scan_id, uint64_t *bytes);

/* Evaluation parameters.
 *   K     number of epipolar planes sampled per pair (Eq. 15), 1..4096;
 *   R_mm  radius of the isocentric object sphere (positive, finite; used by
 *         ECC_KAPPA_OBJECT only);
 *   c     Cauchy parameter of Eq. 16 (c <= 0 or infinite means e = d);
 *   geom  ECC_GEOM_F32 or ECC_GEOM_F64 (per-plane geometry precision);
 *   kappa_range  which planes of the pencil about the baseline C_a C_b are
 *         sampled (the paper leaves the range open, Sec. "Epipolar
 *         Consistency" and Eq. 15's N):
 *     ECC_KAPPA_OBJECT    the planes that meet the object sphere,
 *                         kappa_k = -kappa_max + (k + 1/2) 2 kappa_max / K,
 *                         kappa_max = asin(min(1, R_mm / h)), h = distance
 *                         of the baseline from the isocentre;
 *     ECC_KAPPA_DETECTOR  the arc around kappa = 0 (the plane through the
 *                         isocentre) whose lines meet both detectors,
 *                         kappa_k = lo + (k + 1/2) (hi - lo) / K; a pair
 *                         whose plane at kappa = 0 misses a detector has
 *                         e = 0.  The arc's ends move with theta: the
 *                         gradient follows each end as the zero angle of
 *                         the detector corner whose line fixes it;
 *   reserved  must be 0. */
typedef struct {
    int32_t K;
    int32_t geom;
    double R_mm;
    double c;
    int32_t kappa_range;
    int32_t reserved;
} ecc_eval_params;

/* Device workspace (bytes) an evaluation of B hypotheses needs; with_grad
 * selects ecc_cost_grad. */
ecc_status ecc_workspace_bytes(ecc_ctx *ctx, int32_t scan_id, int32_t B, int32_t with_grad, uint64_t *bytes);

/* Cost of Eq. 17 for B motion hypotheses (Sec. "Optimization"):
 *   theta_dev    [B][n_views][6] FP64 {rx, ry, rz [deg], tx, ty, tz [mm]};
 *                view lam is evaluated with P_lam T(theta), T = [[Rz Ry Rx, t], [0, 1]];
 *   out_cost_dev [B] FP64: sum over pairs a < b of e_ab (Eqs. 15-16);
 *   out_pair_dev [B][n_pairs] FP32 per-pair e_ab, or NULL;
 *   workspace_dev, workspace_bytes: scratch of at least ecc_workspace_bytes.
 * Results are deterministic (fixed reduction order, no atomics).
 * Errors: ECC_E_ARG, ECC_E_NOSCAN, ECC_E_STATE (no sinograms), ECC_E_HIP. */
ecc_status ecc_cost(ecc_ctx *ctx, int32_t scan_id, int32_t B, const double *theta_dev,
                    const ecc_eval_params *params, double *out_cost_dev, float *out_pair_dev,
                    void *workspace_dev, uint64_t workspace_bytes, void *stream);

/* ecc_cost plus the plane count of every pair: out_count_dev [B][n_pairs]
 * int32 (device) = N_kappa of Eq. 15, the sampled planes whose lines hit both
 * detectors (d = 0 when it is 0).  Lets a caller see how many planes carry a
 * pair's term and compare the hit decisions of two precision forms.  Other
 * arguments, the workspace and errors as ecc_cost (ECC_E_ARG for a NULL
 * out_count_dev). */
ecc_status ecc_cost_counts(ecc_ctx *ctx, int32_t scan_id, int32_t B, const double *theta_dev,
                           const ecc_eval_params *params, double *out_cost_dev, float *out_pair_dev,
                           int32_t *out_count_dev, void *workspace_dev, uint64_t workspace_bytes, void *stream);

/* ecc_cost for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving or optimiser loops, harnesses that forbid
 * hipMalloc.  Same kernels, arguments and results as ecc_cost (bitwise), but
 * the workspace is a static device array of 64 MiB per GPU
 * (ECC_NOALLOC_SCRATCH_BYTES) that the library holds until the process ends;
 * the call itself allocates nothing.  It rejects with ECC_E_ARG an
 * evaluation whose workspace (ecc_workspace_bytes with with_grad = 0)
 * exceeds that size, e.g. B > 3 hypotheses of a 496-view scan.  Every call
 * on one GPU shares that GPU's array, so calls that overlap on the device
 * (different streams, or different host threads) race and must be
 * serialised by the caller; the array keeps the last call's contents, and
 * nothing in it needs to start at zero.  Errors as ecc_cost. */
#define ECC_NOALLOC_SCRATCH_BYTES (64ull << 20)
ecc_status ecc_cost_noalloc(ecc_ctx *ctx, int32_t scan_id, int32_t B, const double *theta_dev,
                            const ecc_eval_params *params, double *out_cost_dev, float *out_pair_dev, void *stream);

/* Cost and its gradient with respect to every view's 6 motion parameters
 * (reverse sweep through Eqs. 13-16; the line geometry is recomputed, not
 * stored).  grad_dev [B][n_views][6] FP32 is overwritten.
 * out_pair_grad_dev [B][n_pairs][12] FP32 (d e_ab / d theta_a, then
 * d e_ab / d theta_b) or NULL.  Other arguments as ecc_cost. */
ecc_status ecc_cost_grad(ecc_ctx *ctx, int32_t scan_id, int32_t B, const double *theta_dev,
                         const ecc_eval_params *params, double *out_cost_dev, float *grad_dev,
                         float *out_pair_grad_dev, void *workspace_dev, uint64_t workspace_bytes, void *stream);

/* The prior route to the same cost, kept for comparison (the method the
 * paper improves on; Sec. "Introduction" and "Optimized Algorithm"): every
 * epipolar plane E is mapped to its image line through the pseudo-inverse,
 * l = P'^{+T} E with P'^{+} = P'^T (P' P'^T)^{-1}, which the caller must
 * compute for all moved projection matrices P' = P T(theta) before each
 * evaluation (on the host, as that method does).  The lines equal those of
 * Eqs. 13-14 up to a positive scale, so the cost equals ecc_cost's to
 * rounding.  pinv_dev: [B][n_views][4][3] FP64 device, row-major P'^{+} of
 * hypothesis b, view lam.  Other arguments, the workspace and errors as
 * ecc_cost (ECC_E_ARG for a NULL pinv_dev). */
ecc_status ecc_cost_pinv(ecc_ctx *ctx, int32_t scan_id, int32_t B, const double *theta_dev, const double *pinv_dev,
                         const ecc_eval_params *params, double *out_cost_dev, float *out_pair_dev,
                         void *workspace_dev, uint64_t workspace_bytes, void *stream);

/* Number of views / pairs and the sinogram grid of a scan (any may be NULL). */
ecc_status ecc_scan_info(ecc_ctx *ctx, int32_t scan_id, int32_t *n_views, int32_t *n_pairs, int32_t *n_alpha,
                         int32_t *n_t, int32_t *dtype);

/* ---------------------------------------------------------------------------
 * Motion model of the motion-estimation experiment (Sec. "Optimization"):
 * each of the 6 rigid parameters of view lam follows an Akima spline
 * (Akima 1970) through n_nodes nodes placed at view positions node_x, so an
 * optimiser searches the node values only.  Akima's construction: segment
 * slopes m_i, two linearly extrapolated slopes beyond each end, node
 * derivatives (|m_{i+1} - m_i| m_{i-1} + |m_{i-1} - m_{i-2}| m_i) /
 * (|m_{i+1} - m_i| + |m_{i-1} - m_{i-2}|) (the mean of m_{i-1}, m_i when both
 * weights vanish), cubic Hermite segments.  FP64.
 *   node_x: host [n_nodes], strictly ascending, node_x[0] <= 0 and
 *           node_x[n_nodes - 1] >= n_views - 1; 3 <= n_nodes <= 64.
 *   nodes_dev: device [B][6][n_nodes] FP64 (parameter order as theta).
 * Asynchronous on `stream`.  Errors: ECC_E_ARG, ECC_E_HIP.
 * ------------------------------------------------------------------------- */

/* theta_dev [B][n_views][6] FP64 (device) = the splines at lam = 0 .. n_views - 1. */
ecc_status ecc_spline_motion(ecc_ctx *ctx, int32_t B, int32_t n_views, int32_t n_nodes, const double *node_x,
                             const double *nodes_dev, double *theta_dev, void *stream);

/* Chain rule to the nodes: grad_nodes_dev [B][6][n_nodes] FP64 (device,
 * overwritten) = sum over views of grad_theta_dev [B][n_views][6] FP32 (the
 * gradient ecc_cost_grad writes) times d theta / d node (exact derivative of
 * the piecewise-smooth interpolant; summed in view order, deterministic). */
ecc_status ecc_spline_motion_grad(ecc_ctx *ctx, int32_t B, int32_t n_views, int32_t n_nodes, const double *node_x,
                                  const double *nodes_dev, const float *grad_theta_dev, double *grad_nodes_dev,
                                  void *stream);

/* ---------------------------------------------------------------------------
 * Reconstruction of a compensated scan (Sec. "Experiments" inspects the
 * volume reconstructed with the estimated motion): FDK (Feldkamp, Davis and
 * Kress 1984) for a circular short scan, back-projecting view lam with
 * P'_lam = P_lam T(theta_lam).  Per view: Parker's short-scan weights
 * (Parker 1982; fan angle -atan((u - u0) / f), range [0, pi + 2 delta],
 * delta = (range - pi) / 2) and the cosine weight f / sqrt(f^2 + (u - u0)^2 +
 * (v - v0)^2), the sampled ramp filter along rows (h(0) = 1/4, h(n) =
 * -1 / (pi n)^2 for odd n, 0 for even n; Kak and Slaney ch. 3) scaled by
 * f / D; per voxel x: f(x) = sum over views of dbeta (D / z)^2 Q(u, v) with
 * (u z, v z, z) = P'_lam (x, 1), bilinear, zero off the detector.  D and the
 * orbit angles come from the scan's nominal sources; views must be in
 * increasing orbit angle about +z, evenly spaced (dbeta = range / (N - 1)),
 * over a range between pi + the full fan angle and 2 pi.  FP32.
 * ------------------------------------------------------------------------- */

/* Volume: nx x ny x nz voxels (1..4096 each) of voxel_mm, centred on the
 * isocentre; voxel (i, j, k) at ((i - (nx-1)/2) s, (j - (ny-1)/2) s,
 * (k - (nz-1)/2) s), stored [nz][ny][nx].  reserved must be 0. */
typedef struct {
    int32_t nx, ny, nz;
    int32_t reserved;
    double voxel_mm;
} ecc_volume;

/* Device workspace an ecc_fdk call on this scan needs (the weighted rows,
 * N H W floats, the filtered views, N (H + 3) (W + 4) float pairs, and
 * per-view constants). */
ecc_status ecc_fdk_workspace_bytes(ecc_ctx *ctx, int32_t scan_id, uint64_t *bytes);

/* Reconstructs into out_dev [nz][ny][nx] FP32 (device, overwritten) from
 * images_dev [n_views][H][W] FP32 line integrals (device; the scan's own
 * projections are released once its sinograms exist).  theta_dev [n_views][6]
 * FP64 (device) is the motion to compensate, NULL for none.  Asynchronous on
 * `stream`.  Errors: ECC_E_ARG (bad volume, W > 4096, an orbit that is not a
 * short scan, small workspace), ECC_E_NOSCAN, ECC_E_HIP. */
ecc_status ecc_fdk(ecc_ctx *ctx, int32_t scan_id, const double *theta_dev, const float *images_dev,
                   const ecc_volume *vol, float *out_dev, void *workspace_dev, uint64_t workspace_bytes,
                   void *stream);


/* ---------------------------------------------------------------------------
 * Served form: continuous batching of evaluation requests over resident
 * scans.  A server owns `n_slots` HIP streams and one device arena of
 * `arena_bytes` (the HBM budget for requests' workspaces and buffers) plus a
 * pinned host staging arena.  A worker thread admits queued requests in
 * arrival order as soon as a slot is free and the request's device bytes fit
 * in the arena; admitted requests run concurrently on their slots' streams
 * while later ones keep arriving.  Each request's kernels and reductions do
 * not depend on its neighbours, so its result is the same alone and in the
 * mix (bitwise).  A request for a scan freed before admission fails with
 * ECC_E_NOSCAN; one larger than the whole arena fails with ECC_E_BUDGET.
 * ------------------------------------------------------------------------- */
typedef struct ecc_server ecc_server;

typedef struct {
    double queue_ms;  /* submit -> admission */
    double run_ms;    /* admission -> results on the host */
    double total_ms;  /* submit -> results on the host (the request latency) */
    int32_t slot;     /* stream slot the request ran on */
    int32_t status;   /* ecc_status of the request */
} ecc_request_stats;

/* Creates a server on ctx.  n_slots in [1, 16]; arena_bytes > 0. */
ecc_status ecc_server_create(ecc_ctx *ctx, ecc_server **out, int32_t n_slots, uint64_t arena_bytes);

/* Queues a request: B hypotheses theta_host [B][n_views][6] FP64 (host memory,
 * copied), evaluation parameters, cost only (with_grad = 0) or cost and
 * gradient.  Returns its id.  Never blocks on the device. */
ecc_status ecc_server_submit(ecc_server *srv, int32_t scan_id, int32_t B, const double *theta_host,
                             const ecc_eval_params *params, int32_t with_grad, int64_t *request_id);

/* Sets *done to 1 once the request has finished (successfully or not). */
ecc_status ecc_server_poll(ecc_server *srv, int64_t request_id, int32_t *done);

/* Waits for a request, copies its results -- cost_host [B] FP64 and, for
 * gradient requests, grad_host [B][n_views][6] FP32 (may be NULL) -- and its
 * timing into stats (may be NULL), then forgets the request.  Returns the
 * request's own status. */
ecc_status ecc_server_wait(ecc_server *srv, int64_t request_id, double *cost_host, float *grad_host,
                           ecc_request_stats *stats);

/* Device bytes a request occupies in the arena while it runs. */
ecc_status ecc_server_request_bytes(ecc_server *srv, int32_t scan_id, int32_t B, int32_t with_grad,
                                    uint64_t *bytes);

/* Caps the work in flight: the head of the queue is admitted only while the
 * plane-pair evaluations of the running requests plus its own (B x pairs x
 * K, gradient requests counted twice) stay within work_cap, or when nothing
 * runs.  A large request then shares the device with small ones only, which
 * bounds the tail latency that sharing adds.  0 (the default) = admission by
 * free slot and arena only.  Applies to later admissions.  Errors: ECC_E_ARG
 * (NULL server, negative or non-finite cap). */
ecc_status ecc_server_set_work_cap(ecc_server *srv, double work_cap);

/* Stops the worker after the requests already admitted finish, fails the
 * queued ones, and frees the server's streams and arenas. */
ecc_status ecc_server_destroy(ecc_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* ECC_H */
