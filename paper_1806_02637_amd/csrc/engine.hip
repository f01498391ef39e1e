// Host engine behind include/ecc.h: contexts, resident scans under an HBM
// budget, argument checking, workspace layout and kernel sequencing.  Every
// entry point returns a status and records a thread-local message; nothing
// here aborts.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ecc.h"
#include "ecc_internal.hpp"
#include "fdk.hpp"
#include "poly_coeffs.hpp"

using namespace ecc;

namespace {

thread_local std::string g_err;

ecc_status fail(ecc_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

ecc_status ok() {
    g_err.clear();
    return ECC_OK;
}

#define HIP_TRY(expr)                                                                                       \
    do {                                                                                                    \
        hipError_t _e = (expr);                                                                             \
        if (_e != hipSuccess) return fail(ECC_E_HIP, "%s failed: %s", #expr, hipGetErrorString(_e));        \
    } while (0)

struct Scan {
    int32_t n_views = 0, W = 0, H = 0;
    double *P_dev = nullptr;     // [N][12]
    double *intr_dev = nullptr;  // [N][3]
    float *images_dev = nullptr; // [N][H][W] until sinograms exist
    void *sino_dev = nullptr;
    float *scale_dev = nullptr;  // [N]
    uint32_t *absmax_dev = nullptr;
    std::vector<double> P_host, intr_host;  // copies for host-side geometry checks
    SinoLayout layout{};
    double ds_px = 0.0;
    bool built = false;
    uint64_t bytes = 0;
};

}  // namespace

// ---------------------------------------------------------------------------
// Device scratch of the allocation-free cost entry point (ecc_cost_noalloc):
// one array per GPU, held until the process ends.  Host code never uses the
// array's name as an address: each device's copy is resolved once with
// hipGetSymbolAddress (in ecc_create, with that device current) and only
// that pointer is handed to kernels.
constexpr uint64_t kNoAllocScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

struct ecc_ctx {
    int device = 0;
    uint64_t budget = 0, used = 0;
    std::mutex mu;
    std::map<int32_t, Scan *> scans;
    int32_t next_id = 1;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Allocation charged to the context budget.
ecc_status ctx_alloc(ecc_ctx *ctx, void **p, uint64_t bytes, uint64_t *charged) {
    if (ctx->budget && ctx->used + bytes > ctx->budget)
        return fail(ECC_E_BUDGET, "allocation of %llu bytes exceeds the HBM budget (%llu of %llu in use)",
                    (unsigned long long)bytes, (unsigned long long)ctx->used, (unsigned long long)ctx->budget);
    hipError_t e = hipMalloc(p, bytes ? bytes : 1);
    if (e != hipSuccess) return fail(ECC_E_HIP, "hipMalloc(%llu) failed: %s", (unsigned long long)bytes,
                                     hipGetErrorString(e));
    ctx->used += bytes;
    *charged += bytes;
    return ECC_OK;
}

void ctx_free(ecc_ctx *ctx, void *&p, uint64_t bytes, uint64_t *charged) {
    if (p) {
        (void)hipFree(p);
        ctx->used -= bytes;
        *charged -= bytes;
        p = nullptr;
    }
}

Scan *find_scan(ecc_ctx *ctx, int32_t id) {
    auto it = ctx->scans.find(id);
    return it == ctx->scans.end() ? nullptr : it->second;
}

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// largest accepted distance (px) of a view's principal point from the
// detector centre
constexpr double kPrincipalTolPx = 1e-6;

int n_tiles_for(int n_views) {
    const int nb = (n_views + 7) / 8;  // 8-view blocks, tiles = block pairs I <= J
    return nb * (nb + 1) / 2;
}
// Work tiles of the plane kernels (pair tiles, each cut into
// pair_subtiles(B) parts): one FP64 partial sum per hypothesis and work tile.
int n_work_tiles(int n_views, int B) { return n_tiles_for(n_views) * pair_subtiles(B); }

// Workspace layout of an evaluation.
struct Workspace {
    uint64_t vt_off, vg_off, table_off, part_off, sens_off, pgrad_off, total;
};

Workspace workspace_layout(const Scan *s, int B, bool grad) {
    const int64_t n_pairs = (int64_t)s->n_views * (s->n_views - 1) / 2;
    Workspace w{};
    uint64_t off = 0;
    w.vt_off = off;
    off += align256(sizeof(ViewGeom) * (uint64_t)B * s->n_views);
    w.vg_off = off;
    if (grad) off += align256(sizeof(ViewGeomGrad) * (uint64_t)B * s->n_views);
    w.table_off = off;  // sized for the FP64 plane-geometry form, the larger one
    off += align256(pair_const_bytes(true) * (uint64_t)B * n_pairs);
    w.part_off = off;
    off += align256(sizeof(double) * (uint64_t)B * n_work_tiles(s->n_views, B));
    w.sens_off = off;
    if (grad) off += align256(sizeof(float) * 14ull * (uint64_t)B * n_pairs);  // per-pair sensitivities
    w.pgrad_off = off;
    if (grad) off += align256(sizeof(float) * 12ull * (uint64_t)B * n_pairs);
    w.total = off;
    return w;
}

ecc_status free_scan_memory(ecc_ctx *ctx, Scan *s) {
    (void)hipDeviceSynchronize();
    ctx_free(ctx, (void *&)s->P_dev, sizeof(double) * 12ull * s->n_views, &s->bytes);
    ctx_free(ctx, (void *&)s->intr_dev, sizeof(double) * 3ull * s->n_views, &s->bytes);
    ctx_free(ctx, (void *&)s->images_dev, sizeof(float) * (uint64_t)s->n_views * s->W * s->H, &s->bytes);
    if (s->sino_dev)
        ctx_free(ctx, s->sino_dev, (uint64_t)s->layout.elem_bytes * s->layout.view_elems * s->n_views, &s->bytes);
    ctx_free(ctx, (void *&)s->scale_dev, sizeof(float) * s->n_views, &s->bytes);
    ctx_free(ctx, (void *&)s->absmax_dev, sizeof(uint32_t) * s->n_views, &s->bytes);
    return ECC_OK;
}

ecc_status check_eval(ecc_ctx *ctx, int32_t scan_id, int32_t B, const ecc_eval_params *prm, Scan **out) {
    if (!ctx) return fail(ECC_E_ARG, "null context");
    Scan *s = find_scan(ctx, scan_id);
    if (!s) return fail(ECC_E_NOSCAN, "unknown scan id %d", scan_id);
    if (!s->built) return fail(ECC_E_STATE, "scan %d has no sinograms yet", scan_id);
    if (B < 1 || B > 65536) return fail(ECC_E_ARG, "B = %d out of range [1, 65536]", B);
    if (!prm) return fail(ECC_E_ARG, "null params");
    if (prm->K < 1 || prm->K > 4096) return fail(ECC_E_ARG, "K = %d out of range [1, 4096]", prm->K);
    if (!(prm->R_mm > 0.0) || !isfinite(prm->R_mm)) return fail(ECC_E_ARG, "R_mm must be positive and finite");
    if (prm->geom != ECC_GEOM_F32 && prm->geom != ECC_GEOM_F64) return fail(ECC_E_ARG, "unknown geom %d", prm->geom);
    if (isnan(prm->c)) return fail(ECC_E_ARG, "c is NaN");
    if (prm->kappa_range != ECC_KAPPA_OBJECT && prm->kappa_range != ECC_KAPPA_DETECTOR)
        return fail(ECC_E_ARG, "unknown kappa_range %d", prm->kappa_range);
    if (prm->reserved != 0) return fail(ECC_E_ARG, "reserved field must be 0");
    *out = s;
    return ECC_OK;
}

EvalConsts make_consts(const Scan *s, int B, const ecc_eval_params *prm) {
    EvalConsts ec{};
    ec.n_views = s->n_views;
    ec.n_pairs = (int32_t)((int64_t)s->n_views * (s->n_views - 1) / 2);
    ec.K = prm->K;
    ec.B = B;
    ec.n_alpha = s->layout.n_alpha;
    ec.n_t = s->layout.n_t;
    ec.row_elems = s->layout.row_elems;
    ec.view_elems = s->layout.view_elems;
    ec.geom64 = prm->geom == ECC_GEOM_F64;
    ec.R_mm = prm->R_mm;
    ec.kappa_detector = prm->kappa_range == ECC_KAPPA_DETECTOR;
    ec.inv_c = (prm->c > 0.0 && isfinite(prm->c)) ? (float)(1.0 / prm->c) : 0.0f;
    ec.half_w = 0.5f * s->W;
    ec.half_h = 0.5f * s->H;
    const double t_max = 0.5 * sqrt((double)s->W * s->W + (double)s->H * s->H);
    const double dt = 2.0 * t_max / (s->layout.n_t - 1);
    const double dalpha = M_PI / s->layout.n_alpha;
    ec.t0_tau_d = (t_max + dt) / dt;
    ec.inv_dt_d = 1.0 / dt;
    ec.inv_dalpha_d = 1.0 / dalpha;
    ec.t0_tau = (float)((t_max + dt) / dt);
    ec.inv_dt = (float)(1.0 / dt);
    ec.inv_dalpha = (float)(1.0 / dalpha);
    // the plane angle's polynomial for this storage type, in rows
    const int dtype = s->layout.dtype;
    static_assert(kAsinTermsF32 == 7 && kAsinTerms16 == 6, "coefficient tables: kAsin (7 terms), kAsin6 (6)");
    const float *c = dtype == 0 ? kAsin : kAsin6;
    const int n = dtype == 0 ? kAsinTermsF32 : kAsinTerms16;
    for (int i = 0; i < 7; ++i) ec.asin_rows[i] = i < n ? (float)((double)c[i] / dalpha) : 0.0f;
    ec.rows_half_pi = (float)(0.5 * s->layout.n_alpha);
    ec.rows_pi = (float)s->layout.n_alpha;
    return ec;
}

}  // namespace

namespace ecc {
int ctx_device(ecc_ctx *ctx) { return ctx->device; }
int32_t set_error(int32_t code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
}  // namespace ecc

extern "C" {

const char *ecc_last_error(void) { return g_err.c_str(); }

ecc_status ecc_create(ecc_ctx **out, int hip_device, uint64_t hbm_budget_bytes) {
    if (!out) return fail(ECC_E_ARG, "null output pointer");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return fail(ECC_E_HIP, "hipGetDeviceCount failed: %s", hipGetErrorString(e));
    if (hip_device < 0 || hip_device >= n) return fail(ECC_E_ARG, "device %d not present (%d devices)", hip_device, n);
    if (hip_device >= kMaxScratchDevices)
        return fail(ECC_E_ARG, "device %d beyond the %d devices the engine supports", hip_device, kMaxScratchDevices);
    {
        // this device's copy of the no-alloc scratch, resolved once with the
        // device current
        DeviceGuard g(hip_device);
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[hip_device]) {
            void *ptr = nullptr;
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return fail(ECC_E_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", hip_device,
                            hipGetErrorString(e));
            g_scratch_ptr[hip_device] = ptr;
        }
    }
    ecc_ctx *ctx = new ecc_ctx();
    ctx->device = hip_device;
    ctx->budget = hbm_budget_bytes;
    *out = ctx;
    return ok();
}

ecc_status ecc_destroy(ecc_ctx *ctx) {
    if (!ctx) return fail(ECC_E_ARG, "null context");
    {
        DeviceGuard g(ctx->device);
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (auto &kv : ctx->scans) {
            free_scan_memory(ctx, kv.second);
            delete kv.second;
        }
        ctx->scans.clear();
    }
    delete ctx;
    return ok();
}

ecc_status ecc_scan_load(ecc_ctx *ctx, int32_t *scan_id, int32_t n_views, int32_t W, int32_t H, const double *P,
                         const double *intr, const float *images, int32_t images_on_device) {
    if (!ctx || !scan_id || !P || !intr || !images) return fail(ECC_E_ARG, "null argument");
    if (n_views < 2 || n_views > 65536) return fail(ECC_E_ARG, "n_views = %d out of range [2, 65536]", n_views);
    if (W < 2 || H < 2 || W > 32768 || H > 32768) return fail(ECC_E_ARG, "detector %dx%d out of range", W, H);
    int sign = 0;
    for (int v = 0; v < n_views; ++v) {
        const double *p = P + 12 * v;
        for (int i = 0; i < 12; ++i)
            if (!isfinite(p[i])) return fail(ECC_E_ARG, "non-finite projection matrix entry (view %d)", v);
        for (int i = 0; i < 3; ++i)
            if (!isfinite(intr[3 * v + i])) return fail(ECC_E_ARG, "non-finite intrinsics (view %d)", v);
        if (!(intr[3 * v] > 0.0)) return fail(ECC_E_ARG, "focal length must be positive (view %d)", v);
        // the hit test of Eq. 15 and the sinogram's t range are centred on
        // the principal point, so it must be the detector centre
        if (fabs(intr[3 * v + 1] - 0.5 * (W - 1)) > kPrincipalTolPx || fabs(intr[3 * v + 2] - 0.5 * (H - 1)) > kPrincipalTolPx)
            return fail(ECC_E_ARG,
                        "principal point (%.6f, %.6f) of view %d is not the detector centre ((W-1)/2, (H-1)/2) = "
                        "(%.6f, %.6f)",
                        intr[3 * v + 1], intr[3 * v + 2], v, 0.5 * (W - 1), 0.5 * (H - 1));
        const double det = p[0] * (p[5] * p[10] - p[6] * p[9]) - p[1] * (p[4] * p[10] - p[6] * p[8]) +
                           p[2] * (p[4] * p[9] - p[5] * p[8]);
        const int sg = det > 0 ? 1 : (det < 0 ? -1 : 0);
        if (sg == 0) return fail(ECC_E_ARG, "singular left 3x3 of P (view %d)", v);
        if (sign == 0) sign = sg;
        if (sg != sign) return fail(ECC_E_ARG, "views differ in detector handedness (sign of det M, view %d)", v);
    }
    DeviceGuard g(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->mu);
    Scan *s = new Scan();
    s->n_views = n_views;
    s->P_host.assign(P, P + 12ull * n_views);
    s->intr_host.assign(intr, intr + 3ull * n_views);
    s->W = W;
    s->H = H;
    ecc_status st;
    const uint64_t img_bytes = sizeof(float) * (uint64_t)n_views * W * H;
    if ((st = ctx_alloc(ctx, (void **)&s->P_dev, sizeof(double) * 12ull * n_views, &s->bytes)) ||
        (st = ctx_alloc(ctx, (void **)&s->intr_dev, sizeof(double) * 3ull * n_views, &s->bytes)) ||
        (st = ctx_alloc(ctx, (void **)&s->images_dev, img_bytes, &s->bytes)) ||
        (st = ctx_alloc(ctx, (void **)&s->scale_dev, sizeof(float) * n_views, &s->bytes)) ||
        (st = ctx_alloc(ctx, (void **)&s->absmax_dev, sizeof(uint32_t) * n_views, &s->bytes))) {
        std::string msg = g_err;
        free_scan_memory(ctx, s);
        delete s;
        g_err = msg;
        return st;
    }
    hipError_t e1 = hipMemcpy(s->P_dev, P, sizeof(double) * 12ull * n_views, hipMemcpyHostToDevice);
    hipError_t e2 = hipMemcpy(s->intr_dev, intr, sizeof(double) * 3ull * n_views, hipMemcpyHostToDevice);
    hipError_t e3 = hipMemcpy(s->images_dev, images, img_bytes,
                              images_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        hipError_t e = e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3);
        free_scan_memory(ctx, s);
        delete s;
        return fail(ECC_E_HIP, "copying scan inputs failed: %s", hipGetErrorString(e));
    }
    const int32_t id = ctx->next_id++;
    ctx->scans[id] = s;
    *scan_id = id;
    return ok();
}

static ecc_status install_sinograms(ecc_ctx *ctx, Scan *s, int32_t n_alpha, int32_t n_t, double ds_px, int32_t dtype,
                                    const float *ext_host, const float *ext_dev, hipStream_t stream) {
    const SinoLayout L = make_layout(s->n_views, n_alpha, n_t, dtype);
    const uint64_t sino_bytes = (uint64_t)L.elem_bytes * L.view_elems * s->n_views;
    ecc_status st = ctx_alloc(ctx, &s->sino_dev, sino_bytes, &s->bytes);
    if (st) return st;
    s->layout = L;
    // temporaries (charged while they live)
    uint64_t tmp_charged = 0;
    float *gw = nullptr, *gwT = nullptr, *ext_tmp = nullptr;
    double *G = nullptr;
    // weighted projections in two orientations, rows stored as interleaved pairs
    const uint64_t pad_bytes = 2 * sizeof(float) * (uint64_t)s->n_views * (s->W + 2 * kImgPad) * (s->H + 2 * kImgPad);
    const uint64_t G_bytes = sizeof(double) * (uint64_t)s->n_views * n_alpha * n_t;
    const uint64_t ext_bytes = sizeof(float) * (uint64_t)s->n_views * (n_alpha + 1) * n_t;
    auto cleanup = [&]() {
        ctx_free(ctx, (void *&)gw, pad_bytes, &tmp_charged);
        ctx_free(ctx, (void *&)gwT, pad_bytes, &tmp_charged);
        ctx_free(ctx, (void *&)G, G_bytes, &tmp_charged);
        ctx_free(ctx, (void *&)ext_tmp, ext_bytes, &tmp_charged);
    };
    auto bail = [&](ecc_status code) {
        std::string msg = g_err;
        (void)hipStreamSynchronize(stream);
        cleanup();
        ctx_free(ctx, s->sino_dev, sino_bytes, &s->bytes);
        g_err = msg;
        return code;
    };
    hipError_t e;
    const float *ext = ext_dev;
    if (ext_host) {
        if ((st = ctx_alloc(ctx, (void **)&ext_tmp, ext_bytes, &tmp_charged))) return bail(st);
        if ((e = hipMemcpyAsync(ext_tmp, ext_host, ext_bytes, hipMemcpyHostToDevice, stream)) != hipSuccess)
            return bail(fail(ECC_E_HIP, "sinogram upload failed: %s", hipGetErrorString(e)));
        ext = ext_tmp;
    }
    if (!ext) {
        if ((st = ctx_alloc(ctx, (void **)&gw, pad_bytes, &tmp_charged)) ||
            (st = ctx_alloc(ctx, (void **)&gwT, pad_bytes, &tmp_charged)) ||
            (st = ctx_alloc(ctx, (void **)&G, G_bytes, &tmp_charged)))
            return bail(st);
        if ((e = hipMemsetAsync(gw, 0, pad_bytes, stream)) != hipSuccess ||
            (e = hipMemsetAsync(gwT, 0, pad_bytes, stream)) != hipSuccess ||
            (e = launch_sino_weight(s->images_dev, s->intr_dev, s->n_views, s->W, s->H, gw, gwT, stream)) !=
                hipSuccess ||
            (e = launch_sino_radon(gw, gwT, s->intr_dev, s->n_views, s->W, s->H, n_alpha, n_t, ds_px, G, stream)) !=
                hipSuccess)
            return bail(fail(ECC_E_HIP, "sinogram build launch failed: %s", hipGetErrorString(e)));
    }
    const double t_max = 0.5 * sqrt((double)s->W * s->W + (double)s->H * s->H);
    const double dt = 2.0 * t_max / (n_t - 1);
    if ((e = launch_sino_store(G, ext, s->n_views, n_alpha, n_t, dt, dtype, s->sino_dev, s->scale_dev,
                               s->absmax_dev, stream)) != hipSuccess)
        return bail(fail(ECC_E_HIP, "sinogram store launch failed: %s", hipGetErrorString(e)));
    if ((e = hipStreamSynchronize(stream)) != hipSuccess)
        return bail(fail(ECC_E_HIP, "sinogram build failed: %s", hipGetErrorString(e)));
    cleanup();
    ctx_free(ctx, (void *&)s->images_dev, sizeof(float) * (uint64_t)s->n_views * s->W * s->H, &s->bytes);
    s->ds_px = ds_px;
    s->built = true;
    return ok();
}

ecc_status ecc_scan_build_sinograms(ecc_ctx *ctx, int32_t scan_id, int32_t n_alpha, int32_t n_t, double ds_px,
                                    int32_t dtype, void *stream) {
    if (!ctx) return fail(ECC_E_ARG, "null context");
    if (n_alpha < 2 || n_alpha > 65536 || n_t < 3 || n_t > 65536 || (int64_t)(n_alpha + 1) * (n_t + 2) >= (1ll << 28))
        return fail(ECC_E_ARG, "sinogram grid %d x %d out of range", n_alpha, n_t);
    if (!(ds_px > 0.0) || ds_px > 1.0) return fail(ECC_E_ARG, "ds_px must be in (0, 1]");
    if (dtype < ECC_F32 || dtype > ECC_F16) return fail(ECC_E_ARG, "unknown dtype %d", dtype);
    DeviceGuard g(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->mu);
    Scan *s = find_scan(ctx, scan_id);
    if (!s) return fail(ECC_E_NOSCAN, "unknown scan id %d", scan_id);
    if (s->built || !s->images_dev) return fail(ECC_E_STATE, "scan %d already has sinograms", scan_id);
    return install_sinograms(ctx, s, n_alpha, n_t, ds_px, dtype, nullptr, nullptr, (hipStream_t)stream);
}

ecc_status ecc_scan_set_sinograms(ecc_ctx *ctx, int32_t scan_id, int32_t n_alpha, int32_t n_t, const float *sino,
                                  int32_t sino_on_device, int32_t dtype) {
    if (!ctx || !sino) return fail(ECC_E_ARG, "null argument");
    if (n_alpha < 2 || n_alpha > 65536 || n_t < 3 || n_t > 65536 || (int64_t)(n_alpha + 1) * (n_t + 2) >= (1ll << 28))
        return fail(ECC_E_ARG, "sinogram grid %d x %d out of range", n_alpha, n_t);
    if (dtype < ECC_F32 || dtype > ECC_F16) return fail(ECC_E_ARG, "unknown dtype %d", dtype);
    DeviceGuard g(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->mu);
    Scan *s = find_scan(ctx, scan_id);
    if (!s) return fail(ECC_E_NOSCAN, "unknown scan id %d", scan_id);
    if (s->built) return fail(ECC_E_STATE, "scan %d already has sinograms", scan_id);
    return install_sinograms(ctx, s, n_alpha, n_t, 0.0, dtype, sino_on_device ? nullptr : sino,
                             sino_on_device ? sino : nullptr, nullptr);
}

ecc_status ecc_scan_read_sinogram(ecc_ctx *ctx, int32_t scan_id, int32_t view, float *out) {
    if (!ctx || !out) return fail(ECC_E_ARG, "null argument");
    DeviceGuard g(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->mu);
    Scan *s = find_scan(ctx, scan_id);
    if (!s) return fail(ECC_E_NOSCAN, "unknown scan id %d", scan_id);
    if (!s->built) return fail(ECC_E_STATE, "scan %d has no sinograms yet", scan_id);
    if (view < 0 || view >= s->n_views) return fail(ECC_E_ARG, "view %d out of range", view);
    const uint64_t n = (uint64_t)(s->layout.n_alpha + 1) * s->layout.n_t;
    float *tmp = nullptr;
    HIP_TRY(hipMalloc((void **)&tmp, n * sizeof(float)));
    hipError_t e = launch_sino_read(s->sino_dev, s->scale_dev, s->layout, view, tmp, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out, tmp, n * sizeof(float), hipMemcpyDeviceToHost);
    (void)hipFree(tmp);
    if (e != hipSuccess) return fail(ECC_E_HIP, "reading sinogram failed: %s", hipGetErrorString(e));
    return ok();
}

ecc_status ecc_scan_free(ecc_ctx *ctx, int32_t scan_id) {
    if (!ctx) return fail(ECC_E_ARG, "null context");
    DeviceGuard g(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->mu);
    Scan *s = find_scan(ctx, scan_id);
    if (!s) return fail(ECC_E_NOSCAN, "unknown scan id %d", scan_id);
    free_scan_memory(ctx, s);
    ctx->scans.erase(scan_id);
    delete s;
    return ok();
}

ecc_status ecc_scan_bytes(ecc_ctx *ctx, int32_t scan_id, uint64_t *bytes) {
    if (!ctx || !bytes) return fail(ECC_E_ARG, "null argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    Scan *s = find_scan(ctx, scan_id);
    if (!s) return fail(ECC_E_NOSCAN, "unknown scan id %d", scan_id);
    *bytes = s->bytes;
    return ok();
}

ecc_status ecc_scan_info(ecc_ctx *ctx, int32_t scan_id, int32_t *n_views, int32_t *n_pairs, int32_t *n_alpha,
                         int32_t *n_t, int32_t *dtype) {
    if (!ctx) return fail(ECC_E_ARG, "null context");
    std::lock_guard<std::mutex> lk(ctx->mu);
    Scan *s = find_scan(ctx, scan_id);
    if (!s) return fail(ECC_E_NOSCAN, "unknown scan id %d", scan_id);
    if (n_views) *n_views = s->n_views;
    if (n_pairs) *n_pairs = (int32_t)((int64_t)s->n_views * (s->n_views - 1) / 2);
    if (n_alpha) *n_alpha = s->layout.n_alpha;
    if (n_t) *n_t = s->layout.n_t;
    if (dtype) *dtype = s->built ? s->layout.dtype : -1;
    return ok();
}

static ecc_status check_spline(ecc_ctx *ctx, int32_t B, int32_t n_views, int32_t n_nodes, const double *node_x,
                               SplineKnots *kn) {
    if (!ctx || !node_x) return fail(ECC_E_ARG, "null argument");
    if (B < 1 || B > 65536) return fail(ECC_E_ARG, "B = %d out of range [1, 65536]", B);
    if (n_views < 2 || n_views > 65536) return fail(ECC_E_ARG, "n_views = %d out of range [2, 65536]", n_views);
    if (n_nodes < 3 || n_nodes > kMaxSplineNodes)
        return fail(ECC_E_ARG, "n_nodes = %d out of range [3, %d]", n_nodes, kMaxSplineNodes);
    kn->n = n_nodes;
    for (int j = 0; j < n_nodes; ++j) {
        if (!isfinite(node_x[j])) return fail(ECC_E_ARG, "non-finite node position %d", j);
        if (j > 0 && !(node_x[j] > node_x[j - 1])) return fail(ECC_E_ARG, "node positions must ascend strictly");
        kn->x[j] = node_x[j];
    }
    if (node_x[0] > 0.0 || node_x[n_nodes - 1] < (double)(n_views - 1))
        return fail(ECC_E_ARG, "nodes must cover the views [0, %d]", n_views - 1);
    return ECC_OK;
}

// ---------------------------------------------------------------------------
// FDK reconstruction of a compensated scan.

namespace {

struct FdkWorkspace {
    uint64_t theta_off, nom_off, mov_off, views_off, pw_off, xw_off, q_off, total;
};

FdkWorkspace fdk_workspace_layout(const Scan *s) {
    FdkWorkspace w{};
    uint64_t off = 0;
    w.theta_off = off;
    off += align256(sizeof(double) * 6ull * s->n_views);
    w.nom_off = off;
    off += align256(sizeof(ViewGeom) * (uint64_t)s->n_views);
    w.mov_off = off;
    off += align256(sizeof(ViewGeom) * (uint64_t)s->n_views);
    w.views_off = off;
    off += align256(sizeof(FdkView) * (uint64_t)s->n_views);
    w.pw_off = off;
    off += align256(sizeof(float) * (uint64_t)s->n_views * s->W);
    w.xw_off = off;
    off += align256(sizeof(float) * (uint64_t)s->n_views * s->H * s->W);
    w.q_off = off;
    off += align256(sizeof(float) * 2ull * s->n_views * (s->H + 3) * (uint64_t)(s->W + 4));
    w.total = off;
    return w;
}

// The nominal orbit must be a short scan about the z axis: views in order of
// increasing orbit angle atan2(C_y, C_x), a range between pi + the fan angle
// and 2 pi (Parker's weights need the range to cover every ray once).
ecc_status check_fdk_orbit(const Scan *s) {
    const int n = s->n_views;
    double b0 = 0.0, prev = -1.0, fan = 0.0;
    std::vector<double> betas(n);
    for (int v = 0; v < n; ++v) {
        const double *p = s->P_host.data() + 12 * v;
        // source: the null vector of P, C = -M^{-1} p4 (Cramer's rule)
        const double a = p[0], b = p[1], c = p[2], d = p[4], e = p[5], f = p[6], g = p[8], h = p[9], i = p[10];
        const double det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
        const double r0 = -p[3], r1 = -p[7], r2 = -p[11];
        const double cx = (r0 * (e * i - f * h) - b * (r1 * i - f * r2) + c * (r1 * h - e * r2)) / det;
        const double cy = (a * (r1 * i - f * r2) - r0 * (d * i - f * g) + c * (d * r2 - r1 * g)) / det;
        double beta = atan2(cy, cx);
        if (v == 0) b0 = beta;
        beta = fmod(beta - b0, 2.0 * M_PI);
        if (beta < 0.0) beta += 2.0 * M_PI;
        if (v > 0 && !(beta > prev)) return fail(ECC_E_ARG, "FDK needs views in increasing orbit angle (view %d)", v);
        prev = beta;
        betas[v] = beta;
        const double fpx = s->intr_host[3 * v], u0 = s->intr_host[3 * v + 1];
        fan = fmax(fan, fmax(fabs(atan(u0 / fpx)), fabs(atan((s->W - 1 - u0) / fpx))));
    }
    if (!(prev > M_PI + 2.0 * fan) || !(prev < 2.0 * M_PI))
        return fail(ECC_E_ARG, "orbit range %.4f rad is not a short scan (needs pi + %.4f rad, less than 2 pi)", prev,
                    2.0 * fan);
    // the back-projection weighs every view by the same step range / (N - 1)
    const double step = prev / (n - 1);
    for (int v = 0; v < n; ++v)
        if (fabs(betas[v] - v * step) > 0.01 * step)
            return fail(ECC_E_ARG, "FDK needs evenly spaced views (view %d is %.3g steps off)", v,
                        (betas[v] - v * step) / step);
    return ECC_OK;
}

}  // namespace

ecc_status ecc_fdk_workspace_bytes(ecc_ctx *ctx, int32_t scan_id, uint64_t *bytes) {
    if (!ctx || !bytes) return fail(ECC_E_ARG, "null argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    Scan *s = find_scan(ctx, scan_id);
    if (!s) return fail(ECC_E_NOSCAN, "unknown scan id %d", scan_id);
    *bytes = fdk_workspace_layout(s).total;
    return ECC_OK;
}

ecc_status ecc_fdk(ecc_ctx *ctx, int32_t scan_id, const double *theta_dev, const float *images_dev,
                   const ecc_volume *vol, float *out_dev, void *workspace_dev, uint64_t workspace_bytes,
                   void *stream) {
    if (!ctx || !vol || !images_dev || !out_dev || !workspace_dev) return fail(ECC_E_ARG, "null argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    Scan *s = find_scan(ctx, scan_id);
    if (!s) return fail(ECC_E_NOSCAN, "unknown scan id %d", scan_id);
    if (vol->nx < 1 || vol->ny < 1 || vol->nz < 1 || vol->nx > 4096 || vol->ny > 4096 || vol->nz > 4096)
        return fail(ECC_E_ARG, "volume %dx%dx%d out of range [1, 4096]", vol->nx, vol->ny, vol->nz);
    if (!(vol->voxel_mm > 0.0) || !isfinite(vol->voxel_mm)) return fail(ECC_E_ARG, "voxel_mm must be positive");
    if (vol->reserved != 0) return fail(ECC_E_ARG, "reserved field must be 0");
    if (s->W > 4096) return fail(ECC_E_ARG, "FDK filters rows of at most 4096 pixels (W = %d)", s->W);
    ecc_status st;
    if ((st = check_fdk_orbit(s))) return st;
    const FdkWorkspace w = fdk_workspace_layout(s);
    if (workspace_bytes < w.total)
        return fail(ECC_E_ARG, "workspace of %llu bytes is smaller than the %llu needed",
                    (unsigned long long)workspace_bytes, (unsigned long long)w.total);
    DeviceGuard g(ctx->device);
    hipStream_t hs = (hipStream_t)stream;
    char *ws = (char *)workspace_dev;
    double *zero = (double *)(ws + w.theta_off);
    ViewGeom *nom = (ViewGeom *)(ws + w.nom_off);
    ViewGeom *mov = (ViewGeom *)(ws + w.mov_off);
    HIP_TRY(hipMemsetAsync(zero, 0, sizeof(double) * 6ull * s->n_views, hs));
    HIP_TRY(launch_view_setup(s->P_dev, s->intr_dev, zero, 1, s->n_views, nom, nullptr, hs));
    if (theta_dev) HIP_TRY(launch_view_setup(s->P_dev, s->intr_dev, theta_dev, 1, s->n_views, mov, nullptr, hs));
    const FdkVolume fv{vol->nx, vol->ny, vol->nz, (float)vol->voxel_mm};
    HIP_TRY(launch_fdk(images_dev, nom, theta_dev ? mov : nom, s->n_views, s->W, s->H, fv,
                       (FdkView *)(ws + w.views_off), (float *)(ws + w.pw_off), (float *)(ws + w.xw_off),
                       (float2 *)(ws + w.q_off), out_dev, hs));
    return ECC_OK;
}

ecc_status ecc_spline_motion(ecc_ctx *ctx, int32_t B, int32_t n_views, int32_t n_nodes, const double *node_x,
                             const double *nodes_dev, double *theta_dev, void *stream) {
    SplineKnots kn;
    ecc_status st = check_spline(ctx, B, n_views, n_nodes, node_x, &kn);
    if (st != ECC_OK) return st;
    if (!nodes_dev || !theta_dev) return fail(ECC_E_ARG, "null argument");
    DeviceGuard g(ctx->device);
    HIP_TRY(launch_spline_motion(kn, B, n_views, nodes_dev, theta_dev, (hipStream_t)stream));
    return ok();
}

ecc_status ecc_spline_motion_grad(ecc_ctx *ctx, int32_t B, int32_t n_views, int32_t n_nodes, const double *node_x,
                                  const double *nodes_dev, const float *grad_theta_dev, double *grad_nodes_dev,
                                  void *stream) {
    SplineKnots kn;
    ecc_status st = check_spline(ctx, B, n_views, n_nodes, node_x, &kn);
    if (st != ECC_OK) return st;
    if (!nodes_dev || !grad_theta_dev || !grad_nodes_dev) return fail(ECC_E_ARG, "null argument");
    DeviceGuard g(ctx->device);
    HIP_TRY(launch_spline_grad(kn, B, n_views, nodes_dev, grad_theta_dev, grad_nodes_dev, (hipStream_t)stream));
    return ok();
}

ecc_status ecc_workspace_bytes(ecc_ctx *ctx, int32_t scan_id, int32_t B, int32_t with_grad, uint64_t *bytes) {
    if (!ctx || !bytes) return fail(ECC_E_ARG, "null argument");
    if (B < 1 || B > 65536) return fail(ECC_E_ARG, "B = %d out of range [1, 65536]", B);
    std::lock_guard<std::mutex> lk(ctx->mu);
    Scan *s = find_scan(ctx, scan_id);
    if (!s) return fail(ECC_E_NOSCAN, "unknown scan id %d", scan_id);
    *bytes = workspace_layout(s, B, with_grad != 0).total;
    return ok();
}

static ecc_status cost_impl(ecc_ctx *ctx, int32_t scan_id, int32_t B, const double *theta_dev,
                            const double *pinv_dev, const ecc_eval_params *params, double *out_cost_dev,
                            float *out_pair_dev, int32_t *out_count_dev, void *workspace_dev,
                            uint64_t workspace_bytes, void *stream);

ecc_status ecc_cost(ecc_ctx *ctx, int32_t scan_id, int32_t B, const double *theta_dev, const ecc_eval_params *params,
                    double *out_cost_dev, float *out_pair_dev, void *workspace_dev, uint64_t workspace_bytes,
                    void *stream) {
    return cost_impl(ctx, scan_id, B, theta_dev, nullptr, params, out_cost_dev, out_pair_dev, nullptr,
                     workspace_dev, workspace_bytes, stream);
}

ecc_status ecc_cost_counts(ecc_ctx *ctx, int32_t scan_id, int32_t B, const double *theta_dev,
                           const ecc_eval_params *params, double *out_cost_dev, float *out_pair_dev,
                           int32_t *out_count_dev, void *workspace_dev, uint64_t workspace_bytes, void *stream) {
    if (!out_count_dev) return fail(ECC_E_ARG, "null count pointer");
    return cost_impl(ctx, scan_id, B, theta_dev, nullptr, params, out_cost_dev, out_pair_dev, out_count_dev,
                     workspace_dev, workspace_bytes, stream);
}

ecc_status ecc_cost_pinv(ecc_ctx *ctx, int32_t scan_id, int32_t B, const double *theta_dev, const double *pinv_dev,
                         const ecc_eval_params *params, double *out_cost_dev, float *out_pair_dev,
                         void *workspace_dev, uint64_t workspace_bytes, void *stream) {
    if (!pinv_dev) return fail(ECC_E_ARG, "null pseudo-inverse pointer");
    return cost_impl(ctx, scan_id, B, theta_dev, pinv_dev, params, out_cost_dev, out_pair_dev, nullptr,
                     workspace_dev, workspace_bytes, stream);
}

static ecc_status cost_impl(ecc_ctx *ctx, int32_t scan_id, int32_t B, const double *theta_dev,
                            const double *pinv_dev, const ecc_eval_params *params, double *out_cost_dev,
                            float *out_pair_dev, int32_t *out_count_dev, void *workspace_dev,
                            uint64_t workspace_bytes, void *stream) {
    if (!ctx) return fail(ECC_E_ARG, "null context");
    // the lock spans the (asynchronous) launches so that a concurrent
    // ecc_scan_free cannot release the scan between check and launch
    std::lock_guard<std::mutex> lk(ctx->mu);
    Scan *s = nullptr;
    ecc_status st;
    if ((st = check_eval(ctx, scan_id, B, params, &s))) return st;
    if (!theta_dev || !out_cost_dev || !workspace_dev) return fail(ECC_E_ARG, "null device pointer");
    const Workspace w = workspace_layout(s, B, false);
    if (workspace_bytes < w.total)
        return fail(ECC_E_ARG, "workspace of %llu bytes is smaller than the %llu needed",
                    (unsigned long long)workspace_bytes, (unsigned long long)w.total);
    DeviceGuard g(ctx->device);
    hipStream_t hs = (hipStream_t)stream;
    char *ws = (char *)workspace_dev;
    ViewGeom *vt = (ViewGeom *)(ws + w.vt_off);
    double *partials = (double *)(ws + w.part_off);
    const EvalConsts ec = make_consts(s, B, params);
    const int n_tiles = n_work_tiles(ec.n_views, B);
    void *table = ws + w.table_off;
    HIP_TRY(launch_view_setup(s->P_dev, s->intr_dev, theta_dev, B, s->n_views, vt, nullptr, hs));
    HIP_TRY(launch_pair_setup(s->scale_dev, vt, ec, table, hs, pinv_dev));
    HIP_TRY(launch_ecc_fwd(s->sino_dev, table, ec, s->layout.dtype, out_pair_dev, out_count_dev, partials, n_tiles,
                           hs));
    HIP_TRY(launch_reduce_cost(partials, n_tiles, B, out_cost_dev, hs));
    return ok();
}

ecc_status ecc_cost_noalloc(ecc_ctx *ctx, int32_t scan_id, int32_t B, const double *theta_dev,
                            const ecc_eval_params *params, double *out_cost_dev, float *out_pair_dev, void *stream) {
    if (!ctx) return fail(ECC_E_ARG, "null context");
    uint64_t need = 0;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        Scan *s = find_scan(ctx, scan_id);
        if (!s) return fail(ECC_E_NOSCAN, "unknown scan id %d", scan_id);
        if (B < 1 || B > 65536) return fail(ECC_E_ARG, "B = %d out of range [1, 65536]", B);
        need = workspace_layout(s, B, false).total;
    }
    if (need > kNoAllocScratchBytes)
        return fail(ECC_E_ARG,
                    "ecc_cost_noalloc: %d hypotheses of this scan need %llu bytes of scratch, more than the %llu "
                    "bytes the static scratch holds (use ecc_cost with a caller workspace)",
                    B, (unsigned long long)need, (unsigned long long)kNoAllocScratchBytes);
    void *ptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        ptr = g_scratch_ptr[ctx->device];
    }
    if (!ptr) return fail(ECC_E_STATE, "no-alloc scratch of device %d was not resolved", ctx->device);
    // the scan may change between the size check and the evaluation only by
    // ecc_scan_free, which cost_impl reports as ECC_E_NOSCAN; it checks the
    // size again against the scratch it is given
    return cost_impl(ctx, scan_id, B, theta_dev, nullptr, params, out_cost_dev, out_pair_dev, nullptr, ptr,
                     kNoAllocScratchBytes, stream);
}

ecc_status ecc_cost_grad(ecc_ctx *ctx, int32_t scan_id, int32_t B, const double *theta_dev,
                         const ecc_eval_params *params, double *out_cost_dev, float *grad_dev,
                         float *out_pair_grad_dev, void *workspace_dev, uint64_t workspace_bytes, void *stream) {
    if (!ctx) return fail(ECC_E_ARG, "null context");
    std::lock_guard<std::mutex> lk(ctx->mu);
    Scan *s = nullptr;
    ecc_status st;
    if ((st = check_eval(ctx, scan_id, B, params, &s))) return st;
    if (!theta_dev || !out_cost_dev || !grad_dev || !workspace_dev) return fail(ECC_E_ARG, "null device pointer");
    const Workspace w = workspace_layout(s, B, true);
    if (workspace_bytes < w.total)
        return fail(ECC_E_ARG, "workspace of %llu bytes is smaller than the %llu needed",
                    (unsigned long long)workspace_bytes, (unsigned long long)w.total);
    DeviceGuard g(ctx->device);
    hipStream_t hs = (hipStream_t)stream;
    char *ws = (char *)workspace_dev;
    ViewGeom *vt = (ViewGeom *)(ws + w.vt_off);
    ViewGeomGrad *vg = (ViewGeomGrad *)(ws + w.vg_off);
    double *partials = (double *)(ws + w.part_off);
    float *pgrad = out_pair_grad_dev ? out_pair_grad_dev : (float *)(ws + w.pgrad_off);
    const EvalConsts ec = make_consts(s, B, params);
    const int n_tiles = n_work_tiles(ec.n_views, B);
    void *table = ws + w.table_off;
    HIP_TRY(launch_view_setup(s->P_dev, s->intr_dev, theta_dev, B, s->n_views, vt, vg, hs));
    HIP_TRY(launch_pair_setup(s->scale_dev, vt, ec, table, hs));
    float *sens = (float *)(ws + w.sens_off);
    HIP_TRY(launch_ecc_adj(s->sino_dev, table, vt, vg, ec, s->layout.dtype, sens, pgrad, partials, n_tiles, hs));
    HIP_TRY(launch_reduce_cost(partials, n_tiles, B, out_cost_dev, hs));
    HIP_TRY(launch_reduce_grad(pgrad, B, s->n_views, grad_dev, hs));
    return ok();
}

}  // extern "C"
