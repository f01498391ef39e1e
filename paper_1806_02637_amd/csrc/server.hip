// Served form: continuous batching of evaluation requests over resident
// scans.  One worker thread owns the scheduling:
//   * requests queue in arrival order (submit copies theta, never blocks);
//   * the head of the queue is admitted as soon as a stream slot is free and
//     its device bytes fit in the server's arena (first fit, coalescing free
//     list) -- the HBM-budget admission; admitted requests run concurrently
//     on their slots' streams while later ones keep arriving;
//   * completions are detected with per-request events; results are copied
//     out of the pinned staging arena, the request's arena blocks and slot
//     are released, and waiting clients are woken.
// The per-request work is exactly ecc_cost / ecc_cost_grad on the slot's
// stream with the request's own workspace, so results do not depend on
// which other requests share the device.  The scheduling itself (arena,
// states, admission and completion order) is server_core.hpp; this file is
// its HIP device side and the C entry points.
#include <hip/hip_runtime.h>

#include <string.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ecc.h"
#include "ecc_internal.hpp"
#include "server_core.hpp"

using ecc_serve::align256;
using ecc_serve::Core;
using ecc_serve::Layout;
using ecc_serve::Request;

namespace {

// The device side of the served form: per-slot streams, a device arena for
// the requests' buffers and workspaces, a pinned host arena for staging, and
// one completion event per request.
class HipDevice final : public ecc_serve::Device {
  public:
    ecc_ctx *ctx = nullptr;
    int device = 0;
    std::vector<hipStream_t> streams;
    char *dev_arena = nullptr;
    char *host_arena = nullptr;

    ecc_status prepare(Request &r, std::string *err) override {
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(device);
        hipEvent_t ev = nullptr;
        const hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        (void)hipSetDevice(prev);
        if (e != hipSuccess) {
            *err = std::string("hipEventCreate failed: ") + hipGetErrorString(e);
            return ECC_E_HIP;
        }
        r.token = ev;
        return ECC_OK;
    }

    void discard(Request &r) override {
        if (r.token) (void)hipEventDestroy((hipEvent_t)r.token);
        r.token = nullptr;
    }

    ecc_status workspace_bytes(const Request &r, uint64_t *bytes, std::string *err) override {
        const ecc_status st = ecc_workspace_bytes(ctx, r.scan, r.B, r.with_grad, bytes);
        if (st != ECC_OK) *err = ecc_last_error();
        return st;
    }

    ecc_status launch(Request &r, const Layout &L, std::string *err) override {
        hipStream_t st = streams[r.slot];
        char *dev = dev_arena + r.dev_off;
        char *host = host_arena + r.host_off;
        const uint64_t th_bytes = sizeof(double) * 6ull * r.B * r.n_views;
        memcpy(host + L.theta, r.theta.data(), th_bytes);
        hipError_t e = hipMemcpyAsync(dev + L.theta, host + L.theta, th_bytes, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(st, e, err);
        ecc_status rc;
        if (r.with_grad)
            rc = ecc_cost_grad(ctx, r.scan, r.B, (const double *)(dev + L.theta), &r.prm, (double *)(dev + L.cost),
                               (float *)(dev + L.grad), nullptr, dev + L.ws, r.ws_bytes, st);
        else
            rc = ecc_cost(ctx, r.scan, r.B, (const double *)(dev + L.theta), &r.prm, (double *)(dev + L.cost),
                          nullptr, dev + L.ws, r.ws_bytes, st);
        if (rc != ECC_OK) {
            // nothing but the theta copy reached the stream: let it finish
            // before the arena blocks are handed out again
            *err = ecc_last_error();
            (void)hipStreamSynchronize(st);
            return rc;
        }
        e = hipMemcpyAsync(host + L.cost, dev + L.cost, sizeof(double) * r.B, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && r.with_grad)
            e = hipMemcpyAsync(host + L.grad, dev + L.grad, sizeof(float) * 6ull * r.B * r.n_views,
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipEventRecord((hipEvent_t)r.token, st);
        if (e != hipSuccess) return hip_fail(st, e, err);
        return ECC_OK;
    }

    ecc_status poll(Request &r, int *finished, std::string *err) override {
        const hipError_t q = hipEventQuery((hipEvent_t)r.token);
        if (q == hipErrorNotReady) {
            *finished = 0;
            return ECC_OK;
        }
        if (q != hipSuccess) {
            *err = hipGetErrorString(q);
            return ECC_E_HIP;
        }
        *finished = 1;
        return ECC_OK;
    }

    void collect(Request &r, const Layout &L) override {
        const char *host = host_arena + r.host_off;
        memcpy(r.cost.data(), host + L.cost, sizeof(double) * r.B);
        if (r.with_grad) memcpy(r.grad.data(), host + L.grad, sizeof(float) * 6ull * r.B * r.n_views);
    }

  private:
    static ecc_status hip_fail(hipStream_t st, hipError_t e, std::string *err) {
        (void)hipStreamSynchronize(st);
        *err = hipGetErrorString(e);
        return ECC_E_HIP;
    }
};

ecc_status set_err(ecc_status code, const char *msg) { return ecc::set_error(code, "%s", msg); }

}  // namespace

struct ecc_server {
    HipDevice dev;
    std::unique_ptr<Core> core;
    std::thread worker;
};

extern "C" {

ecc_status ecc_server_create(ecc_ctx *ctx, ecc_server **out, int32_t n_slots, uint64_t arena_bytes) {
    if (!ctx || !out) return set_err(ECC_E_ARG, "null argument");
    *out = nullptr;
    if (n_slots < 1 || n_slots > 16) return ecc::set_error(ECC_E_ARG, "n_slots = %d out of range [1, 16]", n_slots);
    if (arena_bytes < 4096) return set_err(ECC_E_ARG, "arena too small");
    auto s = std::make_unique<ecc_server>();
    HipDevice &d = s->dev;
    d.ctx = ctx;
    d.device = ecc::ctx_device(ctx);
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(d.device);
    // staging for theta, costs and gradients: 1/16 of the device arena, at least 64 MiB
    const uint64_t host_bytes = align256(std::max<uint64_t>(arena_bytes / 16, 64ull << 20));
    hipError_t e = hipMalloc((void **)&d.dev_arena, arena_bytes);
    if (e == hipSuccess) e = hipHostMalloc((void **)&d.host_arena, host_bytes, hipHostMallocDefault);
    for (int i = 0; e == hipSuccess && i < n_slots; ++i) {
        hipStream_t st;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) d.streams.push_back(st);
    }
    if (e != hipSuccess) {
        for (auto st : d.streams) (void)hipStreamDestroy(st);
        if (d.dev_arena) (void)hipFree(d.dev_arena);
        if (d.host_arena) (void)hipHostFree(d.host_arena);
        (void)hipSetDevice(prev);
        return ecc::set_error(ECC_E_HIP, "server allocation failed: %s", hipGetErrorString(e));
    }
    (void)hipSetDevice(prev);
    s->core = std::make_unique<Core>(&s->dev, n_slots, arena_bytes, host_bytes);
    ecc_server *raw = s.release();
    const int device = raw->dev.device;
    Core *core = raw->core.get();
    raw->worker = std::thread([core, device] {
        (void)hipSetDevice(device);
        core->run();
    });
    *out = raw;
    return ECC_OK;
}

ecc_status ecc_server_submit(ecc_server *s, int32_t scan_id, int32_t B, const double *theta_host,
                             const ecc_eval_params *params, int32_t with_grad, int64_t *request_id) {
    if (!s || !theta_host || !params || !request_id) return set_err(ECC_E_ARG, "null argument");
    int32_t n_views = 0;
    ecc_status st = ecc_scan_info(s->dev.ctx, scan_id, &n_views, nullptr, nullptr, nullptr, nullptr);
    if (st != ECC_OK) return st;
    if (B < 1 || B > 65536) return ecc::set_error(ECC_E_ARG, "B = %d out of range", B);
    if (params->K < 1 || params->K > 4096) return ecc::set_error(ECC_E_ARG, "K = %d out of range", params->K);
    auto r = std::make_unique<Request>();
    r->scan = scan_id;
    r->B = B;
    r->n_views = n_views;
    r->with_grad = with_grad != 0;
    r->prm = *params;
    r->work = (double)B * ((double)n_views * (n_views - 1) / 2) * params->K * (with_grad ? 2.0 : 1.0);
    r->theta.assign(theta_host, theta_host + 6ull * B * n_views);
    r->cost.assign(B, 0.0);
    if (r->with_grad) r->grad.assign(6ull * B * n_views, 0.0f);
    std::string err;
    st = s->core->submit(std::move(r), request_id, &err);
    if (st != ECC_OK) return ecc::set_error(st, "%s", err.c_str());
    return ECC_OK;
}

ecc_status ecc_server_poll(ecc_server *s, int64_t request_id, int32_t *done) {
    if (!s || !done) return set_err(ECC_E_ARG, "null argument");
    std::string err;
    const ecc_status st = s->core->poll(request_id, done, &err);
    if (st != ECC_OK) return ecc::set_error(st, "%s", err.c_str());
    return ECC_OK;
}

ecc_status ecc_server_wait(ecc_server *s, int64_t request_id, double *cost_host, float *grad_host,
                           ecc_request_stats *stats) {
    if (!s) return set_err(ECC_E_ARG, "null server");
    std::unique_ptr<Request> r;
    std::string err;
    const ecc_status st = s->core->wait(request_id, &r, &err);
    if (st != ECC_OK) return ecc::set_error(st, "%s", err.c_str());
    s->dev.discard(*r);
    if (stats) {
        auto ms = [](ecc_serve::clk::time_point a, ecc_serve::clk::time_point b) {
            return std::chrono::duration<double, std::milli>(b - a).count();
        };
        const bool admitted = r->t_admit.time_since_epoch().count() != 0;
        stats->queue_ms = admitted ? ms(r->t_submit, r->t_admit) : ms(r->t_submit, r->t_done);
        stats->run_ms = admitted ? ms(r->t_admit, r->t_done) : 0.0;
        stats->total_ms = ms(r->t_submit, r->t_done);
        stats->slot = r->ran_slot;
        stats->status = r->status;
    }
    if (r->status != ECC_OK) return ecc::set_error(r->status, "request %lld failed: %s", (long long)request_id,
                                                   r->error.c_str());
    if (cost_host) memcpy(cost_host, r->cost.data(), sizeof(double) * r->B);
    if (grad_host && r->with_grad) memcpy(grad_host, r->grad.data(), sizeof(float) * r->grad.size());
    return ECC_OK;
}

ecc_status ecc_server_request_bytes(ecc_server *s, int32_t scan_id, int32_t B, int32_t with_grad, uint64_t *bytes) {
    if (!s || !bytes) return set_err(ECC_E_ARG, "null argument");
    int32_t n_views = 0;
    ecc_status st = ecc_scan_info(s->dev.ctx, scan_id, &n_views, nullptr, nullptr, nullptr, nullptr);
    if (st != ECC_OK) return st;
    uint64_t ws = 0;
    if ((st = ecc_workspace_bytes(s->dev.ctx, scan_id, B, with_grad, &ws)) != ECC_OK) return st;
    *bytes = align256(ecc_serve::request_layout(B, n_views, with_grad, ws).dev_total);
    return ECC_OK;
}

ecc_status ecc_server_set_work_cap(ecc_server *s, double work_cap) {
    if (!s) return set_err(ECC_E_ARG, "null server");
    if (!(work_cap >= 0.0) || !std::isfinite(work_cap)) return set_err(ECC_E_ARG, "work cap must be finite and >= 0");
    s->core->set_work_cap(work_cap);
    return ECC_OK;
}

ecc_status ecc_server_destroy(ecc_server *s) {
    if (!s) return set_err(ECC_E_ARG, "null server");
    s->core->request_stop();
    if (s->worker.joinable()) s->worker.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->dev.device);
    s->core.reset();  // discards the completion events of uncollected requests
    for (auto st : s->dev.streams) (void)hipStreamDestroy(st);
    (void)hipFree(s->dev.dev_arena);
    (void)hipHostFree(s->dev.host_arena);
    (void)hipSetDevice(prev);
    delete s;
    return ECC_OK;
}

}  // extern "C"
