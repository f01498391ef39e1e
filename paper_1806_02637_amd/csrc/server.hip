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
// which other requests share the device.
#include <hip/hip_runtime.h>

#include <string.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ecc.h"
#include "ecc_internal.hpp"

namespace {

using clk = std::chrono::steady_clock;

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// First-fit allocator over [0, size) with coalescing.
class Arena {
  public:
    void init(uint64_t size) {
        free_.clear();
        free_[0] = size;
        size_ = size;
    }
    bool alloc(uint64_t bytes, uint64_t *off) {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, start = it->first;
                free_.erase(it);
                if (rest) free_[start + bytes] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = align256(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t size() const { return size_; }

  private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t size_ = 0;
};

enum ReqState { PENDING, RUNNING, DONE };

struct Request {
    int64_t id = 0;
    int32_t scan = 0, B = 0, n_views = 0, with_grad = 0;
    ecc_eval_params prm{};
    std::vector<double> theta;
    std::vector<double> cost;
    std::vector<float> grad;
    ReqState state = PENDING;
    ecc_status status = ECC_OK;
    std::string error;
    clk::time_point t_submit, t_admit, t_done;
    int slot = -1, ran_slot = -1;
    uint64_t dev_off = 0, dev_bytes = 0, host_off = 0, host_bytes = 0;
    uint64_t ws_bytes = 0;
    double work = 0.0;  // plane-pair evaluations, a gradient counted twice
    hipEvent_t done_ev = nullptr;
};

}  // namespace

struct ecc_server {
    ecc_ctx *ctx = nullptr;
    int device = 0;
    std::vector<hipStream_t> streams;
    std::vector<bool> slot_busy;
    char *dev_arena = nullptr;
    char *host_arena = nullptr;
    Arena dev_alloc, host_alloc;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> pending;
    std::vector<Request *> running;
    double work_cap = 0.0;       // 0: none
    double work_in_flight = 0.0;
    std::map<int64_t, std::unique_ptr<Request>> requests;
    int64_t next_id = 1;
    bool stop = false;
    std::thread worker;
};

namespace {

struct Layout {
    uint64_t theta, cost, grad, ws, dev_total, host_total;
};

Layout request_layout(int B, int n_views, int with_grad, uint64_t ws_bytes) {
    Layout L{};
    const uint64_t th = sizeof(double) * 6ull * B * n_views;
    const uint64_t co = sizeof(double) * (uint64_t)B;
    const uint64_t gr = with_grad ? sizeof(float) * 6ull * B * n_views : 0;
    L.theta = 0;
    L.cost = align256(th);
    L.grad = L.cost + align256(co);
    L.ws = L.grad + align256(gr);
    L.dev_total = L.ws + align256(ws_bytes);
    L.host_total = L.ws;  // staging holds theta, cost and grad
    return L;
}

void finish(ecc_server *s, Request *r, ecc_status st, const char *msg) {
    r->status = st;
    if (msg) r->error = msg;
    r->state = DONE;
    r->t_done = clk::now();
}

// Launches an admitted request on its slot (worker thread, lock held).
void launch(ecc_server *s, Request *r, const Layout &L) {
    hipStream_t st = s->streams[r->slot];
    char *dev = s->dev_arena + r->dev_off;
    char *host = s->host_arena + r->host_off;
    const uint64_t th_bytes = sizeof(double) * 6ull * r->B * r->n_views;
    memcpy(host + L.theta, r->theta.data(), th_bytes);
    hipError_t e = hipMemcpyAsync(dev + L.theta, host + L.theta, th_bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        finish(s, r, ECC_E_HIP, hipGetErrorString(e));
        return;
    }
    ecc_status rc;
    if (r->with_grad)
        rc = ecc_cost_grad(s->ctx, r->scan, r->B, (const double *)(dev + L.theta), &r->prm, (double *)(dev + L.cost),
                           (float *)(dev + L.grad), nullptr, dev + L.ws, r->ws_bytes, st);
    else
        rc = ecc_cost(s->ctx, r->scan, r->B, (const double *)(dev + L.theta), &r->prm, (double *)(dev + L.cost),
                      nullptr, dev + L.ws, r->ws_bytes, st);
    if (rc != ECC_OK) {
        // the request never reached the device past the theta copy
        (void)hipStreamSynchronize(st);
        finish(s, r, rc, ecc_last_error());
        return;
    }
    e = hipMemcpyAsync(host + L.cost, dev + L.cost, sizeof(double) * r->B, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && r->with_grad)
        e = hipMemcpyAsync(host + L.grad, dev + L.grad, sizeof(float) * 6ull * r->B * r->n_views,
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(r->done_ev, st);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(st);
        finish(s, r, ECC_E_HIP, hipGetErrorString(e));
        return;
    }
    r->state = RUNNING;
}

void release(ecc_server *s, Request *r) {
    if (r->slot >= 0) {
        s->work_in_flight -= r->work;
        if (s->work_in_flight < 0.5) s->work_in_flight = 0.0;
        s->slot_busy[r->slot] = false;
        s->dev_alloc.release(r->dev_off, r->dev_bytes);
        s->host_alloc.release(r->host_off, r->host_bytes);
        r->slot = -1;
    }
}

void worker_loop(ecc_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        bool progressed = false;
        // completions
        for (size_t i = 0; i < s->running.size();) {
            Request *r = s->running[i];
            const hipError_t q = hipEventQuery(r->done_ev);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            if (q == hipSuccess) {
                const Layout L = request_layout(r->B, r->n_views, r->with_grad, r->ws_bytes);
                const char *host = s->host_arena + r->host_off;
                memcpy(r->cost.data(), host + L.cost, sizeof(double) * r->B);
                if (r->with_grad) memcpy(r->grad.data(), host + L.grad, sizeof(float) * 6ull * r->B * r->n_views);
                finish(s, r, ECC_OK, nullptr);
            } else {
                finish(s, r, ECC_E_HIP, hipGetErrorString(q));
            }
            release(s, r);
            s->running.erase(s->running.begin() + i);
            progressed = true;
        }
        if (progressed) s->cv_done.notify_all();
        // admissions, in arrival order
        while (!s->pending.empty() && !s->stop) {
            Request *r = s->pending.front();
            int slot = -1;
            for (int i = 0; i < (int)s->slot_busy.size(); ++i)
                if (!s->slot_busy[i]) {
                    slot = i;
                    break;
                }
            if (slot < 0) break;
            // with a work cap, an admitted request must fit under it together
            // with the work in flight (an idle device always takes the head)
            if (s->work_cap > 0.0 && !s->running.empty() && s->work_in_flight + r->work > s->work_cap) break;
            uint64_t ws = 0;
            const ecc_status wsst = ecc_workspace_bytes(s->ctx, r->scan, r->B, r->with_grad, &ws);
            if (wsst != ECC_OK) {
                s->pending.pop_front();
                finish(s, r, wsst, ecc_last_error());
                s->cv_done.notify_all();
                continue;
            }
            r->ws_bytes = ws;
            const Layout L = request_layout(r->B, r->n_views, r->with_grad, ws);
            if (align256(L.dev_total) > s->dev_alloc.size() || align256(L.host_total) > s->host_alloc.size()) {
                s->pending.pop_front();
                finish(s, r, ECC_E_BUDGET, "request larger than the server's arena");
                s->cv_done.notify_all();
                continue;
            }
            uint64_t doff = 0, hoff = 0;
            if (!s->dev_alloc.alloc(L.dev_total, &doff)) break;  // wait for memory
            if (!s->host_alloc.alloc(L.host_total, &hoff)) {
                s->dev_alloc.release(doff, L.dev_total);
                break;
            }
            s->pending.pop_front();
            r->slot = slot;
            r->ran_slot = slot;
            s->slot_busy[slot] = true;
            r->dev_off = doff;
            r->dev_bytes = L.dev_total;
            r->host_off = hoff;
            r->host_bytes = L.host_total;
            r->t_admit = clk::now();
            s->work_in_flight += r->work;
            launch(s, r, L);
            if (r->state == RUNNING) {
                s->running.push_back(r);
            } else {
                release(s, r);
                s->cv_done.notify_all();
            }
        }
        if (s->stop && s->running.empty()) break;
        if (s->running.empty() && s->pending.empty()) {
            s->cv_work.wait(lk);
        } else if (!s->running.empty()) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        } else {
            // pending but blocked (no slot/arena) with nothing running cannot
            // happen; wait for a submit or stop anyway
            s->cv_work.wait_for(lk, std::chrono::milliseconds(1));
        }
    }
    // fail whatever is still queued
    for (Request *r : s->pending) finish(s, r, ECC_E_STATE, "server stopped before the request was admitted");
    s->pending.clear();
    s->cv_done.notify_all();
}

ecc_status set_err(ecc_status code, const char *msg) { return ecc::set_error(code, "%s", msg); }

}  // namespace

extern "C" {

ecc_status ecc_server_create(ecc_ctx *ctx, ecc_server **out, int32_t n_slots, uint64_t arena_bytes) {
    if (!ctx || !out) return set_err(ECC_E_ARG, "null argument");
    *out = nullptr;
    if (n_slots < 1 || n_slots > 16) return ecc::set_error(ECC_E_ARG, "n_slots = %d out of range [1, 16]", n_slots);
    if (arena_bytes < 4096) return set_err(ECC_E_ARG, "arena too small");
    auto s = std::make_unique<ecc_server>();
    s->ctx = ctx;
    s->device = ecc::ctx_device(ctx);
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    // staging for theta, costs and gradients: 1/16 of the device arena, at least 64 MiB
    const uint64_t host_bytes = align256(std::max<uint64_t>(arena_bytes / 16, 64ull << 20));
    hipError_t e = hipMalloc((void **)&s->dev_arena, arena_bytes);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->host_arena, host_bytes, hipHostMallocDefault);
    for (int i = 0; e == hipSuccess && i < n_slots; ++i) {
        hipStream_t st;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) s->streams.push_back(st);
    }
    if (e != hipSuccess) {
        for (auto st : s->streams) (void)hipStreamDestroy(st);
        if (s->dev_arena) (void)hipFree(s->dev_arena);
        if (s->host_arena) (void)hipHostFree(s->host_arena);
        (void)hipSetDevice(prev);
        return ecc::set_error(ECC_E_HIP, "server allocation failed: %s", hipGetErrorString(e));
    }
    (void)hipSetDevice(prev);
    s->slot_busy.assign(n_slots, false);
    s->dev_alloc.init(arena_bytes);
    s->host_alloc.init(host_bytes);
    ecc_server *raw = s.release();
    raw->worker = std::thread(worker_loop, raw);
    *out = raw;
    return ECC_OK;
}

ecc_status ecc_server_submit(ecc_server *s, int32_t scan_id, int32_t B, const double *theta_host,
                             const ecc_eval_params *params, int32_t with_grad, int64_t *request_id) {
    if (!s || !theta_host || !params || !request_id) return set_err(ECC_E_ARG, "null argument");
    int32_t n_views = 0;
    ecc_status st = ecc_scan_info(s->ctx, scan_id, &n_views, nullptr, nullptr, nullptr, nullptr);
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
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    hipError_t e = hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) return ecc::set_error(ECC_E_HIP, "hipEventCreate failed: %s", hipGetErrorString(e));
    r->t_submit = clk::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            (void)hipEventDestroy(r->done_ev);
            return set_err(ECC_E_STATE, "server is stopping");
        }
        r->id = s->next_id++;
        *request_id = r->id;
        s->pending.push_back(r.get());
        s->requests[r->id] = std::move(r);
    }
    s->cv_work.notify_one();
    return ECC_OK;
}

ecc_status ecc_server_poll(ecc_server *s, int64_t request_id, int32_t *done) {
    if (!s || !done) return set_err(ECC_E_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->requests.find(request_id);
    if (it == s->requests.end()) return ecc::set_error(ECC_E_ARG, "unknown request %lld", (long long)request_id);
    *done = it->second->state == DONE;
    return ECC_OK;
}

ecc_status ecc_server_wait(ecc_server *s, int64_t request_id, double *cost_host, float *grad_host,
                           ecc_request_stats *stats) {
    if (!s) return set_err(ECC_E_ARG, "null server");
    std::unique_ptr<Request> r;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->requests.find(request_id);
        if (it == s->requests.end()) return ecc::set_error(ECC_E_ARG, "unknown request %lld", (long long)request_id);
        Request *rp = it->second.get();
        s->cv_done.wait(lk, [&] { return rp->state == DONE; });
        r = std::move(it->second);
        s->requests.erase(it);
    }
    if (r->done_ev) (void)hipEventDestroy(r->done_ev);
    if (stats) {
        auto ms = [](clk::time_point a, clk::time_point b) {
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
    ecc_status st = ecc_scan_info(s->ctx, scan_id, &n_views, nullptr, nullptr, nullptr, nullptr);
    if (st != ECC_OK) return st;
    uint64_t ws = 0;
    if ((st = ecc_workspace_bytes(s->ctx, scan_id, B, with_grad, &ws)) != ECC_OK) return st;
    *bytes = align256(request_layout(B, n_views, with_grad, ws).dev_total);
    return ECC_OK;
}

ecc_status ecc_server_set_work_cap(ecc_server *s, double work_cap) {
    if (!s) return set_err(ECC_E_ARG, "null server");
    if (!(work_cap >= 0.0) || !std::isfinite(work_cap)) return set_err(ECC_E_ARG, "work cap must be finite and >= 0");
    std::lock_guard<std::mutex> lk(s->mu);
    s->work_cap = work_cap;
    s->cv_work.notify_all();
    return ECC_OK;
}

ecc_status ecc_server_destroy(ecc_server *s) {
    if (!s) return set_err(ECC_E_ARG, "null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    for (auto &kv : s->requests)
        if (kv.second->done_ev) (void)hipEventDestroy(kv.second->done_ev);
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    (void)hipFree(s->dev_arena);
    (void)hipHostFree(s->host_arena);
    (void)hipSetDevice(prev);
    delete s;
    return ECC_OK;
}

}  // extern "C"
