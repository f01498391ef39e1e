// Host-side scheduling of the served form, free of HIP so that it can be
// built and tested on the CPU (under address/undefined/thread sanitizers):
// the arena allocator behind admission by HBM footprint, the request record
// and its states, and the scheduling pass the worker thread repeats --
// completions first, then admissions in arrival order.  Everything that
// touches the device (creating a request's completion event, launching its
// evaluation on a stream slot, asking whether it finished, copying results
// out of the staging arena) sits behind the Device interface: server.hip
// implements it with HIP streams and events, the host tests with a
// simulated device.
#pragma once

#include <stdint.h>
#include <string.h>

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

namespace ecc_serve {

using clk = std::chrono::steady_clock;

inline uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// First-fit allocator over [0, size) with coalescing of neighbouring free
// blocks; every block is a multiple of 256 bytes.
class Arena {
  public:
    void init(uint64_t size) {
        free_.clear();
        size_ = size & ~uint64_t(255);
        if (size_) free_[0] = size_;
    }
    bool alloc(uint64_t bytes, uint64_t *off) {
        bytes = align256(bytes);
        if (bytes == 0) bytes = 256;
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
        if (bytes == 0) bytes = 256;
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
    uint64_t free_bytes() const {
        uint64_t s = 0;
        for (auto &kv : free_) s += kv.second;
        return s;
    }
    size_t free_blocks() const { return free_.size(); }
    // the free list is sorted, inside [0, size), non-overlapping and fully
    // coalesced (no two free blocks touch)
    bool consistent() const {
        uint64_t end = 0;
        bool first = true;
        for (auto &kv : free_) {
            if (kv.second == 0 || kv.first % 256 || kv.second % 256) return false;
            if (!first && kv.first <= end) return false;  // overlap or touching (not coalesced)
            end = kv.first + kv.second;
            if (end > size_) return false;
            first = false;
        }
        return true;
    }

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
    clk::time_point t_submit{}, t_admit{}, t_done{};
    int slot = -1, ran_slot = -1;
    uint64_t dev_off = 0, dev_bytes = 0, host_off = 0, host_bytes = 0;
    uint64_t ws_bytes = 0;
    double work = 0.0;        // plane-pair evaluations, a gradient counted twice
    void *token = nullptr;    // the device's completion handle
};

// Where a request's buffers sit in its arena blocks.
struct Layout {
    uint64_t theta, cost, grad, ws, dev_total, host_total;
};

inline Layout request_layout(int B, int n_views, int with_grad, uint64_t ws_bytes) {
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

class Device {
  public:
    virtual ~Device() = default;
    // creates the request's completion token (at submit)
    virtual ecc_status prepare(Request &r, std::string *err) = 0;
    // destroys it (after the request was collected, or at shutdown)
    virtual void discard(Request &r) = 0;
    // workspace bytes the evaluation needs
    virtual ecc_status workspace_bytes(const Request &r, uint64_t *bytes, std::string *err) = 0;
    // queues theta's upload, the evaluation and the result copies on slot
    // r.slot; ECC_OK means the request now runs on the device
    virtual ecc_status launch(Request &r, const Layout &L, std::string *err) = 0;
    // 0: still running; 1: finished, results staged; otherwise the failure
    virtual ecc_status poll(Request &r, int *finished, std::string *err) = 0;
    // copies the staged results into r.cost / r.grad
    virtual void collect(Request &r, const Layout &L) = 0;
};

// Scheduling state shared by the worker thread and the client calls; every
// member is guarded by `mu`.
class Core {
  public:
    Core(Device *dev, int n_slots, uint64_t dev_arena_bytes, uint64_t host_arena_bytes) : dev_(dev) {
        slot_busy_.assign(n_slots, false);
        dev_alloc_.init(dev_arena_bytes);
        host_alloc_.init(host_arena_bytes);
    }
    ~Core() {
        for (auto &kv : requests_) dev_->discard(*kv.second);
    }

    // Queues a request (theta, B, params filled in by the caller); never
    // blocks on the device.
    ecc_status submit(std::unique_ptr<Request> r, int64_t *id, std::string *err) {
        ecc_status st = dev_->prepare(*r, err);
        if (st != ECC_OK) return st;
        r->t_submit = clk::now();
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (stop_) {
                dev_->discard(*r);
                *err = "server is stopping";
                return ECC_E_STATE;
            }
            r->id = next_id_++;
            *id = r->id;
            pending_.push_back(r.get());
            requests_[r->id] = std::move(r);
        }
        cv_work_.notify_one();
        return ECC_OK;
    }

    ecc_status poll(int64_t id, int32_t *done, std::string *err) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = requests_.find(id);
        if (it == requests_.end()) {
            *err = "unknown request " + std::to_string(id);
            return ECC_E_ARG;
        }
        *done = it->second->state == DONE;
        return ECC_OK;
    }

    // Blocks until the request is done and hands it over (the core forgets
    // it).  Several callers may wait on one id: the first to wake takes the
    // request, the others find it gone and get ECC_E_ARG; no waiter touches
    // a request after another took it.
    ecc_status wait(int64_t id, std::unique_ptr<Request> *out, std::string *err) {
        std::unique_lock<std::mutex> lk(mu_);
        if (requests_.find(id) == requests_.end()) {
            *err = "unknown request " + std::to_string(id);
            return ECC_E_ARG;
        }
        cv_done_.wait(lk, [&] {
            auto it = requests_.find(id);
            return it == requests_.end() || it->second->state == DONE;
        });
        auto it = requests_.find(id);
        if (it == requests_.end()) {
            *err = "request " + std::to_string(id) + " was collected by another wait";
            return ECC_E_ARG;
        }
        *out = std::move(it->second);
        requests_.erase(it);
        lk.unlock();
        cv_done_.notify_all();  // other waiters on this id see it gone
        return ECC_OK;
    }

    void set_work_cap(double cap) {
        std::lock_guard<std::mutex> lk(mu_);
        work_cap_ = cap;
        cv_work_.notify_all();
    }

    // Stops admitting; the worker lets running requests finish, then fails
    // the queued ones.
    void request_stop() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_work_.notify_all();
    }

    // The worker thread's body: scheduling passes until stopped and drained.
    void run() {
        std::unique_lock<std::mutex> lk(mu_);
        while (true) {
            pass_locked();
            if (stop_ && running_.empty()) break;
            if (running_.empty() && pending_.empty()) {
                cv_work_.wait(lk);
            } else if (!running_.empty()) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            } else {
                // pending but blocked with nothing running cannot happen (an
                // idle device admits the head); wait for a submit or stop
                cv_work_.wait_for(lk, std::chrono::milliseconds(1));
            }
        }
        for (Request *r : pending_) finish(r, ECC_E_STATE, "server stopped before the request was admitted");
        pending_.clear();
        lk.unlock();
        cv_done_.notify_all();
    }

    // One scheduling pass (exposed for deterministic host tests).
    bool pass() {
        std::lock_guard<std::mutex> lk(mu_);
        return pass_locked();
    }

    // Snapshot accessors for tests.
    size_t n_pending() {
        std::lock_guard<std::mutex> lk(mu_);
        return pending_.size();
    }
    size_t n_running() {
        std::lock_guard<std::mutex> lk(mu_);
        return running_.size();
    }
    uint64_t dev_free_bytes() {
        std::lock_guard<std::mutex> lk(mu_);
        return dev_alloc_.free_bytes();
    }
    bool arenas_consistent() {
        std::lock_guard<std::mutex> lk(mu_);
        return dev_alloc_.consistent() && host_alloc_.consistent();
    }
    double work_in_flight() {
        std::lock_guard<std::mutex> lk(mu_);
        return work_in_flight_;
    }
    uint64_t dev_arena_size() const { return dev_alloc_.size(); }
    uint64_t host_arena_size() const { return host_alloc_.size(); }

  private:
    void finish(Request *r, ecc_status st, const std::string &msg) {
        r->status = st;
        if (!msg.empty()) r->error = msg;
        r->state = DONE;
        r->t_done = clk::now();
    }

    void release(Request *r) {
        if (r->slot >= 0) {
            work_in_flight_ -= r->work;
            if (work_in_flight_ < 0.5) work_in_flight_ = 0.0;
            slot_busy_[r->slot] = false;
            dev_alloc_.release(r->dev_off, r->dev_bytes);
            host_alloc_.release(r->host_off, r->host_bytes);
            r->slot = -1;
        }
    }

    bool pass_locked() {
        bool changed = false, done_any = false;
        // completions
        for (size_t i = 0; i < running_.size();) {
            Request *r = running_[i];
            int finished = 0;
            std::string err;
            const ecc_status q = dev_->poll(*r, &finished, &err);
            if (q == ECC_OK && !finished) {
                ++i;
                continue;
            }
            if (q == ECC_OK) {
                dev_->collect(*r, request_layout(r->B, r->n_views, r->with_grad, r->ws_bytes));
                finish(r, ECC_OK, "");
            } else {
                finish(r, q, err);
            }
            release(r);
            running_.erase(running_.begin() + i);
            done_any = changed = true;
        }
        // admissions, in arrival order
        while (!pending_.empty() && !stop_) {
            Request *r = pending_.front();
            int slot = -1;
            for (int i = 0; i < (int)slot_busy_.size(); ++i)
                if (!slot_busy_[i]) {
                    slot = i;
                    break;
                }
            if (slot < 0) break;
            // with a work cap, an admitted request must fit under it together
            // with the work in flight (an idle device always takes the head)
            if (work_cap_ > 0.0 && !running_.empty() && work_in_flight_ + r->work > work_cap_) break;
            uint64_t ws = 0;
            std::string err;
            const ecc_status wsst = dev_->workspace_bytes(*r, &ws, &err);
            if (wsst != ECC_OK) {
                pending_.pop_front();
                finish(r, wsst, err);
                done_any = changed = true;
                continue;
            }
            r->ws_bytes = ws;
            const Layout L = request_layout(r->B, r->n_views, r->with_grad, ws);
            if (align256(L.dev_total) > dev_alloc_.size() || align256(L.host_total) > host_alloc_.size()) {
                pending_.pop_front();
                finish(r, ECC_E_BUDGET, "request larger than the server's arena");
                done_any = changed = true;
                continue;
            }
            uint64_t doff = 0, hoff = 0;
            if (!dev_alloc_.alloc(L.dev_total, &doff)) break;  // wait for memory
            if (!host_alloc_.alloc(L.host_total, &hoff)) {
                dev_alloc_.release(doff, L.dev_total);
                break;
            }
            pending_.pop_front();
            r->slot = slot;
            r->ran_slot = slot;
            slot_busy_[slot] = true;
            r->dev_off = doff;
            r->dev_bytes = L.dev_total;
            r->host_off = hoff;
            r->host_bytes = L.host_total;
            r->t_admit = clk::now();
            work_in_flight_ += r->work;
            changed = true;
            const ecc_status st = dev_->launch(*r, L, &err);
            if (st == ECC_OK) {
                r->state = RUNNING;
                running_.push_back(r);
            } else {
                finish(r, st, err);
                release(r);
                done_any = true;
            }
        }
        if (done_any) cv_done_.notify_all();
        return changed;
    }

    Device *dev_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::vector<bool> slot_busy_;
    Arena dev_alloc_, host_alloc_;
    std::deque<Request *> pending_;
    std::vector<Request *> running_;
    double work_cap_ = 0.0, work_in_flight_ = 0.0;
    std::map<int64_t, std::unique_ptr<Request>> requests_;
    int64_t next_id_ = 1;
    bool stop_ = false;
};

}  // namespace ecc_serve
