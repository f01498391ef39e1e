// Host tests of the served form's scheduling core (server_core.hpp) with a
// simulated device: arena allocation and coalescing, first-in first-out
// admission by free slot and arena space, the work cap, failures at launch
// and on the device, stopping with queued requests, several waiters on one
// request, and a threaded run with many submitting clients.  Built with
// address / undefined-behaviour or thread sanitizers by test_server_core.py.
#include <stdio.h>
#include <stdlib.h>

#include <atomic>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "../paper_1806_02637_amd/csrc/server_core.hpp"

using namespace ecc_serve;

static int g_failures = 0;
#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            fprintf(stderr, "%s:%d: CHECK failed: %s\n", __FILE__, __LINE__, #cond); \
            ++g_failures;                                                        \
        }                                                                        \
    } while (0)

// Simulated device: a request "runs" until the test marks it finished (or,
// with auto_ms > 0, until that much wall time has passed since launch); its
// result is a fixed function of theta, so a test can check what it gets.
class FakeDevice final : public Device {
  public:
    std::mutex mu;
    std::set<int64_t> finished, fail_launch, fail_device;
    std::map<int64_t, clk::time_point> launched_at;
    std::atomic<int> prepared{0}, discarded{0}, launches{0};
    int auto_ms = 0;
    uint64_t ws_per_hyp = 1000;

    static double result_of(const Request &r, int b) {
        double s = 0.0;
        for (int i = 0; i < 6 * r.n_views; ++i) s += r.theta[(size_t)b * 6 * r.n_views + i] * (i + 1);
        return s;
    }

    ecc_status prepare(Request &r, std::string *) override {
        r.token = new int(1);
        ++prepared;
        return ECC_OK;
    }
    void discard(Request &r) override {
        if (r.token) {
            delete (int *)r.token;
            r.token = nullptr;
            ++discarded;
        }
    }
    ecc_status workspace_bytes(const Request &r, uint64_t *bytes, std::string *err) override {
        if (r.scan < 0) {
            *err = "unknown scan";
            return ECC_E_NOSCAN;
        }
        *bytes = ws_per_hyp * (uint64_t)r.B;
        return ECC_OK;
    }
    ecc_status launch(Request &r, const Layout &, std::string *err) override {
        std::lock_guard<std::mutex> lk(mu);
        ++launches;
        if (fail_launch.count(r.id)) {
            *err = "launch refused";
            return ECC_E_ARG;
        }
        launched_at[r.id] = clk::now();
        return ECC_OK;
    }
    ecc_status poll(Request &r, int *fin, std::string *err) override {
        std::lock_guard<std::mutex> lk(mu);
        if (fail_device.count(r.id)) {
            *err = "device fault";
            return ECC_E_HIP;
        }
        bool done = finished.count(r.id) > 0;
        if (auto_ms > 0 && clk::now() - launched_at[r.id] >= std::chrono::milliseconds(auto_ms)) done = true;
        *fin = done;
        return ECC_OK;
    }
    void collect(Request &r, const Layout &) override {
        for (int b = 0; b < r.B; ++b) r.cost[b] = result_of(r, b);
    }
    void finish(int64_t id) {
        std::lock_guard<std::mutex> lk(mu);
        finished.insert(id);
    }
};

static std::unique_ptr<Request> make_request(int B, int n_views, int scan = 0, double seed = 1.0, int K = 64) {
    auto r = std::make_unique<Request>();
    r->scan = scan;
    r->B = B;
    r->n_views = n_views;
    r->prm.K = K;
    r->work = (double)B * n_views * (n_views - 1) / 2 * K;
    r->theta.resize(6ull * B * n_views);
    for (size_t i = 0; i < r->theta.size(); ++i) r->theta[i] = seed + 0.001 * (double)i;
    r->cost.assign(B, 0.0);
    return r;
}

static uint64_t dev_bytes_of(int B, int n_views, uint64_t ws_per_hyp) {
    return align256(request_layout(B, n_views, 0, ws_per_hyp * B).dev_total);
}

static void test_arena() {
    Arena a;
    a.init(1 << 20);
    CHECK(a.consistent() && a.free_bytes() == (1u << 20) && a.free_blocks() == 1);
    uint64_t o1, o2, o3, o4;
    CHECK(a.alloc(1000, &o1) && o1 == 0);
    CHECK(a.alloc(300, &o2) && o2 == 1024);
    CHECK(a.alloc(256, &o3) && o3 == 1536);
    CHECK(a.free_bytes() == (1u << 20) - 1792);
    a.release(o2, 300);  // a hole between o1 and o3
    CHECK(a.consistent() && a.free_blocks() == 2);
    CHECK(a.alloc(200, &o4) && o4 == 1024);  // first fit reuses the hole
    a.release(o4, 200);
    a.release(o1, 1000);  // coalesces with the hole
    CHECK(a.consistent() && a.free_blocks() == 2);
    a.release(o3, 256);  // everything free again: one block
    CHECK(a.consistent() && a.free_blocks() == 1 && a.free_bytes() == (1u << 20));
    uint64_t big;
    CHECK(!a.alloc((1u << 20) + 1, &big));
    // random allocate / release: invariants hold, nothing leaks
    std::mt19937_64 rng(7);
    std::vector<std::pair<uint64_t, uint64_t>> live;
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || (rng() % 3 != 0 && live.size() < 200)) {
            const uint64_t n = 1 + rng() % 20000;
            uint64_t off;
            if (a.alloc(n, &off)) {
                for (auto &b : live)  // no overlap with a live block
                    CHECK(off + align256(n) <= b.first || b.first + align256(b.second) <= off);
                live.push_back({off, n});
            }
        } else {
            const size_t i = rng() % live.size();
            a.release(live[i].first, live[i].second);
            live.erase(live.begin() + i);
        }
        if (it % 997 == 0) CHECK(a.consistent());
    }
    for (auto &b : live) a.release(b.first, b.second);
    CHECK(a.consistent() && a.free_blocks() == 1 && a.free_bytes() == (1u << 20));
}

static void test_fifo_admission_by_slot() {
    FakeDevice dev;
    Core core(&dev, 2, 64 << 20, 64 << 20);
    int64_t id[3];
    std::string err;
    for (int i = 0; i < 3; ++i) CHECK(core.submit(make_request(2, 10, 0, i), &id[i], &err) == ECC_OK);
    core.pass();
    CHECK(core.n_running() == 2 && core.n_pending() == 1);
    int32_t done = -1;
    CHECK(core.poll(id[0], &done, &err) == ECC_OK && done == 0);
    dev.finish(id[1]);  // the second finishes first: its slot goes to the third
    core.pass();
    CHECK(core.n_running() == 2 && core.n_pending() == 0);
    CHECK(core.poll(id[1], &done, &err) == ECC_OK && done == 1);
    std::unique_ptr<Request> r;
    CHECK(core.wait(id[1], &r, &err) == ECC_OK);
    CHECK(r->status == ECC_OK && r->cost[1] == FakeDevice::result_of(*r, 1));
    dev.discard(*r);
    CHECK(core.poll(id[1], &done, &err) == ECC_E_ARG);  // forgotten after the wait
    dev.finish(id[0]);
    dev.finish(id[2]);
    core.pass();
    CHECK(core.n_running() == 0);
    for (int i : {0, 2}) {
        CHECK(core.wait(id[i], &r, &err) == ECC_OK && r->status == ECC_OK);
        CHECK(r->ran_slot == (i == 0 ? 0 : 1));
        dev.discard(*r);
    }
    CHECK(core.arenas_consistent() && core.dev_free_bytes() == core.dev_arena_size());
    CHECK(core.work_in_flight() == 0.0);
}

static void test_admission_waits_for_arena() {
    FakeDevice dev;
    const uint64_t one = dev_bytes_of(4, 20, dev.ws_per_hyp);
    Core core(&dev, 4, one + one / 2, 64 << 20);  // room for one request, slots for four
    int64_t a, b, c;
    std::string err;
    CHECK(core.submit(make_request(4, 20), &a, &err) == ECC_OK);
    CHECK(core.submit(make_request(4, 20), &b, &err) == ECC_OK);
    CHECK(core.submit(make_request(1, 20), &c, &err) == ECC_OK);  // small, but behind b: arrival order
    core.pass();
    CHECK(core.n_running() == 1 && core.n_pending() == 2);
    dev.finish(a);
    core.pass();
    CHECK(core.n_running() == 2 && core.n_pending() == 0);  // b, and c in the space left
    // a request larger than the whole arena fails at once
    int64_t huge;
    CHECK(core.submit(make_request(64, 20), &huge, &err) == ECC_OK);
    dev.finish(b);
    dev.finish(c);
    core.pass();
    std::unique_ptr<Request> r;
    CHECK(core.wait(huge, &r, &err) == ECC_OK && r->status == ECC_E_BUDGET);
    dev.discard(*r);
    for (int64_t i : {a, b, c}) {
        CHECK(core.wait(i, &r, &err) == ECC_OK && r->status == ECC_OK);
        dev.discard(*r);
    }
    CHECK(core.arenas_consistent() && core.dev_free_bytes() == core.dev_arena_size());
}

static void test_work_cap() {
    FakeDevice dev;
    Core core(&dev, 8, 64 << 20, 64 << 20);
    const double w = make_request(2, 10)->work;
    core.set_work_cap(2.5 * w);
    int64_t id[4];
    std::string err;
    CHECK(core.submit(make_request(2, 10), &id[0], &err) == ECC_OK);
    CHECK(core.submit(make_request(2, 10), &id[1], &err) == ECC_OK);
    CHECK(core.submit(make_request(2, 10), &id[2], &err) == ECC_OK);
    core.pass();
    CHECK(core.n_running() == 2 && core.n_pending() == 1);  // a third would exceed the cap
    CHECK(core.work_in_flight() == 2 * w);
    // a request above the cap on its own still runs on an idle device
    CHECK(core.submit(make_request(8, 10), &id[3], &err) == ECC_OK);
    dev.finish(id[0]);
    dev.finish(id[1]);
    core.pass();
    CHECK(core.n_running() == 1 && core.n_pending() == 1);  // the third; the big one waits for idle
    dev.finish(id[2]);
    core.pass();
    CHECK(core.n_running() == 1 && core.n_pending() == 0);
    dev.finish(id[3]);
    core.pass();
    std::unique_ptr<Request> r;
    for (int i = 0; i < 4; ++i) {
        CHECK(core.wait(id[i], &r, &err) == ECC_OK && r->status == ECC_OK);
        dev.discard(*r);
    }
}

static void test_failures_release_resources() {
    FakeDevice dev;
    Core core(&dev, 2, 64 << 20, 64 << 20);
    int64_t a, b, c, d;
    std::string err;
    CHECK(core.submit(make_request(2, 10), &a, &err) == ECC_OK);
    CHECK(core.submit(make_request(2, 10), &b, &err) == ECC_OK);
    CHECK(core.submit(make_request(2, 10, -1), &c, &err) == ECC_OK);  // its scan is gone
    CHECK(core.submit(make_request(2, 10), &d, &err) == ECC_OK);
    dev.fail_launch.insert(a);
    dev.fail_device.insert(b);
    core.pass();  // a fails at launch, b runs, c fails its workspace query, d runs
    core.pass();  // b's device failure is seen
    std::unique_ptr<Request> r;
    CHECK(core.wait(a, &r, &err) == ECC_OK && r->status == ECC_E_ARG && r->error == "launch refused");
    dev.discard(*r);
    CHECK(core.wait(b, &r, &err) == ECC_OK && r->status == ECC_E_HIP && r->error == "device fault");
    dev.discard(*r);
    CHECK(core.wait(c, &r, &err) == ECC_OK && r->status == ECC_E_NOSCAN);
    dev.discard(*r);
    CHECK(core.n_running() == 1);
    dev.finish(d);
    core.pass();
    CHECK(core.wait(d, &r, &err) == ECC_OK && r->status == ECC_OK);
    dev.discard(*r);
    CHECK(core.arenas_consistent() && core.dev_free_bytes() == core.dev_arena_size());
    CHECK(core.work_in_flight() == 0.0);
    CHECK(core.wait(12345, &r, &err) == ECC_E_ARG);
}

static void test_stop_fails_queued_and_drains_running() {
    FakeDevice dev;
    dev.auto_ms = 5;
    auto core = std::make_unique<Core>(&dev, 1, 64 << 20, 64 << 20);
    std::thread worker([&] { core->run(); });
    int64_t id[3];
    std::string err;
    for (int i = 0; i < 3; ++i) CHECK(core->submit(make_request(1, 8), &id[i], &err) == ECC_OK);
    while (core->n_running() == 0) std::this_thread::sleep_for(std::chrono::microseconds(50));
    core->request_stop();
    int64_t late;
    CHECK(core->submit(make_request(1, 8), &late, &err) == ECC_E_STATE);
    worker.join();
    std::unique_ptr<Request> r;
    CHECK(core->wait(id[0], &r, &err) == ECC_OK && r->status == ECC_OK);
    dev.discard(*r);
    for (int i : {1, 2}) {
        CHECK(core->wait(id[i], &r, &err) == ECC_OK && r->status == ECC_E_STATE);
        dev.discard(*r);
    }
    core.reset();
    CHECK(dev.prepared == dev.discarded);  // every completion token freed exactly once
}

static void test_concurrent_waits_on_one_request() {
    FakeDevice dev;
    dev.auto_ms = 20;
    Core core(&dev, 2, 64 << 20, 64 << 20);
    std::thread worker([&] { core.run(); });
    for (int round = 0; round < 20; ++round) {
        int64_t id;
        std::string err;
        CHECK(core.submit(make_request(2, 10, 0, round), &id, &err) == ECC_OK);
        std::atomic<int> got{0}, gone{0};
        std::vector<std::thread> waiters;
        for (int w = 0; w < 4; ++w)
            waiters.emplace_back([&] {
                std::unique_ptr<Request> r;
                std::string e;
                const ecc_status st = core.wait(id, &r, &e);
                if (st == ECC_OK) {
                    if (r->status == ECC_OK && r->cost[0] == FakeDevice::result_of(*r, 0)) ++got;
                    dev.discard(*r);
                } else if (st == ECC_E_ARG) {
                    ++gone;
                }
            });
        for (auto &t : waiters) t.join();
        CHECK(got == 1 && gone == 3);
    }
    core.request_stop();
    worker.join();
    CHECK(dev.prepared == dev.discarded);
}

static void test_threaded_clients() {
    FakeDevice dev;
    dev.auto_ms = 1;
    Core core(&dev, 4, 3 * dev_bytes_of(8, 30, dev.ws_per_hyp), 64 << 20);
    core.set_work_cap(3 * make_request(8, 30)->work);
    std::thread worker([&] { core.run(); });
    std::atomic<int> ok{0}, bad{0};
    std::vector<std::thread> clients;
    for (int c = 0; c < 8; ++c)
        clients.emplace_back([&, c] {
            std::mt19937 rng(100 + c);
            for (int i = 0; i < 40; ++i) {
                const int B = 1 + rng() % 8, n = 5 + rng() % 26;
                int64_t id;
                std::string err;
                auto r = make_request(B, n, 0, c * 1000 + i);
                if (core.submit(std::move(r), &id, &err) != ECC_OK) {
                    ++bad;
                    continue;
                }
                std::unique_ptr<Request> out;
                if (core.wait(id, &out, &err) == ECC_OK && out->status == ECC_OK) {
                    bool same = true;
                    for (int b = 0; b < B; ++b) same &= out->cost[b] == FakeDevice::result_of(*out, b);
                    same ? ++ok : ++bad;
                    dev.discard(*out);
                } else {
                    ++bad;
                }
            }
        });
    for (auto &t : clients) t.join();
    core.request_stop();
    worker.join();
    CHECK(ok == 320 && bad == 0);
    CHECK(core.arenas_consistent() && core.dev_free_bytes() == core.dev_arena_size());
    CHECK(core.work_in_flight() == 0.0);
    CHECK(dev.prepared == dev.discarded);
}

int main(int argc, char **argv) {
    const std::string which = argc > 1 ? argv[1] : "all";
    if (which == "all" || which == "serial") {
        test_arena();
        test_fifo_admission_by_slot();
        test_admission_waits_for_arena();
        test_work_cap();
        test_failures_release_resources();
    }
    if (which == "all" || which == "threads") {
        test_stop_fails_queued_and_drains_running();
        test_concurrent_waits_on_one_request();
        test_threaded_clients();
    }
    if (g_failures) {
        fprintf(stderr, "%d check(s) failed\n", g_failures);
        return 1;
    }
    printf("server core tests passed (%s)\n", which.c_str());
    return 0;
}
