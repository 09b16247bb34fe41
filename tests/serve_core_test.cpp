// Host test of the serving loop's scheduling core with a fake executor: no
// GPU, deterministic (launches finish only when the test says so).  Built
// and run by test_serve_core.py, plain and under the address,
// undefined-behaviour and thread sanitizers.  Exit status 0 when every check
// holds; a failed check prints its line and exits 1.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "serve_core.h"

using vcm::serve::Core;
using vcm::serve::Executor;
using vcm::serve::RequestInfo;

#define CHECK(cond)                                                          \
    do {                                                                     \
        if (!(cond)) {                                                       \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            std::exit(1);                                                    \
        }                                                                    \
    } while (0)

// Launches run until finish() is called for their slot (or at once with
// auto_finish); start can be made to fail.
class Fake final : public Executor<int> {
public:
    explicit Fake(int slots) : state_(static_cast<size_t>(slots), 0) {}

    vcm_status start(int slot, const std::vector<const int *> &batch, std::string *msg) override {
        std::lock_guard<std::mutex> lock(m_);
        CHECK(state_[slot] == 0);
        std::vector<int> ids;
        for (const int *p : batch) ids.push_back(*p);
        started_.push_back(ids);
        slot_of_.push_back(slot);
        if (fail_start_) {
            *msg = "fake start failure";
            return VCM_E_DEVICE;
        }
        state_[slot] = auto_finish_ ? 2 : 1;
        return VCM_OK;
    }
    vcm_status poll(int slot, std::string *msg) override {
        std::lock_guard<std::mutex> lock(m_);
        const int s = state_[slot];
        if (s == 1) return VCM_E_PENDING;
        state_[slot] = 0;
        if (s == 3) {
            *msg = "fake launch failure";
            return VCM_E_DEVICE;
        }
        CHECK(s == 2);
        return VCM_OK;
    }
    void finish(int slot, bool ok = true) {
        std::lock_guard<std::mutex> lock(m_);
        CHECK(state_[slot] == 1);
        state_[slot] = ok ? 2 : 3;
    }
    size_t launches() {
        std::lock_guard<std::mutex> lock(m_);
        return started_.size();
    }
    std::vector<int> batch(size_t i) {
        std::lock_guard<std::mutex> lock(m_);
        return started_.at(i);
    }
    int slot(size_t i) {
        std::lock_guard<std::mutex> lock(m_);
        return slot_of_.at(i);
    }
    void set_auto(bool on) {
        std::lock_guard<std::mutex> lock(m_);
        auto_finish_ = on;
    }
    void set_fail_start(bool on) {
        std::lock_guard<std::mutex> lock(m_);
        fail_start_ = on;
    }

private:
    std::mutex m_;
    std::vector<int> state_;  // 0 idle, 1 running, 2 finished, 3 failed
    std::vector<std::vector<int>> started_;
    std::vector<int> slot_of_;
    bool auto_finish_ = false, fail_start_ = false;
};

// Wait (bounded) until the fake has seen n launches.
static void await_launches(Fake &f, size_t n) {
    const auto t0 = std::chrono::steady_clock::now();
    while (f.launches() < n) {
        CHECK(std::chrono::steady_clock::now() - t0 < std::chrono::seconds(20));
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
}

struct Rig {
    Fake fake;
    Core<int> core;
    std::thread engine;
    Rig(size_t budget, int slots, int max_batch) : fake(slots), core(budget, slots, max_batch, &fake) {
        engine = std::thread([this] { core.run(std::chrono::microseconds(20)); });
    }
    ~Rig() {
        core.stop();
        engine.join();
    }
    uint64_t submit(int id, size_t bytes, vcm_status want = VCM_OK) {
        uint64_t t = 0;
        std::string msg;
        const vcm_status st = core.submit(id, bytes, 10, &t, &msg);
        CHECK(st == want);
        return t;
    }
    vcm_status wait(uint64_t t) {
        std::string msg;
        RequestInfo info;
        return core.wait(t, 20000, &info, &msg);
    }
};

// Admission by budget: refused while the budget is in use, admitted again
// once a request finishes; larger than the whole budget is invalid.
static void test_admission() {
    Rig r(100, 1, 64);
    r.core.hold(true);
    const uint64_t a = r.submit(1, 40), b = r.submit(2, 40);
    r.submit(3, 40, VCM_E_AGAIN);
    r.submit(4, 101, VCM_E_INVALID);
    CHECK(r.core.stats().rejected == 1);
    CHECK(r.core.stats().mem_in_use == 80);
    r.core.hold(false);
    await_launches(r.fake, 1);
    CHECK((r.fake.batch(0) == std::vector<int>{1, 2}));
    r.submit(5, 40, VCM_E_AGAIN);  // the launch still holds its budget
    r.fake.finish(0);
    CHECK(r.wait(a) == VCM_OK && r.wait(b) == VCM_OK);
    CHECK(r.core.stats().mem_in_use == 0);
    const uint64_t c = r.submit(6, 100);
    await_launches(r.fake, 2);
    r.fake.finish(0);
    CHECK(r.wait(c) == VCM_OK);
    const auto s = r.core.stats();
    CHECK(s.mem_peak <= 100 && s.completed == 3 && s.failed == 0 && s.rejected == 2);
}

// Held requests go out in submission order, max_batch per launch.
static void test_hold_batches_in_order() {
    Rig r(1 << 20, 1, 3);
    r.core.hold(true);
    std::vector<uint64_t> t;
    for (int i = 1; i <= 8; ++i) t.push_back(r.submit(i, 10));
    std::this_thread::sleep_for(std::chrono::milliseconds(2));
    CHECK(r.fake.launches() == 0);
    r.core.hold(false);
    await_launches(r.fake, 1);
    CHECK((r.fake.batch(0) == std::vector<int>{1, 2, 3}));
    r.fake.finish(0);
    await_launches(r.fake, 2);
    CHECK((r.fake.batch(1) == std::vector<int>{4, 5, 6}));
    r.fake.finish(0);
    await_launches(r.fake, 3);
    CHECK((r.fake.batch(2) == std::vector<int>{7, 8}));
    r.fake.finish(0);
    for (uint64_t x : t) CHECK(r.wait(x) == VCM_OK);
    CHECK(r.core.stats().launches == 3);
}

// Continuous batching: requests that arrive while the only slot runs wait
// and share the next launch.
static void test_arrivals_share_the_next_launch() {
    Rig r(1 << 20, 1, 64);
    const uint64_t a = r.submit(1, 10);
    await_launches(r.fake, 1);
    std::vector<uint64_t> t;
    for (int i = 2; i <= 6; ++i) t.push_back(r.submit(i, 10));
    std::string msg;
    RequestInfo info;
    CHECK(r.core.poll(t[0], &info, &msg) == VCM_E_PENDING);
    r.fake.finish(0);
    await_launches(r.fake, 2);
    CHECK((r.fake.batch(1) == std::vector<int>{2, 3, 4, 5, 6}));
    r.fake.finish(0);
    CHECK(r.wait(a) == VCM_OK);
    for (uint64_t x : t) CHECK(r.wait(x) == VCM_OK);
    CHECK(r.core.stats().launches == 2);
}

// Two slots: a second launch starts while the first runs.
static void test_two_slots_overlap() {
    Rig r(1 << 20, 2, 64);
    const uint64_t a = r.submit(1, 10);
    await_launches(r.fake, 1);
    const uint64_t b = r.submit(2, 10);
    await_launches(r.fake, 2);
    CHECK(r.fake.slot(0) != r.fake.slot(1));
    r.fake.finish(r.fake.slot(1));
    CHECK(r.wait(b) == VCM_OK);
    std::string msg;
    RequestInfo info;
    CHECK(r.core.poll(a, &info, &msg) == VCM_E_PENDING);
    r.fake.finish(r.fake.slot(0));
    CHECK(r.wait(a) == VCM_OK);
}

// A ticket reports its end once; unknown tickets are not found.
static void test_poll_semantics() {
    Rig r(1 << 20, 1, 64);
    const uint64_t a = r.submit(1, 10);
    await_launches(r.fake, 1);
    std::string msg;
    RequestInfo info;
    CHECK(r.core.poll(a, &info, &msg) == VCM_E_PENDING);
    r.fake.finish(0);
    CHECK(r.core.wait(a, 20000, &info, &msg) == VCM_OK);
    CHECK(info.viewpoints == 10 && info.latency_ms >= info.queue_ms && info.queue_ms >= 0.0);
    CHECK(r.core.poll(a, &info, &msg) == VCM_E_NOTFOUND);
    CHECK(r.core.poll(999, &info, &msg) == VCM_E_NOTFOUND);
}

// Failures: a launch that cannot start and a launch that fails both end
// their requests with the error and return the budget.
static void test_failures() {
    Rig r(1000, 1, 64);
    r.fake.set_fail_start(true);
    const uint64_t a = r.submit(1, 10);
    CHECK(r.wait(a) == VCM_E_DEVICE);
    r.fake.set_fail_start(false);
    const uint64_t b = r.submit(2, 10);
    await_launches(r.fake, 2);
    r.fake.finish(0, false);
    CHECK(r.wait(b) == VCM_E_DEVICE);
    const auto s = r.core.stats();
    CHECK(s.failed == 2 && s.completed == 0 && s.mem_in_use == 0);
}

// Shutdown: queued requests are cancelled, the launch in flight finishes.
static void test_shutdown() {
    Fake fake(1);
    Core<int> core(1 << 20, 1, 2, &fake);
    std::thread engine([&] { core.run(std::chrono::microseconds(20)); });
    uint64_t t[4];
    std::string msg;
    core.hold(true);
    for (int i = 0; i < 4; ++i) CHECK(core.submit(i, 10, 1, &t[i], &msg) == VCM_OK);
    core.hold(false);
    await_launches(fake, 1);  // the first two run, the last two wait
    CHECK((fake.batch(0) == std::vector<int>{0, 1}));
    core.stop();
    std::this_thread::sleep_for(std::chrono::milliseconds(2));
    RequestInfo info;
    CHECK(core.poll(t[2], &info, &msg) == VCM_E_INTERNAL);
    CHECK(core.poll(t[3], &info, &msg) == VCM_E_INTERNAL);
    CHECK(core.poll(t[0], &info, &msg) == VCM_E_PENDING);
    fake.finish(0);
    engine.join();
    CHECK(core.poll(t[0], &info, &msg) == VCM_OK && core.poll(t[1], &info, &msg) == VCM_OK);
    CHECK(core.submit(9, 10, 1, &t[0], &msg) == VCM_E_INVALID);
}

static void test_percentile() {
    std::vector<double> v;
    for (int i = 100; i >= 1; --i) v.push_back(i);
    CHECK(vcm::serve::percentile(v, 50.0) == 50.0);
    CHECK(vcm::serve::percentile(v, 99.0) == 99.0);
    CHECK(vcm::serve::percentile({7.0}, 99.0) == 7.0);
    CHECK(vcm::serve::percentile({}, 50.0) == 0.0);
}

// Many submitters and waiters at once, launches finishing immediately:
// every request completes exactly once and the budget is never exceeded.
static void test_concurrent() {
    Rig r(5000, 3, 16);
    r.fake.set_auto(true);
    constexpr int kThreads = 4, kEach = 300;
    std::atomic<int> ok{0};
    std::vector<std::thread> th;
    for (int w = 0; w < kThreads; ++w)
        th.emplace_back([&, w] {
            std::mt19937 g(w);
            std::vector<uint64_t> mine;
            for (int i = 0; i < kEach; ++i) {
                uint64_t t = 0;
                std::string msg;
                const size_t bytes = 50 + g() % 400;
                for (;;) {
                    const vcm_status st = r.core.submit(w * kEach + i, bytes, 1, &t, &msg);
                    if (st == VCM_OK) break;
                    CHECK(st == VCM_E_AGAIN);
                    if (!mine.empty()) {
                        RequestInfo info;
                        CHECK(r.core.wait(mine.front(), 20000, &info, &msg) == VCM_OK);
                        mine.erase(mine.begin());
                        ++ok;
                    } else {
                        std::this_thread::yield();
                    }
                }
                mine.push_back(t);
            }
            for (uint64_t t : mine) {
                RequestInfo info;
                std::string msg;
                CHECK(r.core.wait(t, 20000, &info, &msg) == VCM_OK);
                ++ok;
            }
        });
    for (auto &t : th) t.join();
    r.core.drain();
    const auto s = r.core.stats();
    CHECK(ok.load() == kThreads * kEach);
    CHECK(s.completed == static_cast<uint64_t>(kThreads * kEach) && s.failed == 0);
    CHECK(s.mem_in_use == 0 && s.mem_peak <= 5000);
    CHECK(s.launches <= s.completed);
}

int main() {
    test_percentile();
    test_admission();
    test_hold_batches_in_order();
    test_arrivals_share_the_next_launch();
    test_two_slots_overlap();
    test_poll_semantics();
    test_failures();
    test_shutdown();
    test_concurrent();
    std::printf("serve core: all checks passed\n");
    return 0;
}
