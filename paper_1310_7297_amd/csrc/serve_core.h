// Scheduling core of the serving loop, host code only (no HIP): admission by
// a memory budget, a FIFO of admitted requests, batched launches on a fixed
// number of slots, completion, latency statistics and shutdown.  The device
// side is an Executor: serve.hip gives it streams and batched kernel
// launches; the host tests give it a fake that finishes launches when told,
// so that admission and ordering are checked without a GPU (and under the
// address, undefined-behaviour and thread sanitizers).
//
// Threading: submit / poll / wait / drain / stats / hold may be called from
// any thread; run() is the engine loop, on a thread of its own, and is the
// only caller of the Executor.  One mutex guards all state.
#pragma once

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "vcm.h"

namespace vcm {
namespace serve {

using Clock = std::chrono::steady_clock;

// What the engine needs from the device.  A slot runs at most one launch at
// a time.
template <class Payload>
class Executor {
public:
    virtual ~Executor() = default;
    // Start one launch of the given requests on `slot`.  VCM_OK: running
    // (poll() reports its end); otherwise nothing runs and *msg says why.
    virtual vcm_status start(int slot, const std::vector<const Payload *> &batch, std::string *msg) = 0;
    // VCM_E_PENDING while the launch on `slot` runs; then VCM_OK, or the
    // error that ended it (with *msg).
    virtual vcm_status poll(int slot, std::string *msg) = 0;
};

struct RequestInfo {
    double latency_ms = 0.0;  // submit to completion seen by the engine
    double queue_ms = 0.0;    // submit to launch
    uint64_t viewpoints = 0;
};

struct Stats {
    uint64_t completed = 0, failed = 0, rejected = 0, launches = 0, viewpoints = 0;
    double p50_ms = 0.0, p99_ms = 0.0, max_ms = 0.0;
    double requests_per_s = 0.0, viewpoints_per_s = 0.0;
    size_t mem_in_use = 0, mem_peak = 0, mem_budget = 0;
};

// Nearest-rank percentile of v (0 when empty).
inline double percentile(std::vector<double> v, double p) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    size_t k = static_cast<size_t>(std::ceil(p / 100.0 * static_cast<double>(v.size())));
    k = std::min(std::max<size_t>(k, 1), v.size());
    return v[k - 1];
}

template <class Payload>
class Core {
public:
    Core(size_t budget, int slots, int max_batch, Executor<Payload> *ex)
        : budget_(budget), max_batch_(max_batch), ex_(ex), slots_(static_cast<size_t>(slots)) {}

    // Admit a request of `footprint` bytes.  VCM_E_INVALID: larger than the
    // whole budget, or the core is stopping; VCM_E_AGAIN: the budget is in
    // use now (counted as a rejection, nothing queued).
    vcm_status submit(Payload p, size_t footprint, uint64_t viewpoints, uint64_t *ticket, std::string *msg) {
        std::lock_guard<std::mutex> lock(m_);
        if (stop_) {
            *msg = "server is shutting down";
            return VCM_E_INVALID;
        }
        if (footprint > budget_) {
            *msg = "request needs " + std::to_string(footprint) + " bytes, more than the whole budget";
            return VCM_E_INVALID;
        }
        if (used_ + footprint > budget_) {
            ++rejected_;
            *msg = "memory budget in use; retry later";
            return VCM_E_AGAIN;
        }
        used_ += footprint;
        peak_ = std::max(peak_, used_);
        const uint64_t t = next_++;
        Request &r = req_[t];
        r.payload = std::move(p);
        r.footprint = footprint;
        r.viewpoints = viewpoints;
        r.t_submit = Clock::now();
        waiting_.push_back(t);
        cv_.notify_all();
        *ticket = t;
        return VCM_OK;
    }

    // VCM_E_PENDING while unfinished; then the request's status, once.
    vcm_status poll(uint64_t t, RequestInfo *info, std::string *msg) {
        std::lock_guard<std::mutex> lock(m_);
        return poll_locked(t, info, msg);
    }

    // poll after waiting up to timeout_ms (< 0: no limit).
    vcm_status wait(uint64_t t, int timeout_ms, RequestInfo *info, std::string *msg) {
        std::unique_lock<std::mutex> lock(m_);
        auto ready = [&] {
            auto it = req_.find(t);
            return it == req_.end() || it->second.done;
        };
        if (timeout_ms < 0)
            cv_.wait(lock, ready);
        else
            cv_.wait_for(lock, std::chrono::milliseconds(timeout_ms), ready);
        return poll_locked(t, info, msg);
    }

    // Wait until nothing is queued or running.  While launches are held,
    // queued requests do not count (they would never start).
    void drain() {
        std::unique_lock<std::mutex> lock(m_);
        cv_.wait(lock, [&] {
            if (!hold_ && !waiting_.empty()) return false;
            for (const Slot &s : slots_)
                if (s.busy) return false;
            return true;
        });
    }

    // Hold launches: admitted requests queue but none starts until released;
    // on release every free slot takes up to max_batch of them at once.
    void hold(bool on) {
        std::lock_guard<std::mutex> lock(m_);
        hold_ = on;
        cv_.notify_all();
    }

    Stats stats() {
        std::lock_guard<std::mutex> lock(m_);
        Stats s;
        s.completed = completed_;
        s.failed = failed_;
        s.rejected = rejected_;
        s.launches = launches_;
        s.viewpoints = vp_done_;
        s.p50_ms = percentile(latency_ms_, 50.0);
        s.p99_ms = percentile(latency_ms_, 99.0);
        s.max_ms = latency_ms_.empty() ? 0.0 : *std::max_element(latency_ms_.begin(), latency_ms_.end());
        const double span = any_ ? std::chrono::duration<double>(t_last_ - t_first_).count() : 0.0;
        s.requests_per_s = span > 0 ? static_cast<double>(completed_) / span : 0.0;
        s.viewpoints_per_s = span > 0 ? static_cast<double>(vp_done_) / span : 0.0;
        s.mem_in_use = used_;
        s.mem_peak = peak_;
        s.mem_budget = budget_;
        return s;
    }

    void reset_stats() {
        std::lock_guard<std::mutex> lock(m_);
        latency_ms_.clear();
        completed_ = failed_ = rejected_ = launches_ = vp_done_ = 0;
        peak_ = used_;
        any_ = false;
    }

    // Ask the engine to stop: queued requests are cancelled, launches in
    // flight are waited for, then run() returns.
    void stop() {
        std::lock_guard<std::mutex> lock(m_);
        stop_ = true;
        cv_.notify_all();
    }

    // The engine loop.  `idle_poll` is how long it sleeps between looks at
    // launches in flight.
    void run(std::chrono::microseconds idle_poll = std::chrono::microseconds(50)) {
        std::unique_lock<std::mutex> lock(m_);
        for (;;) {
            bool busy = false;
            for (size_t i = 0; i < slots_.size(); ++i) {
                Slot &s = slots_[i];
                if (!s.busy) continue;
                std::string msg;
                const vcm_status st = ex_->poll(static_cast<int>(i), &msg);
                if (st == VCM_E_PENDING) {
                    busy = true;
                    continue;
                }
                for (uint64_t t : s.tickets) finish(t, st, msg);
                s.tickets.clear();
                s.busy = false;
            }
            if (stop_) {
                while (!waiting_.empty()) {
                    finish(waiting_.front(), VCM_E_INTERNAL, "cancelled: server shut down");
                    waiting_.pop_front();
                }
                cv_.notify_all();
                if (!busy) break;
            }
            for (size_t i = 0; i < slots_.size() && !hold_ && !waiting_.empty(); ++i) {
                Slot &s = slots_[i];
                if (s.busy) continue;
                std::vector<uint64_t> tk;
                std::vector<const Payload *> batch;
                const Clock::time_point now = Clock::now();
                while (!waiting_.empty() && static_cast<int>(tk.size()) < max_batch_) {
                    const uint64_t t = waiting_.front();
                    waiting_.pop_front();
                    Request &r = req_[t];
                    r.t_launch = now;
                    tk.push_back(t);
                    batch.push_back(&r.payload);
                }
                std::string msg;
                const vcm_status st = ex_->start(static_cast<int>(i), batch, &msg);
                if (st != VCM_OK) {
                    for (uint64_t t : tk) finish(t, st, msg);
                    continue;
                }
                s.tickets = std::move(tk);
                s.busy = true;
                ++launches_;
                busy = true;
            }
            cv_.notify_all();
            if (busy)
                cv_.wait_for(lock, idle_poll);
            else
                cv_.wait(lock, [&] { return stop_ || (!hold_ && !waiting_.empty()); });
        }
        cv_.notify_all();
    }

private:
    struct Request {
        Payload payload{};
        size_t footprint = 0;
        uint64_t viewpoints = 0;
        Clock::time_point t_submit, t_launch, t_done;
        bool done = false;
        vcm_status status = VCM_OK;
        std::string message;
    };
    struct Slot {
        std::vector<uint64_t> tickets;
        bool busy = false;
    };

    void finish(uint64_t t, vcm_status st, const std::string &msg) {
        auto it = req_.find(t);
        if (it == req_.end()) return;
        Request &r = it->second;
        r.done = true;
        r.status = st;
        r.message = msg;
        r.t_done = Clock::now();
        if (r.t_launch == Clock::time_point{}) r.t_launch = r.t_done;
        used_ -= r.footprint;
        if (st == VCM_OK) {
            ++completed_;
            vp_done_ += r.viewpoints;
            latency_ms_.push_back(std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count());
            if (!any_ || r.t_submit < t_first_) t_first_ = r.t_submit;
            if (!any_ || r.t_done > t_last_) t_last_ = r.t_done;
            any_ = true;
        } else {
            ++failed_;
        }
    }

    vcm_status poll_locked(uint64_t t, RequestInfo *info, std::string *msg) {
        auto it = req_.find(t);
        if (it == req_.end()) {
            *msg = "unknown ticket";
            return VCM_E_NOTFOUND;
        }
        Request &r = it->second;
        if (!r.done) return VCM_E_PENDING;
        if (info) {
            info->latency_ms = std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count();
            info->queue_ms = std::chrono::duration<double, std::milli>(r.t_launch - r.t_submit).count();
            info->viewpoints = r.viewpoints;
        }
        const vcm_status st = r.status;
        *msg = r.message;
        req_.erase(it);
        return st;
    }

    const size_t budget_;
    const int max_batch_;
    Executor<Payload> *const ex_;

    std::mutex m_;
    std::condition_variable cv_;
    bool stop_ = false, hold_ = false;
    uint64_t next_ = 1;
    size_t used_ = 0, peak_ = 0;
    std::unordered_map<uint64_t, Request> req_;
    std::deque<uint64_t> waiting_;
    std::vector<Slot> slots_;

    std::vector<double> latency_ms_;
    uint64_t completed_ = 0, failed_ = 0, rejected_ = 0, launches_ = 0, vp_done_ = 0;
    Clock::time_point t_first_, t_last_;
    bool any_ = false;
};

}  // namespace serve
}  // namespace vcm
