// Serving loop: admission by device memory, continuous batching, latency
// statistics.
//
// Callers submit queries from any thread.  A request is admitted when its
// device footprint (its result buffers, its work record and, for the pruned
// methods, its block gates) fits in what the budget has left; otherwise the
// submit returns VCM_E_AGAIN and the caller retries later.  One engine thread
// per server turns the admitted requests into batched launches: whenever a
// launch slot (a stream) is free it takes every waiting request (up to
// max_batch) into one persistent launch, so requests that arrive while
// others run are batched together and start as soon as a slot frees up,
// overlapping on the device with the launches still running.  Completion is
// observed through events; the budget is returned then.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "vcm_internal.h"

using namespace vcm;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    vcm_query query;
    vcm_result result;
    size_t footprint = 0;
    uint64_t viewpoints = 0;
    Clock::time_point t_submit, t_launch, t_done;
    bool done = false;
    vcm_status status = VCM_OK;
    std::string message;
};

struct Launch {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::vector<uint64_t> tickets;
    bool busy = false;
};

}  // namespace

struct vcm_server {
    const Index *ix = nullptr;
    int device = 0;
    vcm_server_opts opts{};
    Tuning tune;

    std::mutex m;
    std::condition_variable cv;
    bool stop = false;
    std::thread engine;

    uint64_t next_ticket = 1;
    size_t used = 0;
    std::unordered_map<uint64_t, Request> req;
    std::deque<uint64_t> waiting;
    std::vector<Launch> slots;

    // statistics (completed requests)
    std::vector<double> latency_ms;
    uint64_t completed = 0, failed = 0, rejected = 0, launches = 0, vp_done = 0;
    size_t peak_used = 0;
    Clock::time_point t_first, t_last;
    bool any = false;
};

namespace {

// Device bytes a request holds while admitted.
size_t footprint(const vcm_query &q, const vcm_result &r, uint64_t n) {
    size_t b = 0;
    if (r.bin) b += n;
    if (r.c) b += 4 * n;
    if (r.count) b += 2 * n;
    b += sizeof(BruteArgs) + 64;
    if (q.params.method != VCM_BRUTE) {
        const int th = std::max(1, q.params.theta_blocks);
        uint64_t blocks = 1;
        for (int k = 0; k < 3; ++k) blocks *= (static_cast<uint64_t>(std::max(q.grid.n[k], 1)) + th - 1) / th;
        b += 4 * blocks;
    }
    return b;
}

void finish(vcm_server *s, uint64_t t, vcm_status st, const std::string &msg) {
    auto it = s->req.find(t);
    if (it == s->req.end()) return;
    Request &r = it->second;
    r.done = true;
    r.status = st;
    r.message = msg;
    r.t_done = Clock::now();
    s->used -= r.footprint;
    if (st == VCM_OK) {
        ++s->completed;
        s->vp_done += r.viewpoints;
        s->latency_ms.push_back(std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count());
        if (!s->any || r.t_submit < s->t_first) s->t_first = r.t_submit;
        if (!s->any || r.t_done > s->t_last) s->t_last = r.t_done;
        s->any = true;
    } else {
        ++s->failed;
    }
}

// Enqueue one launch of the given requests on a slot's stream (engine thread,
// lock held).  The plan's buffer is allocated and freed in stream order.
void dispatch(vcm_server *s, Launch &L, std::vector<uint64_t> &&tk) {
    std::vector<vcm_query> qs;
    std::vector<vcm_result> rs;
    for (uint64_t t : tk) {
        Request &r = s->req[t];
        r.t_launch = Clock::now();
        qs.push_back(r.query);
        rs.push_back(r.result);
    }
    BatchPlan p;
    p.device = s->device;
    p.tune = s->tune;
    vcm_status st = p.prepare(*s->ix, qs.data(), static_cast<int>(qs.size()), rs.data());
    if (st == VCM_OK) {
        p.layout();
        const hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&p.d_base), p.bytes, L.stream);
        if (e != hipSuccess) st = set_error(VCM_E_NOMEM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
    }
    if (st == VCM_OK) {
        std::vector<char> img;
        p.image(img);
        st = upload(img.data(), img.size(), p.d_base, s->device, L.stream);
        if (st == VCM_OK) st = p.enqueue(L.stream, nullptr);
        hipFreeAsync(p.d_base, L.stream);
    }
    if (st == VCM_OK && hipEventRecord(L.done, L.stream) != hipSuccess)
        st = set_error(VCM_E_DEVICE, "event record failed");
    if (st != VCM_OK) {
        const std::string msg = vcm_last_error();
        hipStreamSynchronize(L.stream);
        for (uint64_t t : tk) finish(s, t, st, msg);
        return;
    }
    L.tickets = std::move(tk);
    L.busy = true;
    ++s->launches;
}

void engine_main(vcm_server *s) {
    hipSetDevice(s->device);
    std::unique_lock<std::mutex> lock(s->m);
    for (;;) {
        // completions
        bool busy = false;
        for (auto &L : s->slots) {
            if (!L.busy) continue;
            const hipError_t q = hipEventQuery(L.done);
            if (q == hipErrorNotReady) {
                busy = true;
                continue;
            }
            const vcm_status st = q == hipSuccess ? VCM_OK : VCM_E_DEVICE;
            const std::string msg = q == hipSuccess ? "" : std::string("launch failed: ") + hipGetErrorString(q);
            for (uint64_t t : L.tickets) finish(s, t, st, msg);
            L.tickets.clear();
            L.busy = false;
        }
        if (s->stop) {
            // shutting down: requests not yet launched are cancelled, the
            // launches in flight are waited for
            while (!s->waiting.empty()) {
                finish(s, s->waiting.front(), VCM_E_INTERNAL, "cancelled: server shut down");
                s->waiting.pop_front();
            }
            s->cv.notify_all();
            if (!busy) break;
        }
        // new launches: every waiting request, up to max_batch per launch
        for (auto &L : s->slots) {
            if (s->waiting.empty()) break;
            if (L.busy) continue;
            std::vector<uint64_t> tk;
            while (!s->waiting.empty() && static_cast<int>(tk.size()) < s->opts.max_batch) {
                tk.push_back(s->waiting.front());
                s->waiting.pop_front();
            }
            dispatch(s, L, std::move(tk));
            busy = busy || L.busy;
        }
        s->cv.notify_all();  // completions wake waiters
        if (busy)
            s->cv.wait_for(lock, std::chrono::microseconds(50));
        else
            s->cv.wait(lock, [s] { return s->stop || !s->waiting.empty(); });
    }
    s->cv.notify_all();
}

double percentile(std::vector<double> v, double p) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    // nearest rank
    size_t k = static_cast<size_t>(std::ceil(p / 100.0 * v.size()));
    k = std::min(std::max<size_t>(k, 1), v.size());
    return v[k - 1];
}

}  // namespace

extern "C" {

vcm_status vcm_server_create(const vcm_index *index, const vcm_server_opts *opts, vcm_server **out) {
    clear_error();
    if (!index || !out) return set_error(VCM_E_INVALID, "null argument");
    vcm_server_opts o{};
    if (opts) o = *opts;
    if (o.max_inflight == 0) o.max_inflight = 2;
    if (o.max_batch == 0) o.max_batch = 64;
    if (o.max_inflight < 1 || o.max_inflight > 8) return set_error(VCM_E_INVALID, "max_inflight must be in 1..8");
    if (o.max_batch < 1 || o.max_batch > 4096) return set_error(VCM_E_INVALID, "max_batch must be in 1..4096");
    if (o.chunk < 0 || o.chunk > 64) return set_error(VCM_E_INVALID, "chunk must be in 0..64");
    if (o.blocks_per_cu < 0 || o.blocks_per_cu > 16) return set_error(VCM_E_INVALID, "blocks_per_cu must be in 0..16");
    const Index &ix = index->impl;
    DeviceGuard guard(ix.device);
    if (o.mem_budget_bytes == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return set_error(VCM_E_DEVICE, "hipMemGetInfo failed");
        o.mem_budget_bytes = free_b / 2;
    }
    vcm_server *s = new (std::nothrow) vcm_server;
    if (!s) return set_error(VCM_E_NOMEM, "host allocation failed");
    s->ix = &ix;
    s->device = ix.device;
    s->opts = o;
    if (o.chunk) s->tune.chunk = o.chunk;
    if (o.blocks_per_cu) s->tune.blocks_per_cu = o.blocks_per_cu;
    device_cus(ix.device);
    s->slots.resize(o.max_inflight);
    for (auto &L : s->slots) {
        if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess) {
            for (auto &x : s->slots) {
                if (x.stream) hipStreamDestroy(x.stream);
                if (x.done) hipEventDestroy(x.done);
            }
            delete s;
            return set_error(VCM_E_DEVICE, "stream or event creation failed");
        }
    }
    s->engine = std::thread(engine_main, s);
    *out = s;
    return VCM_OK;
}

vcm_status vcm_submit(vcm_server *server, const vcm_query *query, const vcm_result *result,
                      uint64_t *ticket) {
    clear_error();
    if (!server || !query || !result || !ticket) return set_error(VCM_E_INVALID, "null argument");
    if (!result->bin) return set_error(VCM_E_INVALID, "result->bin is required");
    if (result->host) return set_error(VCM_E_INVALID, "served requests need device result buffers");
    // validate now, so that a bad request fails at submit, not in the engine
    TargetDesc t;
    GridDesc g;
    ParamDesc p;
    vcm_status st = prepare_query(*server->ix, *query, &t, &g, &p);
    if (st != VCM_OK) return st;
    if (g.count >= (int64_t(1) << 31)) return set_error(VCM_E_INVALID, "grid too large to serve");
    const uint64_t n = static_cast<uint64_t>(g.count);
    const size_t f = footprint(*query, *result, n);
    std::lock_guard<std::mutex> lock(server->m);
    if (server->stop) return set_error(VCM_E_INVALID, "server is shutting down");
    if (f > server->opts.mem_budget_bytes)
        return set_error(VCM_E_INVALID, "request needs " + std::to_string(f) + " bytes, more than the whole budget");
    if (server->used + f > server->opts.mem_budget_bytes) {
        ++server->rejected;
        return set_error(VCM_E_AGAIN, "memory budget in use; retry later");
    }
    server->used += f;
    server->peak_used = std::max(server->peak_used, server->used);
    const uint64_t tk = server->next_ticket++;
    Request &r = server->req[tk];
    r.query = *query;
    r.result = *result;
    r.footprint = f;
    r.viewpoints = n;
    r.t_submit = Clock::now();
    server->waiting.push_back(tk);
    server->cv.notify_all();
    *ticket = tk;
    return VCM_OK;
}

vcm_status vcm_poll(vcm_server *server, uint64_t ticket, vcm_request_info *info) {
    clear_error();
    if (!server) return set_error(VCM_E_INVALID, "null server");
    std::lock_guard<std::mutex> lock(server->m);
    auto it = server->req.find(ticket);
    if (it == server->req.end()) return set_error(VCM_E_NOTFOUND, "unknown ticket");
    Request &r = it->second;
    if (!r.done) return VCM_E_PENDING;
    if (info) {
        info->latency_ms = std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count();
        info->queue_ms = std::chrono::duration<double, std::milli>(r.t_launch - r.t_submit).count();
        info->viewpoints = r.viewpoints;
    }
    const vcm_status st = r.status;
    const std::string msg = r.message;
    server->req.erase(it);
    if (st != VCM_OK) return set_error(st, msg);
    return VCM_OK;
}

vcm_status vcm_wait(vcm_server *server, uint64_t ticket, int32_t timeout_ms, vcm_request_info *info) {
    clear_error();
    if (!server) return set_error(VCM_E_INVALID, "null server");
    {
        std::unique_lock<std::mutex> lock(server->m);
        auto ready = [&] {
            auto it = server->req.find(ticket);
            return it == server->req.end() || it->second.done;
        };
        if (timeout_ms < 0)
            server->cv.wait(lock, ready);
        else
            server->cv.wait_for(lock, std::chrono::milliseconds(timeout_ms), ready);
    }
    return vcm_poll(server, ticket, info);
}

vcm_status vcm_server_drain(vcm_server *server) {
    clear_error();
    if (!server) return set_error(VCM_E_INVALID, "null server");
    std::unique_lock<std::mutex> lock(server->m);
    server->cv.wait(lock, [&] {
        if (!server->waiting.empty()) return false;
        for (auto &L : server->slots)
            if (L.busy) return false;
        return true;
    });
    return VCM_OK;
}

vcm_status vcm_server_get_stats(vcm_server *server, vcm_server_stats *out) {
    clear_error();
    if (!server || !out) return set_error(VCM_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lock(server->m);
    out->completed = server->completed;
    out->failed = server->failed;
    out->rejected = server->rejected;
    out->launches = server->launches;
    out->viewpoints = server->vp_done;
    out->p50_ms = percentile(server->latency_ms, 50.0);
    out->p99_ms = percentile(server->latency_ms, 99.0);
    out->max_ms = server->latency_ms.empty() ? 0.0
                                             : *std::max_element(server->latency_ms.begin(), server->latency_ms.end());
    const double span = server->any ? std::chrono::duration<double>(server->t_last - server->t_first).count() : 0.0;
    out->requests_per_s = span > 0 ? server->completed / span : 0.0;
    out->viewpoints_per_s = span > 0 ? server->vp_done / span : 0.0;
    out->mem_in_use = server->used;
    out->mem_peak = server->peak_used;
    out->mem_budget = server->opts.mem_budget_bytes;
    return VCM_OK;
}

vcm_status vcm_server_reset_stats(vcm_server *server) {
    clear_error();
    if (!server) return set_error(VCM_E_INVALID, "null server");
    std::lock_guard<std::mutex> lock(server->m);
    server->latency_ms.clear();
    server->completed = server->failed = server->rejected = server->launches = server->vp_done = 0;
    server->peak_used = server->used;
    server->any = false;
    return VCM_OK;
}

vcm_status vcm_server_destroy(vcm_server *server) {
    clear_error();
    if (!server) return VCM_OK;
    {
        std::lock_guard<std::mutex> lock(server->m);
        server->stop = true;
        server->cv.notify_all();
    }
    if (server->engine.joinable()) server->engine.join();
    DeviceGuard guard(server->device);
    for (auto &L : server->slots) {
        if (L.stream) hipStreamSynchronize(L.stream);
        if (L.stream) hipStreamDestroy(L.stream);
        if (L.done) hipEventDestroy(L.done);
    }
    delete server;
    return VCM_OK;
}

}  // extern "C"
