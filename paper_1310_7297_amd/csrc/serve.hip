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
#include <chrono>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "serve_core.h"
#include "vcm_internal.h"

using namespace vcm;

namespace {

struct Payload {
    vcm_query query;
    vcm_result result;
};

// The device side of the engine: one stream and one completion event per
// launch slot; a launch is one batched persistent launch of its requests.
class HipExecutor final : public serve::Executor<Payload> {
public:
    const Index *ix = nullptr;
    int device = 0;
    Tuning tune;
    std::vector<hipStream_t> stream;
    std::vector<hipEvent_t> done;

    // The plan's buffer is allocated and freed in stream order.
    vcm_status start(int slot, const std::vector<const Payload *> &batch, std::string *msg) override {
        std::vector<vcm_query> qs;
        std::vector<vcm_result> rs;
        for (const Payload *p : batch) {
            qs.push_back(p->query);
            rs.push_back(p->result);
        }
        const hipStream_t s = stream[slot];
        BatchPlan p;
        p.device = device;
        p.tune = tune;
        vcm_status st = p.prepare(*ix, qs.data(), static_cast<int>(qs.size()), rs.data());
        if (st == VCM_OK) {
            p.layout();
            const hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&p.d_base), p.bytes, s);
            if (e != hipSuccess) st = set_error(VCM_E_NOMEM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
        }
        if (st == VCM_OK) {
            std::vector<char> img;
            p.image(img);
            st = upload(img.data(), img.size(), p.d_base, device, s);
            if (st == VCM_OK) st = p.enqueue(s, nullptr);
            hipFreeAsync(p.d_base, s);
        }
        if (st == VCM_OK && hipEventRecord(done[slot], s) != hipSuccess)
            st = set_error(VCM_E_DEVICE, "event record failed");
        if (st != VCM_OK) {
            *msg = vcm_last_error();
            hipStreamSynchronize(s);
        }
        return st;
    }

    vcm_status poll(int slot, std::string *msg) override {
        const hipError_t q = hipEventQuery(done[slot]);
        if (q == hipErrorNotReady) return VCM_E_PENDING;
        if (q == hipSuccess) return VCM_OK;
        *msg = std::string("launch failed: ") + hipGetErrorString(q);
        return VCM_E_DEVICE;
    }
};

// Device bytes a request holds while admitted: its result buffers, its work
// record and, for the pruned methods, the workspace of the block hierarchy
// (a gate word per viewpoint and the block lists of every level).
size_t footprint(const vcm_query &q, const vcm_result &r, const GridDesc &g, int dim) {
    const uint64_t n = static_cast<uint64_t>(g.count);
    size_t b = 0;
    if (r.bin) b += n;
    if (r.c) b += 4 * n;
    if (r.count) b += 2 * n;
    b += sizeof(BruteArgs) + 64;
    if (q.params.method != VCM_BRUTE)
        b += query_workspace(g, dim, q.params.method, std::max(1, q.params.theta_blocks), false).bytes;
    return b;
}

}  // namespace

struct vcm_server {
    const Index *ix = nullptr;
    vcm_server_opts opts{};
    HipExecutor ex;
    serve::Core<Payload> *core = nullptr;
    std::thread engine;
};

namespace {

void release_slots(vcm_server *s) {
    for (hipStream_t x : s->ex.stream)
        if (x) hipStreamDestroy(x);
    for (hipEvent_t x : s->ex.done)
        if (x) hipEventDestroy(x);
}

vcm_status finish_status(vcm_status st, const std::string &msg) {
    if (st == VCM_OK || st == VCM_E_PENDING) return st;
    return set_error(st, msg);
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
    s->opts = o;
    s->ex.ix = &ix;
    s->ex.device = ix.device;
    if (o.chunk) s->ex.tune.chunk = o.chunk;
    if (o.blocks_per_cu) s->ex.tune.blocks_per_cu = o.blocks_per_cu;
    device_cus(ix.device);
    s->ex.stream.assign(o.max_inflight, nullptr);
    s->ex.done.assign(o.max_inflight, nullptr);
    for (int i = 0; i < o.max_inflight; ++i) {
        if (hipStreamCreateWithFlags(&s->ex.stream[i], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s->ex.done[i], hipEventDisableTiming) != hipSuccess) {
            release_slots(s);
            delete s;
            return set_error(VCM_E_DEVICE, "stream or event creation failed");
        }
    }
    s->core = new (std::nothrow) serve::Core<Payload>(o.mem_budget_bytes, o.max_inflight, o.max_batch, &s->ex);
    if (!s->core) {
        release_slots(s);
        delete s;
        return set_error(VCM_E_NOMEM, "host allocation failed");
    }
    const int dev = ix.device;
    serve::Core<Payload> *core = s->core;
    s->engine = std::thread([dev, core] {
        hipSetDevice(dev);
        core->run();
    });
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
    std::string msg;
    st = server->core->submit(Payload{*query, *result}, footprint(*query, *result, g, server->ix->dim), n, ticket,
                              &msg);
    return finish_status(st, msg);
}

vcm_status vcm_poll(vcm_server *server, uint64_t ticket, vcm_request_info *info) {
    clear_error();
    if (!server) return set_error(VCM_E_INVALID, "null server");
    serve::RequestInfo ri;
    std::string msg;
    const vcm_status st = server->core->poll(ticket, &ri, &msg);
    if (info && st != VCM_E_PENDING && st != VCM_E_NOTFOUND) {
        info->latency_ms = ri.latency_ms;
        info->queue_ms = ri.queue_ms;
        info->viewpoints = ri.viewpoints;
    }
    return finish_status(st, msg);
}

vcm_status vcm_wait(vcm_server *server, uint64_t ticket, int32_t timeout_ms, vcm_request_info *info) {
    clear_error();
    if (!server) return set_error(VCM_E_INVALID, "null server");
    serve::RequestInfo ri;
    std::string msg;
    const vcm_status st = server->core->wait(ticket, timeout_ms, &ri, &msg);
    if (info && st != VCM_E_PENDING && st != VCM_E_NOTFOUND) {
        info->latency_ms = ri.latency_ms;
        info->queue_ms = ri.queue_ms;
        info->viewpoints = ri.viewpoints;
    }
    return finish_status(st, msg);
}

vcm_status vcm_server_drain(vcm_server *server) {
    clear_error();
    if (!server) return set_error(VCM_E_INVALID, "null server");
    server->core->drain();
    return VCM_OK;
}

vcm_status vcm_server_hold(vcm_server *server, int32_t hold) {
    clear_error();
    if (!server) return set_error(VCM_E_INVALID, "null server");
    server->core->hold(hold != 0);
    return VCM_OK;
}

vcm_status vcm_server_get_stats(vcm_server *server, vcm_server_stats *out) {
    clear_error();
    if (!server || !out) return set_error(VCM_E_INVALID, "null argument");
    const serve::Stats s = server->core->stats();
    out->completed = s.completed;
    out->failed = s.failed;
    out->rejected = s.rejected;
    out->launches = s.launches;
    out->viewpoints = s.viewpoints;
    out->p50_ms = s.p50_ms;
    out->p99_ms = s.p99_ms;
    out->max_ms = s.max_ms;
    out->requests_per_s = s.requests_per_s;
    out->viewpoints_per_s = s.viewpoints_per_s;
    out->mem_in_use = s.mem_in_use;
    out->mem_peak = s.mem_peak;
    out->mem_budget = s.mem_budget;
    return VCM_OK;
}

vcm_status vcm_server_reset_stats(vcm_server *server) {
    clear_error();
    if (!server) return set_error(VCM_E_INVALID, "null server");
    server->core->reset_stats();
    return VCM_OK;
}

vcm_status vcm_server_destroy(vcm_server *server) {
    clear_error();
    if (!server) return VCM_OK;
    server->core->stop();
    if (server->engine.joinable()) server->engine.join();
    {
        DeviceGuard guard(server->ex.device);
        for (hipStream_t x : server->ex.stream)
            if (x) hipStreamSynchronize(x);
        release_slots(server);
    }
    delete server->core;
    delete server;
    return VCM_OK;
}

}  // extern "C"
