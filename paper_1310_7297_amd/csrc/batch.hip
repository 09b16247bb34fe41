// Batched VCM queries over one shared, device-resident obstacle index.
//
// The queries of a batch are grouped by the compile-time variant of the ray
// kernel they need (precision and mode); each group is one persistent launch
// over the work items of all its queries, so small and large maps share the
// machine instead of running one under-filled launch after another.  Pruned
// queries run their visible-region tree and colouring afterwards, one query
// after another (run_query).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "vcm_internal.h"

namespace vcm {

// ------------------------------------------------------------- staging ---

vcm_status Staging::acquire(size_t bytes, int device, int *slot, void **ptr) {
    std::lock_guard<std::mutex> lock(m_);
    bytes = std::max<size_t>(bytes, 4096);
    for (int pass = 0; pass < 2; ++pass) {
        for (size_t i = 0; i < slots_.size(); ++i) {
            Slot &s = slots_[i];
            if (s.device != device || s.busy) continue;
            if (s.pending) {
                // pass 0 takes only finished slots; pass 1 waits for one
                hipError_t q = pass == 0 ? hipEventQuery(s.ev) : hipEventSynchronize(s.ev);
                if (q == hipErrorNotReady) continue;
                if (q != hipSuccess)
                    return set_error(VCM_E_DEVICE, std::string("staging event: ") + hipGetErrorString(q));
                s.pending = false;
            }
            if (s.cap < bytes) {
                if (s.h) hipHostFree(s.h);
                s.h = nullptr;
                s.cap = 0;
                if (hipHostMalloc(&s.h, bytes, hipHostMallocDefault) != hipSuccess)
                    return set_error(VCM_E_NOMEM, "pinned staging allocation failed");
                s.cap = bytes;
            }
            s.busy = true;
            *slot = static_cast<int>(i);
            *ptr = s.h;
            return VCM_OK;
        }
        if (pass == 0 && slots_.size() < kMaxSlotsStaging) {
            Slot s;
            s.device = device;
            if (hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess)
                return set_error(VCM_E_DEVICE, "staging event creation failed");
            if (hipHostMalloc(&s.h, bytes, hipHostMallocDefault) != hipSuccess) {
                hipEventDestroy(s.ev);
                return set_error(VCM_E_NOMEM, "pinned staging allocation failed");
            }
            s.cap = bytes;
            s.busy = true;
            slots_.push_back(s);
            *slot = static_cast<int>(slots_.size() - 1);
            *ptr = s.h;
            return VCM_OK;
        }
    }
    return set_error(VCM_E_AGAIN, "no staging buffer free");
}

vcm_status Staging::release(int slot, hipStream_t s) {
    std::lock_guard<std::mutex> lock(m_);
    Slot &x = slots_[slot];
    x.busy = false;
    const hipError_t e = hipEventRecord(x.ev, s);
    if (e != hipSuccess) {
        // the copy may not have been enqueued: wait for the device instead
        hipStreamSynchronize(s);
        x.pending = false;
        return set_error(VCM_E_DEVICE, std::string("staging event: ") + hipGetErrorString(e));
    }
    x.pending = true;
    return VCM_OK;
}

Staging &staging() {
    // Pinned buffers are kept for the life of the process.
    static Staging *s = new Staging;
    return *s;
}

vcm_status upload(const void *src, size_t bytes, void *dst, int device, hipStream_t s) {
    if (bytes == 0) return VCM_OK;
    int slot = -1;
    void *h = nullptr;
    vcm_status st = staging().acquire(bytes, device, &slot, &h);
    if (st != VCM_OK) return st;
    std::memcpy(h, src, bytes);
    const hipError_t e = hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, s);
    st = staging().release(slot, s);
    if (e != hipSuccess) return set_error(VCM_E_DEVICE, std::string("upload: ") + hipGetErrorString(e));
    return st;
}

// ---------------------------------------------------------------- plans ---

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Work items of one brute-force query at a given chunk.
uint64_t query_items(const PlanQuery &q, int chunk) {
    const uint64_t cpr = (static_cast<uint64_t>(q.g.n[0]) + chunk - 1) / chunk;
    return cpr * static_cast<uint64_t>(q.g.n[1]) * static_cast<uint64_t>(q.g.n[2]);
}

}  // namespace

vcm_status BatchPlan::prepare(const Index &index, const vcm_query *qs, int nq, const vcm_result *rs) {
    ix = &index;
    q.clear();
    viewpoints = 0;
    for (int i = 0; i < nq; ++i) {
        PlanQuery pq{};
        if (!rs[i].bin) return set_error(VCM_E_INVALID, "result " + std::to_string(i) + ": bin is required");
        if (rs[i].host)
            return set_error(VCM_E_INVALID, "result " + std::to_string(i) + ": batches need device result buffers");
        vcm_status st = prepare_query(index, qs[i], &pq.t, &pq.g, &pq.p);
        if (st != VCM_OK) return set_error(st, "query " + std::to_string(i) + ": " + vcm_last_error());
        pq.method = qs[i].params.method;
        pq.theta = qs[i].params.theta_blocks;
        pq.r = rs[i];
        pq.ns = slots_for(pq.t);
        if (pq.ns < 1 || pq.ns > kMaxSlots)
            return set_error(VCM_E_INVALID, "query " + std::to_string(i) + ": too many target samples");
        if (pq.g.count >= (int64_t(1) << 31))
            return set_error(VCM_E_INVALID, "query " + std::to_string(i) + ": grid too large for a batch");
        viewpoints += static_cast<uint64_t>(pq.g.count);
        q.push_back(pq);
    }
    return VCM_OK;
}

void BatchPlan::layout() {
    groups.clear();
    items = 0;
    const uint64_t kMaxItems = uint64_t(1) << 31;
    for (size_t i = 0; i < q.size(); ++i) {
        const PlanQuery &pq = q[i];
        if (pq.g.count <= 0 || pq.method != VCM_BRUTE) continue;
        const uint64_t wi = query_items(pq, chunk_for(tune, pq.p.mode));
        const uint64_t it = (wi + 3) / 4;  // groups of four work items (one workgroup claim)
        PlanGroup *g = nullptr;
        for (auto &x : groups)
            if (x.fp64 == (pq.p.fp64 != 0) && x.mode == pq.p.mode && x.n_items + it < kMaxItems) g = &x;
        if (!g) {
            groups.push_back(PlanGroup{});
            g = &groups.back();
            g->fp64 = pq.p.fp64 != 0;
            g->mode = pq.p.mode;
        }
        g->members.push_back(static_cast<int>(i));
        g->ns = std::max(g->ns, pq.ns);
        g->n_items += static_cast<uint32_t>(it);
        items += wi;
    }
    size_t off = 0;
    for (auto &g : groups) {
        g.rec_off = off;
        off = align_up(off + sizeof(BruteArgs) * g.members.size());
        g.end_off = off;
        off = align_up(off + sizeof(uint32_t) * g.members.size());
        g.ctr_off = off;
        off = align_up(off + kCounterBytes);
    }
    image_bytes = off;
    for (auto &pq : q) {
        pq.ws_off = off;
        if (pq.method != VCM_BRUTE && pq.g.count > 0)
            off = align_up(off + query_workspace(pq.g, ix->dim, pq.method, pq.theta, false).bytes);
    }
    bytes = std::max<size_t>(off, kAlign);
}

void BatchPlan::image(std::vector<char> &img) const {
    img.assign(image_bytes, 0);
    for (const auto &g : groups) {
        BruteArgs *recs = reinterpret_cast<BruteArgs *>(img.data() + g.rec_off);
        uint32_t *ends = reinterpret_cast<uint32_t *>(img.data() + g.end_off);
        uint32_t acc = 0;
        for (size_t m = 0; m < g.members.size(); ++m) {
            const PlanQuery &pq = q[g.members[m]];
            const int chunk = chunk_for(tune, pq.p.mode);
            recs[m] = make_brute_args(*ix, pq.t, pq.g, pq.p, pq.r, nullptr, 1, chunk);
            acc += static_cast<uint32_t>((query_items(pq, chunk) + 3) / 4);
            ends[m] = acc;
        }
    }
}

vcm_status BatchPlan::enqueue(hipStream_t s, DevStats *stats) const {
    const int cus = device_cus(ix->device);
    for (const auto &g : groups) {
        BatchArgs b{};
        b.counter = reinterpret_cast<unsigned *>(d_base + g.ctr_off);
        b.stats = stats;
        b.nq = static_cast<int32_t>(g.members.size());
        b.n_items = g.n_items;
        const int64_t blocks = std::min<int64_t>(int64_t(g.n_items), int64_t(cus) * tune.blocks_per_cu);
        vcm_status st = launch_brute_batch(*ix, g.fp64, g.mode, g.ns, b,
                                           reinterpret_cast<const BruteArgs *>(d_base + g.rec_off),
                                           reinterpret_cast<const uint32_t *>(d_base + g.end_off),
                                           static_cast<int>(std::max<int64_t>(blocks, 1)), s);
        if (st != VCM_OK) return st;
    }
    // pruned queries: their own visible-region tree and colouring, in order
    for (const auto &pq : q) {
        if (pq.method == VCM_BRUTE || pq.g.count <= 0) continue;
        vcm_status st = run_query(*ix, pq.t, pq.g, pq.p, pq.method, pq.theta, pq.r, s, stats, d_base + pq.ws_off,
                                  false);
        if (st != VCM_OK) return st;
    }
    return VCM_OK;
}

}  // namespace vcm

using namespace vcm;

struct vcm_batch {
    BatchPlan plan;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double tune_ms = 0.0;
};

namespace {

void destroy_batch(vcm_batch *b) {
    if (!b) return;
    DeviceGuard guard(b->plan.device);
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    if (b->cap_stream) hipStreamDestroy(b->cap_stream);
    if (b->plan.d_base) hipFree(b->plan.d_base);
    delete b;
}

// Upload the plan's records synchronously (creation time only).
vcm_status upload_plan(BatchPlan &p) {
    std::vector<char> img;
    p.image(img);
    if (img.empty()) return VCM_OK;
    const hipError_t e = hipMemcpy(p.d_base, img.data(), img.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return set_error(VCM_E_DEVICE, std::string("upload: ") + hipGetErrorString(e));
    return VCM_OK;
}

// Time the plan at a launch shape: one warm-up and two timed runs, best kept.
vcm_status time_shape(BatchPlan &p, const Tuning &t, hipStream_t s, float *ms) {
    p.tune = t;
    p.layout();
    vcm_status st = upload_plan(p);
    if (st != VCM_OK) return st;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return set_error(VCM_E_DEVICE, "event creation failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return set_error(VCM_E_DEVICE, "event creation failed");
    }
    float best = 1e30f;
    for (int r = 0; r < 3 && st == VCM_OK; ++r) {
        hipEventRecord(e0, s);
        st = p.enqueue(s, nullptr);
        hipEventRecord(e1, s);
        if (hipStreamSynchronize(s) != hipSuccess) st = set_error(VCM_E_DEVICE, "autotune run failed");
        float x = 0.0f;
        if (st == VCM_OK && r > 0 && hipEventElapsedTime(&x, e0, e1) == hipSuccess) best = std::min(best, x);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *ms = best;
    return st;
}

// Pick the launch shape on a sample of the batch's queries (about 2^22
// viewpoints, spread over the batch), timing each candidate shape.
vcm_status autotune(vcm_batch *b, const vcm_query *qs, const vcm_result *rs, int nq) {
    const auto t0 = std::chrono::steady_clock::now();
    BatchPlan &p = b->plan;
    std::vector<int> pick;
    uint64_t vp = 0;
    const uint64_t want = uint64_t(1) << 22;
    const int stride = std::max<int>(1, static_cast<int>(p.viewpoints / std::max<uint64_t>(want, 1)));
    for (int off = 0; off < stride && vp < want; ++off)
        for (int i = off; i < nq && vp < want; i += stride) {
            pick.push_back(i);
            vp += static_cast<uint64_t>(std::max<int64_t>(p.q[i].g.count, 0));
        }
    std::vector<vcm_query> sq;
    std::vector<vcm_result> sr;
    for (int i : pick) {
        sq.push_back(qs[i]);
        sr.push_back(rs[i]);
    }
    BatchPlan sub;
    sub.device = p.device;
    vcm_status st = sub.prepare(*p.ix, sq.data(), static_cast<int>(sq.size()), sr.data());
    if (st != VCM_OK) return st;
    // the largest layout is the one with the smallest chunk
    Tuning widest;
    widest.chunk = 1;
    sub.tune = widest;
    sub.layout();
    if (hipMalloc(reinterpret_cast<void **>(&sub.d_base), sub.bytes) != hipSuccess)
        return set_error(VCM_E_NOMEM, "autotune allocation failed");
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        hipFree(sub.d_base);
        return set_error(VCM_E_DEVICE, "stream creation failed");
    }
    static const int kChunks[] = {4, 8, 16, 32, 64};
    static const int kBlocks[] = {4, 8};
    Tuning best = p.tune;
    float best_ms = 1e30f;
    for (int c : kChunks)
        for (int bpc : kBlocks) {
            Tuning t;
            t.chunk = c;
            t.blocks_per_cu = bpc;
            float ms = 0.0f;
            st = time_shape(sub, t, s, &ms);
            if (st != VCM_OK) break;
            if (ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
    hipStreamSynchronize(s);
    hipStreamDestroy(s);
    hipFree(sub.d_base);
    if (st != VCM_OK) return st;
    p.tune = best;
    b->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return VCM_OK;
}

vcm_status fill_stats(const DevStats &h, uint64_t viewpoints, float ms, vcm_stats *stats) {
    *stats = vcm_stats{};
    stats->viewpoints = viewpoints;
    stats->rays = h.rays;
    stats->box_tests = h.box_tests;
    stats->rechecks = h.rechecks;
    stats->fp32_disagree = h.fp32_disagree;
    stats->columns = h.columns;
    stats->slot_tests = h.slot_tests;
    stats->inside_box = h.inside_box;
    stats->t_fallbacks = h.t_fallbacks;
    stats->records = h.records;
    stats->narrow_tests = h.narrow_tests;
    stats->kernel_ms = ms;
    stats->blocks = h.blocks;
    stats->blocks_decided = h.blocks_decided;
    stats->leaves = h.leaves;
    return VCM_OK;
}

vcm_status check_batch_args(const vcm_index *index, const vcm_query *queries, int32_t nq,
                            const vcm_result *results) {
    if (!index) return set_error(VCM_E_INVALID, "null index");
    if (nq < 0) return set_error(VCM_E_INVALID, "negative query count");
    if (nq > 0 && (!queries || !results)) return set_error(VCM_E_INVALID, "null queries or results");
    return VCM_OK;
}

}  // namespace

extern "C" {

vcm_status vcm_compute_batch(const vcm_index *index, const vcm_query *queries, int32_t nq,
                             const vcm_result *results, void *stream, vcm_stats *stats) {
    clear_error();
    vcm_status st = check_batch_args(index, queries, nq, results);
    if (st != VCM_OK) return st;
    const Index &ix = index->impl;
    DeviceGuard guard(ix.device);
    hipStream_t s = (hipStream_t)stream;
    BatchPlan p;
    p.device = ix.device;
    st = p.prepare(ix, queries, nq, results);
    if (st != VCM_OK) return st;
    p.layout();
    if (p.groups.empty() && !stats) return VCM_OK;

    hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&p.d_base), p.bytes, s);
    if (e != hipSuccess) return set_error(VCM_E_NOMEM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
    std::vector<char> img;
    p.image(img);
    st = upload(img.data(), img.size(), p.d_base, ix.device, s);

    DevStats *d_stats = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == VCM_OK && stats) {
        if (hipMalloc(&d_stats, sizeof(DevStats)) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
            hipEventCreate(&e1) != hipSuccess || hipMemsetAsync(d_stats, 0, sizeof(DevStats), s) != hipSuccess ||
            hipEventRecord(e0, s) != hipSuccess)
            st = set_error(VCM_E_DEVICE, "statistics set-up failed");
    }
    if (st == VCM_OK) st = p.enqueue(s, d_stats);
    hipFreeAsync(p.d_base, s);
    if (!stats) return st;
    DevStats h{};
    float ms = 0.0f;
    if (d_stats) {
        if (e1) hipEventRecord(e1, s);
        hipMemcpyAsync(&h, d_stats, sizeof(DevStats), hipMemcpyDeviceToHost, s);
        if (hipStreamSynchronize(s) != hipSuccess && st == VCM_OK)
            st = set_error(VCM_E_DEVICE, "batch failed on the device");
        if (e0 && e1) hipEventElapsedTime(&ms, e0, e1);
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (d_stats) hipFree(d_stats);
    if (st != VCM_OK) return st;
    return fill_stats(h, p.viewpoints, ms, stats);
}

vcm_status vcm_batch_create(const vcm_index *index, const vcm_query *queries, int32_t nq,
                            const vcm_result *results, const vcm_batch_opts *opts, vcm_batch **out) {
    clear_error();
    vcm_status st = check_batch_args(index, queries, nq, results);
    if (st != VCM_OK) return st;
    if (!out) return set_error(VCM_E_INVALID, "null output");
    vcm_batch_opts o{};
    if (opts) o = *opts;
    if (o.chunk < 0 || o.chunk > 64) return set_error(VCM_E_INVALID, "chunk must be in 0..64");
    if (o.blocks_per_cu < 0 || o.blocks_per_cu > 16)
        return set_error(VCM_E_INVALID, "blocks_per_cu must be in 0..16");
    const Index &ix = index->impl;
    DeviceGuard guard(ix.device);
    vcm_batch *b = new (std::nothrow) vcm_batch;
    if (!b) return set_error(VCM_E_NOMEM, "host allocation failed");
    BatchPlan &p = b->plan;
    p.device = ix.device;
    st = p.prepare(ix, queries, nq, results);
    if (st == VCM_OK && o.autotune && p.viewpoints > 0) st = autotune(b, queries, results, nq);
    if (st == VCM_OK) {
        if (o.chunk) p.tune.chunk = o.chunk;
        if (o.blocks_per_cu) p.tune.blocks_per_cu = o.blocks_per_cu;
        p.layout();
        if (hipMalloc(reinterpret_cast<void **>(&p.d_base), p.bytes) != hipSuccess)
            st = set_error(VCM_E_NOMEM, "batch allocation failed");
    }
    if (st == VCM_OK) st = upload_plan(p);
    if (st == VCM_OK && o.use_graph) {
        device_cus(ix.device);  // query the device before capturing
        if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
            st = set_error(VCM_E_DEVICE, "stream creation failed");
        else if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            st = set_error(VCM_E_DEVICE, "graph capture failed to start");
        else {
            const vcm_status se = p.enqueue(b->cap_stream, nullptr);
            const hipError_t ee = hipStreamEndCapture(b->cap_stream, &b->graph);
            if (se != VCM_OK) st = se;
            else if (ee != hipSuccess) st = set_error(VCM_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(ee));
            else if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
                st = set_error(VCM_E_DEVICE, "graph instantiation failed");
        }
    }
    if (st != VCM_OK) {
        destroy_batch(b);
        return st;
    }
    *out = b;
    return VCM_OK;
}

vcm_status vcm_batch_run(vcm_batch *batch, void *stream) {
    clear_error();
    if (!batch) return set_error(VCM_E_INVALID, "null batch");
    DeviceGuard guard(batch->plan.device);
    hipStream_t s = (hipStream_t)stream;
    if (batch->exec) {
        const hipError_t e = hipGraphLaunch(batch->exec, s);
        if (e != hipSuccess) return set_error(VCM_E_DEVICE, std::string("graph launch: ") + hipGetErrorString(e));
        return VCM_OK;
    }
    return batch->plan.enqueue(s, nullptr);
}

vcm_status vcm_batch_get_info(const vcm_batch *batch, vcm_batch_info *info) {
    clear_error();
    if (!batch || !info) return set_error(VCM_E_INVALID, "null argument");
    const BatchPlan &p = batch->plan;
    info->chunk = p.tune.chunk;
    info->blocks_per_cu = p.tune.blocks_per_cu;
    info->launches = static_cast<int32_t>(p.groups.size());
    info->graph = batch->exec != nullptr;
    info->viewpoints = p.viewpoints;
    info->work_items = p.items;
    info->device_bytes = p.bytes;
    info->tune_ms = batch->tune_ms;
    return VCM_OK;
}

vcm_status vcm_batch_destroy(vcm_batch *batch) {
    clear_error();
    if (!batch) return VCM_OK;
    DeviceGuard guard(batch->plan.device);
    hipDeviceSynchronize();
    destroy_batch(batch);
    return VCM_OK;
}

}  // extern "C"
