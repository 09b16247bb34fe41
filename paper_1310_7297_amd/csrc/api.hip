// C-ABI entry points: argument validation, ownership, launches.
#include <chrono>
#include <cmath>
#include <mutex>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>
#include <algorithm>

#include "vcm_internal.h"

namespace vcm {

static thread_local std::string g_err;

vcm_status set_error(vcm_status st, const std::string &msg) {
    g_err = msg;
    return st;
}
void clear_error() { g_err.clear(); }

namespace {

constexpr double kLimit = 16384.0;  // |coordinate| < 2^14

bool dyadic(double x) {
    const double y = x * 256.0;
    return std::isfinite(y) && std::fabs(x) < kLimit && y == std::floor(y);
}

double deg2rad(double d) { return d * M_PI / 180.0; }

// Does the closed box of the target (centre c, half extents half) meet a
// closed obstacle box?  The target is not an obstacle, so an obstacle that
// touches or enters it makes the query ill-posed (Def. 2.1 separates the
// target from the obstacle set).  Scans the host copy of the columns the
// target's footprint overlaps.
bool target_meets_obstacle(const Index &ix, const double *c, const double *half) {
    if (ix.h_col_start.empty()) return false;
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = c[k] - half[k] - ix.frame[k];
        hi[k] = c[k] + half[k] - ix.frame[k];
    }
    const double cs = ix.dev.cs;
    auto col = [&](double x, int n) {
        return static_cast<int>(std::max(0.0, std::min(double(n - 1), std::floor(x / cs))));
    };
    const int x0 = col(lo[0], ix.dev.nx), x1 = col(hi[0], ix.dev.nx);
    const int y0 = col(lo[1], ix.dev.ny), y1 = col(hi[1], ix.dev.ny);
    for (int y = y0; y <= y1; ++y)
        for (int x = x0; x <= x1; ++x) {
            const int cidx = x + ix.dev.nx * y;
            for (int32_t r = ix.h_col_start[cidx]; r < ix.h_col_start[cidx + 1]; ++r) {
                const BoxRec &b = ix.h_recs[r];
                if (b.id < 0) continue;  // the sentinel
                bool meet = true;
                for (int k = 0; k < ix.dim; ++k) meet = meet && b.lo[k] <= hi[k] && b.hi[k] >= lo[k];
                if (meet) return true;
            }
        }
    return false;
}

}  // namespace

vcm_status prepare_query(const Index &ix, const vcm_query &q, TargetDesc *t, GridDesc *g,
                         ParamDesc *p) {
    const vcm_target &T = q.target;
    const vcm_grid &G = q.grid;
    const vcm_params &P = q.params;
    const int dim = ix.dim;
    // ---- target
    if (T.kind != VCM_SEGMENT && T.kind != VCM_BILLBOARD && T.kind != VCM_CUBE && T.kind != VCM_VIEWER)
        return set_error(VCM_E_INVALID, "unknown target kind");
    if (T.kind != VCM_VIEWER && (T.kind == VCM_SEGMENT) != (dim == 2))
        return set_error(VCM_E_INVALID, "segment targets need a 2-D index, billboards and cubes a 3-D index");
    if (T.kind == VCM_VIEWER && (T.samples_u != 1 || T.samples_v != 1))
        return set_error(VCM_E_INVALID, "a viewer has samples_u = samples_v = 1");
    if (T.kind == VCM_VIEWER && dim == 2 && T.center[2] != 0.0)
        return set_error(VCM_E_INVALID, "a 2-D viewer has center[2] = 0");
    if (T.samples_u < 1 || T.samples_u > 64 || T.samples_v < 1 || T.samples_v > 64)
        return set_error(VCM_E_INVALID, "samples_u and samples_v must be in [1, 64]");
    if (T.kind == VCM_SEGMENT && T.samples_v != 1)
        return set_error(VCM_E_INVALID, "a segment has samples_v == 1");
    if (T.kind != VCM_CUBE && T.normal_axis != 0 && T.normal_axis != 1)
        return set_error(VCM_E_INVALID, "normal_axis must be 0 or 1");
    if (T.normal_sign != 1 && T.normal_sign != -1)
        return set_error(VCM_E_INVALID, "normal_sign must be +1 or -1");
    const int per_facet = T.samples_u * T.samples_v;
    const int max_live = per_facet * (T.kind == VCM_CUBE ? 3 : 1);
    if (max_live > kMaxSamples)
        return set_error(VCM_E_INVALID, "at most 384 live samples per viewpoint");
    if (!(T.size[0] > 0) || (T.kind == VCM_BILLBOARD && !(T.size[1] > 0)))
        return set_error(VCM_E_INVALID, "target sizes must be positive");
    for (int k = 0; k < dim; ++k)
        if (!dyadic(T.center[k])) return set_error(VCM_E_INVALID, "target centre off the 2^-8 lattice");
    double half[3] = {0, 0, 0};
    double su_len = T.size[0], sv_len = 0;
    if (T.kind == VCM_VIEWER) {
        su_len = 0;  // a point: one sample at the centre
        if (!dyadic(T.size[0])) return set_error(VCM_E_INVALID, "a viewer's d_max (size[0]) must be on the 2^-8 lattice");
    } else if (T.kind == VCM_CUBE) {
        half[0] = half[1] = half[2] = T.size[0] / 2;
        sv_len = T.size[0];
    } else {
        half[1 - T.normal_axis] = T.size[0] / 2;
        if (T.kind == VCM_BILLBOARD) {
            half[2] = T.size[1] / 2;
            sv_len = T.size[1];
        }
    }
    const double hu = su_len / (2.0 * T.samples_u);
    const double hv = T.kind == VCM_SEGMENT ? 0.0 : sv_len / (2.0 * T.samples_v);
    for (int k = 0; k < 3; ++k)
        if (!dyadic(T.center[k] - half[k]) || !dyadic(T.center[k] + half[k]))
            return set_error(VCM_E_INVALID, "target extent off the 2^-8 lattice");
    for (int i = 0; i < T.samples_u; ++i)
        if (!dyadic((2 * i + 1 - T.samples_u) * hu) || !dyadic(T.center[0] + (2 * i + 1 - T.samples_u) * hu) ||
            !dyadic(T.center[1] + (2 * i + 1 - T.samples_u) * hu))
            return set_error(VCM_E_INVALID, "sample lattice off the 2^-8 lattice (size / samples_u)");
    for (int i = 0; i < T.samples_v; ++i)
        if (!dyadic((2 * i + 1 - T.samples_v) * hv) || !dyadic(T.center[2] + (2 * i + 1 - T.samples_v) * hv) ||
            !dyadic(T.center[1] + (2 * i + 1 - T.samples_v) * hv))
            return set_error(VCM_E_INVALID, "sample lattice off the 2^-8 lattice (size / samples_v)");
    const double mu_p = deg2rad(P.mu_arcmin / 60.0);
    // a viewer's S: the size whose visual angle at d_max is mu (Sec. IV-B)
    const double S = T.kind == VCM_BILLBOARD ? std::max(T.size[0], T.size[1])
                     : T.kind == VCM_VIEWER  ? 2.0 * T.size[0] * std::tan(mu_p / 2.0)
                                             : T.size[0];
    if (target_meets_obstacle(ix, T.center, half))
        return set_error(VCM_E_INVALID, "the target's box meets an obstacle");
    // ---- grid
    int64_t count = 1;
    for (int k = 0; k < 3; ++k) {
        if (G.n[k] < 1) return set_error(VCM_E_INVALID, "grid dimensions must be >= 1");
        count *= G.n[k];
    }
    if (dim == 2 && G.n[2] != 1) return set_error(VCM_E_INVALID, "2-D grids have n[2] == 1");
    if (G.n[1] > 65535) return set_error(VCM_E_INVALID, "grid n[1] must be <= 65535");
    double h2[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) {
        if (!(G.extent[k] >= 0)) return set_error(VCM_E_INVALID, "grid extent must be >= 0");
        h2[k] = G.extent[k] / (2.0 * G.n[k]);
        if (!dyadic(G.origin[k]) || !dyadic(h2[k]) || !dyadic(G.origin[k] + G.extent[k]))
            return set_error(VCM_E_INVALID,
                             "viewpoints off the 2^-8 lattice (origin, extent / (2 n)) or beyond 2^14");
    }
    if (count >= (int64_t(1) << 40)) return set_error(VCM_E_INVALID, "grid too large");
    // ---- parameters
    if (!(P.mu_arcmin > 0)) return set_error(VCM_E_INVALID, "mu_arcmin must be > 0");
    if (!(P.near_d0 > 0)) return set_error(VCM_E_INVALID, "near_d0 must be > 0");
    if (!(P.fov_deg > 0 && P.fov_deg <= 360)) return set_error(VCM_E_INVALID, "fov_deg must be in (0, 360]");
    if (P.gaze < -dim || P.gaze > dim) return set_error(VCM_E_INVALID, "gaze must be 0 or +-(1 + axis), axis < dim");
    if (T.kind == VCM_CUBE && P.fov_deg < 360 && P.gaze == 0)
        return set_error(VCM_E_INVALID, "a cube has no normal: give a gaze, or use fov_deg = 360");
    if (P.n_bins < 2 || P.n_bins > 256) return set_error(VCM_E_INVALID, "n_bins must be in [2, 256]");
    if (P.bin_scale != VCM_BIN_LINEAR && P.bin_scale != VCM_BIN_LOG)
        return set_error(VCM_E_INVALID, "unknown bin_scale");
    if (P.mode != VCM_FULL && P.mode != VCM_FRACTION) return set_error(VCM_E_INVALID, "unknown mode");
    if (P.method < VCM_BRUTE || P.method > VCM_PRUNED_T)
        return set_error(VCM_E_INVALID, "unknown method");
    if (P.theta_blocks < 1 || P.theta_blocks > 4096)
        return set_error(VCM_E_INVALID, "theta_blocks must be in [1, 4096]");
    // The float32 slab gap carries at most 3.5 * 2^-23 of rounding error (the
    // reciprocal within 1 ulp, one rounding per product and one for the
    // difference, on parameters in [0, 1]); a smaller margin would let
    // float32 decide rays it cannot decide exactly.
    if (!(P.recheck_eps >= kMinRecheckEps))
        return set_error(VCM_E_INVALID, "recheck_eps must be at least 2^-21 (float32 error bound) or +inf");
    if (P.precision != VCM_FP32_RECHECK && P.precision != VCM_FP64)
        return set_error(VCM_E_INVALID, "unknown precision");
    const double mu = deg2rad(P.mu_arcmin / 60.0);
    const double V0 = 2.0 * std::atan(S / (2.0 * P.near_d0));
    if (!(V0 > mu)) return set_error(VCM_E_INVALID, "target below the angular resolution at the near point");

    *t = TargetDesc{};
    t->kind = T.kind;
    t->nax = T.kind == VCM_CUBE ? 0 : T.normal_axis;
    t->nsign = T.normal_sign;
    t->su = T.samples_u;
    t->sv = T.samples_v;
    t->per_facet = per_facet;
    t->m_pf = (uint64_t)((0x100000000ull + per_facet - 1) / per_facet);
    t->m_su = (uint64_t)((0x100000000ull + T.samples_u - 1) / T.samples_u);
    // kernels work in the index frame (exact translation)
    for (int k = 0; k < 3; ++k) {
        t->c[k] = (k < dim) ? (float)(T.center[k] - ix.frame[k]) : 0.0f;
        t->half[k] = (float)half[k];
    }
    t->hu = (float)hu;
    t->hv = (float)hv;
    t->S = (float)S;
    t->rmax = T.kind == VCM_VIEWER ? (float)T.size[0] : 0.0f;

    *g = GridDesc{};
    for (int k = 0; k < 3; ++k) {
        g->o[k] = (k < dim) ? (float)(G.origin[k] - ix.frame[k]) : 0.0f;
        g->h2[k] = (float)h2[k];
        g->n[k] = G.n[k];
    }
    g->count = count;

    *p = ParamDesc{};
    p->region_r2 = T.kind == VCM_VIEWER ? double(t->rmax) * double(t->rmax) : HUGE_VAL;
    p->fov_axis = P.gaze == 0 ? T.normal_axis : std::abs(P.gaze) - 1;
    p->fov_sign = P.gaze == 0 ? T.normal_sign : (P.gaze > 0 ? 1 : -1);
    const double half_fov = P.fov_deg / 2.0;
    if (half_fov >= 180.0) {
        p->fov_kind = kFovAll;
    } else if (half_fov == 90.0) {
        p->fov_kind = kFovHalf;
    } else {
        p->fov_kind = half_fov < 90.0 ? kFovNarrow : kFovWide;
        // exact for these half angles: a viewpoint on the wedge's boundary is inside
        if (half_fov == 30.0 || half_fov == 150.0)
            p->fov_c2 = 0.75;
        else if (half_fov == 45.0 || half_fov == 135.0)
            p->fov_c2 = 0.5;
        else if (half_fov == 60.0 || half_fov == 120.0)
            p->fov_c2 = 0.25;
        else {
            const double cs = std::cos(deg2rad(half_fov));
            p->fov_c2 = cs * cs;
        }
    }
    p->n_bins = P.n_bins;
    p->bin_scale = P.bin_scale;
    p->mode = P.mode;
    p->d0 = (float)P.near_d0;
    p->V0 = (float)V0;
    p->inv_V0 = (float)(1.0 / V0);
    p->mu = (float)mu;
    p->mu_d = mu;
    p->d0_d = P.near_d0;
    p->inv_log_V0_mu = (float)(1.0 / std::log(V0 / mu));
    p->eps = (float)P.recheck_eps;  // +inf stays +inf: every test goes to the exact predicate
    p->eps_ref = 0x1p-20f;
    p->fp64 = P.precision == VCM_FP64 ? 1 : 0;

    return VCM_OK;
}

namespace {

constexpr size_t kWsAlign = 256;
size_t ws_align(size_t x) { return (x + kWsAlign - 1) / kWsAlign * kWsAlign; }

}  // namespace

// Workspace layout: the work-item range counters of the ray kernel; for the
// pruned methods, one gate word per viewpoint, the block lists of the
// visible-region tree, their counters and, with sums, the colouring's
// partial sums.
WsLayout query_workspace(const GridDesc &g, int dim, int method, int theta, bool sums) {
    WsLayout w;
    w.counter = 0;
    size_t off = ws_align(kCounterBytes);
    if (method != VCM_BRUTE && g.count > 0) {
        w.plan = block_plan(g, dim, theta);
        w.gate = off;
        off += ws_align(sizeof(uint32_t) * static_cast<size_t>(g.count));
        // the block lists launch_blocks reads and writes: the inputs of the
        // classified levels below the root, and (theta > 1) the undecided
        // smallest blocks
        for (int l = 1; l <= w.plan.levels; ++l) {
            if (!(l < w.plan.classified || (w.plan.leaf > 1 && l == w.plan.leaf_list))) continue;
            w.lists[l] = off;
            off += ws_align(sizeof(uint32_t) * static_cast<size_t>(w.plan.count[std::min(l, w.plan.levels - 1)]));
        }
        w.ctr = off;
        off += ws_align(sizeof(unsigned) * 2 * (w.plan.levels + 1));
        if (sums) {
            w.sums = off;
            w.n_sums = pruned_sum_blocks(g);
            off += ws_align(sizeof(double) * kPrunedSums * static_cast<size_t>(w.n_sums));
        }
    }
    w.bytes = off;
    return w;
}

vcm_status run_query(const Index &ix, const TargetDesc &t, const GridDesc &g, const ParamDesc &p,
                     int method, int theta, const vcm_result &r, hipStream_t s, DevStats *stats,
                     char *ws, bool sums) {
    const Tuning tune{};
    const WsLayout w = query_workspace(g, ix.dim, method, theta, sums);
    unsigned *counter = reinterpret_cast<unsigned *>(ws + w.counter);
    if (method == VCM_BRUTE) return launch_brute(ix, t, g, p, r, s, stats, nullptr, 1, tune, counter);
    if (g.count <= 0) return VCM_OK;
    if (g.count >= (int64_t(1) << 32))
        return set_error(VCM_E_INVALID, "pruned methods take grids of fewer than 2^32 viewpoints");
    // pruned: the visible-region blocks, the viewpoints (or, theta > 1, the
    // representatives of the smallest blocks) they leave undecided, then the
    // cell colours of every viewpoint
    uint32_t *gate = reinterpret_cast<uint32_t *>(ws + w.gate);
    uint32_t *lists[kMaxBlockLevels + 1] = {};
    for (int l = 1; l <= w.plan.levels; ++l) lists[l] = reinterpret_cast<uint32_t *>(ws + w.lists[l]);
    unsigned *ctr = reinterpret_cast<unsigned *>(ws + w.ctr);
    if (w.plan.leaf == 1) launch_gate_clear(gate, g.count, s);
    vcm_status st = launch_blocks(ix, t, g, p, w.plan, gate, lists, ctr, s, stats);
    if (st == VCM_OK) st = launch_undecided(ix, t, g, p, w.plan, gate, lists, ctr, counter, s, stats);
    if (st == VCM_OK)
        st = launch_pruned(ix, t, g, p, method, gate, r, s, stats ? &stats->t_fallbacks : nullptr,
                           w.n_sums ? reinterpret_cast<double *>(ws + w.sums) : nullptr);
    return st;
}

// ------------------------------------------------ allocation-free scratch ---

// Scratch memory of vcm_compute_noalloc: one copy per device, held until the
// process ends.  Host code must not use this name as a device address (it is
// a host-side stand-in there); scratch_address() gives the device's own
// address, taken once per device.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
char *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// Device address of `scratch` on `device`, which must be current.
vcm_status scratch_address(int device, char **out) {
    if (device < 0 || device >= kMaxDevices) return set_error(VCM_E_INVALID, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return set_error(VCM_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = static_cast<char *>(ptr);
    }
    *out = g_scratch_ptr[device];
    return VCM_OK;
}

}  // namespace vcm

using namespace vcm;

#define TRY_HIP(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return set_error(e_ == hipErrorOutOfMemory ? VCM_E_NOMEM : VCM_E_DEVICE,      \
                             std::string(#expr) + ": " + hipGetErrorString(e_));          \
    } while (0)

extern "C" {

const char *vcm_last_error(void) { return g_err.c_str(); }

const char *vcm_version(void) { return "vcm-mi355x 0.1 (gfx950)"; }

vcm_status vcm_build_index(const vcm_obstacles *obs, const vcm_index_opts *opts, vcm_index **out) {
    clear_error();
    if (!obs || !out) return set_error(VCM_E_INVALID, "null argument");
    if (obs->dim != 2 && obs->dim != 3) return set_error(VCM_E_INVALID, "dim must be 2 or 3");
    if (obs->n < 0) return set_error(VCM_E_INVALID, "negative box count");
    if (obs->n >= (int64_t(1) << 26)) return set_error(VCM_E_INVALID, "too many boxes");
    const int64_t n = obs->n;
    for (int k = 0; k < obs->dim; ++k)
        if (n > 0 && (!obs->lo[k] || !obs->hi[k])) return set_error(VCM_E_INVALID, "null box array");
    std::vector<float> lo(3 * std::max<int64_t>(n, 1), 0.0f), hi(3 * std::max<int64_t>(n, 1), 0.0f);
    for (int k = 0; k < obs->dim; ++k)
        for (int64_t i = 0; i < n; ++i) {
            const double a = obs->lo[k][i], b = obs->hi[k][i];
            if (!dyadic(a) || !dyadic(b))
                return set_error(VCM_E_INVALID, "box coordinate off the 2^-8 lattice or beyond 2^14 (box " +
                                                    std::to_string(i) + ")");
            if (a > b) return set_error(VCM_E_INVALID, "box with lo > hi (box " + std::to_string(i) + ")");
            lo[k * n + i] = (float)a;
            hi[k * n + i] = (float)b;
        }
    const int device = opts ? opts->device : 0;
    hipStream_t stream = opts ? (hipStream_t)opts->stream : nullptr;
    const double cs = opts ? opts->cell_size : 0.0;
    DeviceGuard guard(device);
    vcm_index *h = new (std::nothrow) vcm_index;
    if (!h) return set_error(VCM_E_NOMEM, "host allocation failed");
    h->impl.device = device;
    h->impl.dim = obs->dim;
    vcm_status st = build_index_device(&h->impl, lo.data(), hi.data(), n, cs, stream);
    if (st != VCM_OK) {
        if (h->impl.d_col_start) hipFree(h->impl.d_col_start);
        if (h->impl.d_recs) hipFree(h->impl.d_recs);
        delete h;
        return st;
    }
    *out = h;
    return VCM_OK;
}

vcm_status vcm_free_index(vcm_index *index) {
    clear_error();
    if (!index) return VCM_OK;
    DeviceGuard guard(index->impl.device);
    if (index->impl.d_col_start) hipFree(index->impl.d_col_start);
    if (index->impl.d_recs) hipFree(index->impl.d_recs);
    delete index;
    return VCM_OK;
}

vcm_status vcm_index_get_info(const vcm_index *index, vcm_index_info *info) {
    clear_error();
    if (!index || !info) return set_error(VCM_E_INVALID, "null argument");
    const Index &ix = index->impl;
    info->n_boxes = ix.n_boxes;
    info->n_refs = ix.n_refs;
    info->nx = ix.dev.nx;
    info->ny = ix.dev.ny;
    info->cell_size = ix.dev.cs;
    info->origin[0] = ix.frame[0];
    info->origin[1] = ix.frame[1];
    info->device_bytes = ix.bytes;
    info->build_ms = ix.build_ms;
    info->kernel_ms = ix.build_kernel_ms;
    info->longest_list = ix.longest_list;
    return VCM_OK;
}

vcm_status vcm_compute(const vcm_index *index, const vcm_query *query, const vcm_result *result,
                       void *stream, vcm_stats *stats) {
    clear_error();
    if (!index || !query || !result) return set_error(VCM_E_INVALID, "null argument");
    if (!result->bin) return set_error(VCM_E_INVALID, "result->bin is required");
    if (result->host != 0 && result->host != 1) return set_error(VCM_E_INVALID, "result->host must be 0 or 1");
    const Index &ix = index->impl;
    TargetDesc t;
    GridDesc g;
    ParamDesc p;
    vcm_status st = prepare_query(ix, *query, &t, &g, &p);
    if (st != VCM_OK) return st;
    DeviceGuard guard(ix.device);
    hipStream_t s = (hipStream_t)stream;
    const int method = query->params.method, theta = query->params.theta_blocks;
    const WsLayout w = query_workspace(g, ix.dim, method, theta, stats != nullptr);
    const size_t n = static_cast<size_t>(std::max<int64_t>(g.count, 0));

    // Host result buffers: the maps are computed into device buffers of the
    // call and copied back before it returns.
    vcm_result dev = *result;
    char *tmp = nullptr;
    if (result->host) {
        const size_t bytes = n * (1 + (result->c ? 4 : 0) + (result->count ? 2 : 0)) + 512;
        TRY_HIP(hipMallocAsync(reinterpret_cast<void **>(&tmp), bytes, s));
        size_t off = 0;
        dev.c = result->c ? reinterpret_cast<float *>(tmp + off) : nullptr;
        off += result->c ? (n * 4 + 255) / 256 * 256 : 0;
        dev.count = result->count ? reinterpret_cast<uint16_t *>(tmp + off) : nullptr;
        off += result->count ? (n * 2 + 255) / 256 * 256 : 0;
        dev.bin = reinterpret_cast<uint8_t *>(tmp + off);
        dev.host = 0;
    }

    char *ws = nullptr;
    TRY_HIP(hipMallocAsync(reinterpret_cast<void **>(&ws), w.bytes, s));
    DevStats *d_stats = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (stats) {
        TRY_HIP(hipMalloc(&d_stats, sizeof(DevStats)));
        TRY_HIP(hipEventCreate(&e0));
        TRY_HIP(hipEventCreate(&e1));
        TRY_HIP(hipMemsetAsync(d_stats, 0, sizeof(DevStats), s));
        TRY_HIP(hipEventRecord(e0, s));
    }
    st = run_query(ix, t, g, p, method, theta, dev, s, d_stats, ws, stats != nullptr);
    if (stats && st == VCM_OK) TRY_HIP(hipEventRecord(e1, s));
    std::vector<double> sums(static_cast<size_t>(w.n_sums) * kPrunedSums);
    DevStats h{};
    if (stats && st == VCM_OK) {
        TRY_HIP(hipMemcpyAsync(&h, d_stats, sizeof(DevStats), hipMemcpyDeviceToHost, s));
        if (!sums.empty())
            TRY_HIP(hipMemcpyAsync(sums.data(), ws + w.sums, sizeof(double) * sums.size(), hipMemcpyDeviceToHost, s));
    }
    if (result->host && st == VCM_OK) {
        TRY_HIP(hipMemcpyAsync(result->bin, dev.bin, n, hipMemcpyDeviceToHost, s));
        if (result->c) TRY_HIP(hipMemcpyAsync(result->c, dev.c, n * 4, hipMemcpyDeviceToHost, s));
        if (result->count) TRY_HIP(hipMemcpyAsync(result->count, dev.count, n * 2, hipMemcpyDeviceToHost, s));
    }
    hipFreeAsync(ws, s);
    if (tmp) hipFreeAsync(tmp, s);
    if (result->host || stats) {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess && st == VCM_OK)
            st = set_error(VCM_E_DEVICE, std::string("vcm_compute: ") + hipGetErrorString(e));
    }
    float ms = 0;
    if (e0 && e1 && st == VCM_OK) hipEventElapsedTime(&ms, e0, e1);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (d_stats) hipFree(d_stats);
    if (st != VCM_OK || !stats) return st;
    *stats = vcm_stats{};
    stats->viewpoints = (uint64_t)g.count;
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
    if (method != VCM_BRUTE) {
        // Sec. V-A error against the reference map, and the Sec. IV-A
        // comparison: the summed |V_approx - V_E| times the size each
        // viewpoint stands for, against the bound over the whole space (the
        // printed sums cover one meridian quadrant in 2-D, one half-space on
        // a side of the target plane in 3-D)
        double acc[kPrunedSums] = {0, 0, 0, 0};
        for (int64_t b = 0; b < w.n_sums; ++b)
            for (int k = 0; k < kPrunedSums; ++k) acc[k] += sums[static_cast<size_t>(b) * kPrunedSums + k];
        stats->err_signed = acc[2] > 0 ? acc[0] / acc[2] : 0.0;
        stats->err_abs = acc[2] > 0 ? acc[1] / acc[2] : 0.0;
        if (method != VCM_PRUNED_E) {
            double cell = 1.0;
            for (int k = 0; k < ix.dim; ++k) cell *= query->grid.extent[k] / query->grid.n[k];
            double bounds[2];
            error_bounds(t.S, p.mu_d, p.d0_d, ix.dim, bounds);
            const double copies = ix.dim == 2 ? 4.0 : 2.0;
            stats->bound = copies * bounds[method == VCM_PRUNED_M ? 0 : 1];
            stats->bound_measured = acc[3] * p.V0 * cell;
        }
    }
    return VCM_OK;
}

vcm_status vcm_compute_noalloc(const vcm_index *index, const vcm_query *query,
                               const vcm_result *result, void *stream) {
    clear_error();
    if (!index || !query || !result) return set_error(VCM_E_INVALID, "null argument");
    if (!result->bin) return set_error(VCM_E_INVALID, "result->bin is required");
    if (result->host) return set_error(VCM_E_INVALID, "vcm_compute_noalloc needs device result buffers");
    const Index &ix = index->impl;
    TargetDesc t;
    GridDesc g;
    ParamDesc p;
    vcm_status st = prepare_query(ix, *query, &t, &g, &p);
    if (st != VCM_OK) return st;
    const int method = query->params.method, theta = query->params.theta_blocks;
    const size_t need = query_workspace(g, ix.dim, method, theta, false).bytes;
    if (need > kScratchBytes)
        return set_error(VCM_E_INVALID, "vcm_compute_noalloc: the query needs " + std::to_string(need) +
                                            " bytes of scratch memory, more than the " +
                                            std::to_string(kScratchBytes) + " bytes it has");
    DeviceGuard guard(ix.device);
    char *ws = nullptr;
    st = scratch_address(ix.device, &ws);
    if (st != VCM_OK) return st;
    return run_query(ix, t, g, p, method, theta, *result, (hipStream_t)stream, nullptr, ws, false);
}

vcm_status vcm_map_error(const float *c_exact, const float *c_approx, int64_t n, int device,
                         void *stream, double out[2]) {
    clear_error();
    if (!out || n < 0 || (n > 0 && (!c_exact || !c_approx)))
        return set_error(VCM_E_INVALID, "invalid arguments");
    DeviceGuard guard(device);
    return map_error(c_exact, c_approx, n, (hipStream_t)stream, out);
}

vcm_status vcm_error_bounds(const vcm_query *query, int32_t dim, double out[2]) {
    clear_error();
    if (!query || !out || (dim != 2 && dim != 3)) return set_error(VCM_E_INVALID, "invalid arguments");
    const vcm_target &T = query->target;
    const double mu = query->params.mu_arcmin / 60.0 * M_PI / 180.0;
    const double S = T.kind == VCM_BILLBOARD ? std::max(T.size[0], T.size[1])
                     : T.kind == VCM_VIEWER  ? 2.0 * T.size[0] * std::tan(mu / 2.0)
                                             : T.size[0];
    const double d0 = query->params.near_d0;
    if (!(S > 0) || !(mu > 0) || !(d0 > 0) || !(2.0 * std::atan(S / (2.0 * d0)) > mu))
        return set_error(VCM_E_INVALID, "target size, mu and near point must be positive, V0 > mu");
    error_bounds(S, mu, d0, dim, out);
    return VCM_OK;
}

}  // extern "C"
