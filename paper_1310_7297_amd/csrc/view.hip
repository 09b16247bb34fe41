// Incremental processing (Sec. IV-C): the visibility of every viewpoint is
// computed once with the field of view at 360 degrees (the paper builds its
// colour tree and visible-region quad-tree that way), and a map for any gaze
// direction and field of view is then a re-masking and re-colouring of the
// stored gates, with no ray traced again.
//
// A view keeps one gate word per viewpoint (count | N << 10, in the field of
// view) in device memory.  Rendering takes the wedge of the new gaze:
// brute-force maps are coloured from the gates directly (the same device code
// as the ray kernel's, so a render equals vcm_compute of the query with that
// field of view bit for bit); pruned maps re-mask the gates and run the cell
// colouring.  A pruned map with a minimum block size above one viewpoint
// masks each viewpoint by its own position, where vcm_compute would give a
// smallest block that straddles the wedge its representative's gate.
#include <chrono>
#include <cmath>
#include <string>

#include "trace_common.h"

namespace vcm {
namespace {

struct RenderArgs {
    TargetDesc tgt;
    GridDesc grid;
    ParamDesc prm;           // the render's field of view
    const uint32_t *gate;    // the view's gates (field of view 360)
    uint32_t *regate;        // pruned: the re-masked gates; else null
    uint8_t *bin;
    float *c;
    uint16_t *count;
};

template <int DIM, typename R, int MODE>
__global__ __launch_bounds__(256) void k_render(RenderArgs A) {
    const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= A.grid.count) return;
    const int n0 = A.grid.n[0], n1 = A.grid.n[1];
    const int ii[3] = {static_cast<int>(v % n0), static_cast<int>((v / n0) % n1),
                       static_cast<int>(v / (static_cast<int64_t>(n0) * n1))};
    float q[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        q[k] = k < DIM ? A.grid.o[k] + static_cast<float>(2 * ii[k] + 1) * A.grid.h2[k] : 0.0f;
    const uint32_t w = A.gate[v];
    const bool fov = in_fov<DIM>(A.tgt, A.prm, q);
    const int n = static_cast<int>((w >> 10) & 1023u);
    const int cnt = fov ? static_cast<int>(w & 1023u) : 0;
    if (A.regate) {
        A.regate[v] = static_cast<uint32_t>(cnt) | (static_cast<uint32_t>(n) << 10) | (fov ? (1u << 20) : 0u);
        return;
    }
    R col;
    int bn;
    colour_and_bin<DIM, R, MODE>(A.tgt, A.prm, q, cnt, n, col, bn);
    A.bin[v] = static_cast<uint8_t>(bn);
    if (A.c) A.c[v] = static_cast<float>(col);
    if (A.count) A.count[v] = static_cast<uint16_t>(cnt);
}

}  // namespace
}  // namespace vcm

using namespace vcm;

struct vcm_view {
    const Index *ix = nullptr;
    vcm_query query{};      // as given, with the field of view of the gates at 360
    TargetDesc t{};
    GridDesc g{};
    ParamDesc p{};
    uint32_t *gate = nullptr;    // per viewpoint
    uint32_t *regate = nullptr;  // pruned methods: the gates of a render
    size_t bytes = 0;
    double create_ms = 0.0;
};

namespace {

void destroy_view(vcm_view *v) {
    if (!v) return;
    DeviceGuard guard(v->ix->device);
    if (v->gate) hipFree(v->gate);
    if (v->regate) hipFree(v->regate);
    delete v;
}

}  // namespace

extern "C" {

vcm_status vcm_view_create(const vcm_index *index, const vcm_query *query, void *stream, vcm_view **out) {
    clear_error();
    if (!index || !query || !out) return set_error(VCM_E_INVALID, "null argument");
    const auto t0 = std::chrono::steady_clock::now();
    const Index &ix = index->impl;
    vcm_view *v = new (std::nothrow) vcm_view;
    if (!v) return set_error(VCM_E_NOMEM, "host allocation failed");
    v->ix = &ix;
    v->query = *query;
    v->query.params.fov_deg = 360.0;
    v->query.params.gaze = 0;
    vcm_status st = prepare_query(ix, v->query, &v->t, &v->g, &v->p);
    if (st != VCM_OK) {
        delete v;
        return st;
    }
    if (v->g.count >= (int64_t(1) << 32)) {
        delete v;
        return set_error(VCM_E_INVALID, "views take grids of fewer than 2^32 viewpoints");
    }
    DeviceGuard guard(ix.device);
    hipStream_t s = (hipStream_t)stream;
    const int method = query->params.method, theta = query->params.theta_blocks;
    const size_t n = static_cast<size_t>(std::max<int64_t>(v->g.count, 1));
    const WsLayout w = query_workspace(v->g, ix.dim, method, theta, false);
    char *ws = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&v->gate), sizeof(uint32_t) * n) != hipSuccess ||
        (method != VCM_BRUTE && hipMalloc(reinterpret_cast<void **>(&v->regate), sizeof(uint32_t) * n) != hipSuccess) ||
        hipMalloc(reinterpret_cast<void **>(&ws), w.bytes) != hipSuccess) {
        if (ws) hipFree(ws);
        destroy_view(v);
        return set_error(VCM_E_NOMEM, "view allocation failed");
    }
    v->bytes = sizeof(uint32_t) * n * (method == VCM_BRUTE ? 1 : 2);
    if (v->g.count > 0) {
        if (method == VCM_BRUTE) {
            // the ray kernel's gate mode over blocks of one viewpoint
            st = launch_brute(ix, v->t, v->g, v->p, vcm_result{}, s, nullptr, v->gate, 1, Tuning{},
                              reinterpret_cast<unsigned *>(ws + w.counter));
        } else {
            uint32_t *lists[kMaxBlockLevels + 1] = {};
            for (int l = 1; l <= w.plan.levels; ++l) lists[l] = reinterpret_cast<uint32_t *>(ws + w.lists[l]);
            unsigned *ctr = reinterpret_cast<unsigned *>(ws + w.ctr);
            if (w.plan.leaf == 1) launch_gate_clear(v->gate, v->g.count, s);
            st = launch_blocks(ix, v->t, v->g, v->p, w.plan, v->gate, lists, ctr, s, nullptr);
            if (st == VCM_OK)
                st = launch_undecided(ix, v->t, v->g, v->p, w.plan, v->gate, lists, ctr,
                                      reinterpret_cast<unsigned *>(ws + w.counter), s, nullptr);
        }
    }
    const hipError_t e = hipStreamSynchronize(s);
    hipFree(ws);
    if (st == VCM_OK && e != hipSuccess) st = set_error(VCM_E_DEVICE, std::string("view: ") + hipGetErrorString(e));
    if (st != VCM_OK) {
        destroy_view(v);
        return st;
    }
    v->create_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = v;
    return VCM_OK;
}

vcm_status vcm_view_render(vcm_view *view, double fov_deg, int32_t gaze, const vcm_result *result, void *stream) {
    clear_error();
    if (!view || !result) return set_error(VCM_E_INVALID, "null argument");
    if (!result->bin) return set_error(VCM_E_INVALID, "result->bin is required");
    if (result->host) return set_error(VCM_E_INVALID, "views render into device result buffers");
    vcm_query q = view->query;
    q.params.fov_deg = fov_deg;
    q.params.gaze = gaze;
    TargetDesc t;
    GridDesc g;
    ParamDesc p;
    vcm_status st = prepare_query(*view->ix, q, &t, &g, &p);
    if (st != VCM_OK) return st;
    if (g.count <= 0) return VCM_OK;
    DeviceGuard guard(view->ix->device);
    hipStream_t s = (hipStream_t)stream;
    RenderArgs a{};
    a.tgt = t;
    a.grid = g;
    a.prm = p;
    a.gate = view->gate;
    a.regate = view->regate;
    a.bin = result->bin;
    a.c = result->c;
    a.count = result->count;
    const dim3 grid(static_cast<unsigned>((g.count + 255) / 256));
    const bool fp64 = p.fp64 != 0;
    const int dim = view->ix->dim;
    auto go = [&](auto dimv, auto realv, auto modev) {
        constexpr int D = decltype(dimv)::value, M = decltype(modev)::value;
        using R = typename decltype(realv)::type;
        hipLaunchKernelGGL((k_render<D, R, M>), grid, dim3(256), 0, s, a);
    };
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    using F = std::integral_constant<int, VCM_FULL>;
    using X = std::integral_constant<int, VCM_FRACTION>;
    struct Fl { using type = float; };
    struct Db { using type = double; };
    if (dim == 2) {
        if (fp64) { if (p.mode == VCM_FULL) go(I2{}, Db{}, F{}); else go(I2{}, Db{}, X{}); }
        else { if (p.mode == VCM_FULL) go(I2{}, Fl{}, F{}); else go(I2{}, Fl{}, X{}); }
    } else {
        if (fp64) { if (p.mode == VCM_FULL) go(I3{}, Db{}, F{}); else go(I3{}, Db{}, X{}); }
        else { if (p.mode == VCM_FULL) go(I3{}, Fl{}, F{}); else go(I3{}, Fl{}, X{}); }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(VCM_E_DEVICE, std::string("render launch: ") + hipGetErrorString(e));
    if (view->regate)
        return launch_pruned(*view->ix, t, g, p, q.params.method, view->regate, *result, s, nullptr, nullptr);
    return VCM_OK;
}

vcm_status vcm_view_get_info(const vcm_view *view, vcm_view_info *info) {
    clear_error();
    if (!view || !info) return set_error(VCM_E_INVALID, "null argument");
    info->viewpoints = static_cast<uint64_t>(std::max<int64_t>(view->g.count, 0));
    info->device_bytes = view->bytes;
    info->create_ms = view->create_ms;
    return VCM_OK;
}

vcm_status vcm_view_destroy(vcm_view *view) {
    clear_error();
    if (!view) return VCM_OK;
    {
        DeviceGuard guard(view->ix->device);
        hipDeviceSynchronize();
    }
    destroy_view(view);
    return VCM_OK;
}

}  // extern "C"
