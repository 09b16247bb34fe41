// Index autotuner: the column width of the obstacle index for a workload.
//
// The width trades the number of columns a corridor crosses against the
// number of boxes listed per column, and the best choice depends on the
// scene, the targets and the mode (a FULL-mode map stops at its first blocked
// ray, a FRACTION-mode map resolves every ray).  The tuner builds the index
// at every candidate width and times the workload itself on it.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "vcm_internal.h"

using namespace vcm;

namespace {
// Candidate column widths one tuning run may try (the size of the result arrays).
constexpr int kTuneMaxCandidates = 16;
}  // namespace

extern "C" {

vcm_status vcm_tune_cell_size(const vcm_obstacles *obstacles, const vcm_query *queries, int32_t nq,
                              const vcm_tune_opts *opts, vcm_tune_result *out) {
    clear_error();
    if (!obstacles || !queries || !out || nq < 1) return set_error(VCM_E_INVALID, "invalid arguments");
    vcm_tune_opts o{};
    if (opts) o = *opts;
    if (o.cell_min == 0) o.cell_min = 16.0;
    if (o.cell_max == 0) o.cell_max = 128.0;
    if (o.reps == 0) o.reps = 2;
    int e;
    if (std::frexp(o.cell_min, &e) != 0.5 || std::frexp(o.cell_max, &e) != 0.5 || o.cell_min > o.cell_max ||
        o.cell_min < 1.0 / 16 || o.cell_max > 4096)
        return set_error(VCM_E_INVALID, "cell_min and cell_max must be powers of two in [1/16, 4096]");
    if (o.reps < 1 || o.reps > 100) return set_error(VCM_E_INVALID, "reps must be in 1..100");
    const int n_cand = static_cast<int>(std::lround(std::log2(o.cell_max / o.cell_min))) + 1;
    if (n_cand > kTuneMaxCandidates) return set_error(VCM_E_INVALID, "too many candidate widths");

    DeviceGuard guard(o.device);
    // result buffers for every query, in one allocation
    size_t total = 0;
    std::vector<size_t> off(nq);
    for (int i = 0; i < nq; ++i) {
        const vcm_grid &g = queries[i].grid;
        int64_t n = 1;
        for (int k = 0; k < 3; ++k) n *= std::max(g.n[k], 1);
        off[i] = total;
        total += static_cast<size_t>(n) * 8 + 256;
    }
    char *buf = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&buf), total) != hipSuccess)
        return set_error(VCM_E_NOMEM, "tuner result buffers");
    std::vector<vcm_result> res(nq);
    for (int i = 0; i < nq; ++i) {
        const vcm_grid &g = queries[i].grid;
        int64_t n = 1;
        for (int k = 0; k < 3; ++k) n *= std::max(g.n[k], 1);
        char *b = buf + off[i];
        res[i].c = reinterpret_cast<float *>(b);
        res[i].count = reinterpret_cast<uint16_t *>(b + 4 * n);
        res[i].bin = reinterpret_cast<uint8_t *>(b + 6 * n);
    }
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    vcm_status st = VCM_OK;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess)
        st = set_error(VCM_E_DEVICE, "tuner stream or events");
    out->n = 0;
    out->best_cell = 0.0;
    double best_ms = 1e300;
    for (int c = 0; c < n_cand && st == VCM_OK; ++c) {
        const double cs = o.cell_min * std::ldexp(1.0, c);
        vcm_index_opts io{};
        io.cell_size = cs;
        io.device = o.device;
        io.stream = s;
        vcm_index *ix = nullptr;
        st = vcm_build_index(obstacles, &io, &ix);
        if (st != VCM_OK) break;
        float best = 1e30f;
        for (int r = 0; r <= o.reps && st == VCM_OK; ++r) {
            hipEventRecord(e0, s);
            st = vcm_compute_batch(ix, queries, nq, res.data(), s, nullptr);
            hipEventRecord(e1, s);
            if (hipStreamSynchronize(s) != hipSuccess && st == VCM_OK)
                st = set_error(VCM_E_DEVICE, "tuner run failed");
            float ms = 0.0f;
            if (st == VCM_OK && r > 0 && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) best = std::min(best, ms);
        }
        // the width the index really used (a grid too fine is coarsened)
        const double used = ix->impl.dev.cs;
        vcm_free_index(ix);
        if (st != VCM_OK) break;
        out->cell[out->n] = used;
        out->ms[out->n] = best;
        ++out->n;
        if (best < best_ms) {
            best_ms = best;
            out->best_cell = used;
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (s) hipStreamDestroy(s);
    hipFree(buf);
    return st;
}

}  // extern "C"
