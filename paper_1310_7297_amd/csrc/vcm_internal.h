// Internal declarations shared by the HIP sources of libvcm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "vcm.h"

namespace vcm {

// Boxes are inserted into every column their footprint, grown by this much,
// overlaps.  It absorbs the rounding of the float32 corridor walk, whose
// position error is below 2^-9 m for scenes within 2^14 m.
constexpr float kFatMargin = 1.0f / 64.0f;

// Smallest float32 slab-test margin accepted (see prepare_query).
constexpr double kMinRecheckEps = 0x1p-21;

// Largest number of live samples per viewpoint (64-lane slots x 6).
constexpr int kMaxSamples = 384;
constexpr int kMaxSlots = 6;

// XCDs of an MI355X; work-item lists are split into this many ranges.
constexpr int kXcd = 8;
// The range counters sit 256 bytes apart, so that they do not share a cache
// line (every claim is a device-scope atomic).
constexpr int kCtrStride = 64;
constexpr size_t kCounterBytes = sizeof(unsigned) * kXcd * kCtrStride;

// One box reference inside a column list (32 bytes, one scalar load).
// Coordinates are in the index frame (see DevIndex), where they are >= 0,
// so two of them compare like their bit patterns as unsigned integers.
struct alignas(32) BoxRec {
    float lo[3];
    float hi[3];
    int32_t id;
    int32_t pad;
};

// Device view of the obstacle index.
// The index frame is the scene translated by -frame (an exact dyadic
// offset): the column grid starts at (0, 0) and every box has z >= 0.
struct DevIndex {
    const int32_t *col_start;  // nx*ny + 1 offsets into recs
    const BoxRec *recs;        // column lists, each sorted by decreasing hi.z
                               // and ended by a sentinel record (top -inf)
    float x0, y0;              // grid origin in the frame (0, 0)
    float cs, inv_cs;          // cell size (a power of two) and its inverse
    int32_t nx, ny;
    int32_t dim;
    int32_t pad;
};

// Target as the kernels use it.
struct TargetDesc {
    int32_t kind;       // VCM_SEGMENT / VCM_BILLBOARD / VCM_CUBE
    int32_t nax;        // normal axis (segment, billboard)
    int32_t nsign;
    int32_t su, sv;     // lattice per facet
    int32_t per_facet;  // su * sv
    uint64_t m_pf;      // ceil(2^32 / per_facet): exact division of sample indices
    uint64_t m_su;      // ceil(2^32 / su)
    float c[3];         // centre
    float half[3];      // half extents of the target's bounding box
    float hu, hv;       // half lattice spacing along u and v
    float S;            // size entering Eq. 1
    float rmax;         // viewer: radius of the covered ball (d_max); else 0
};

// Viewpoint lattice: q = o + (2i + 1) h2 (exact in float32).
struct GridDesc {
    float o[3];
    float h2[3];
    int32_t n[3];
    int32_t pad;
    int64_t count;
};

enum FovKind : int32_t { kFovAll = 0, kFovHalf = 1, kFovNarrow = 2, kFovWide = 3 };

struct ParamDesc {
    double fov_c2;      // cos^2 of the half angle (exact for the table's FOVs)
    double region_r2;   // viewer-centric maps: d_max^2 (the covered ball); else +inf
    int32_t fov_axis;   // axis and orientation of the wedge
    int32_t fov_sign;
    int32_t fov_kind;
    int32_t n_bins;
    int32_t bin_scale;
    int32_t mode;
    float d0;           // near point
    float V0;           // 2 atan(S / 2 d0)
    float inv_V0;
    float mu;           // angular resolution, radians
    float inv_log_V0_mu;
    float eps;          // slab-test margin (+inf: every test exact)
    float eps_ref;      // the default margin (disagreement statistics)
    double mu_d;        // angular resolution and near point in float64
    double d0_d;
    int32_t fp64;       // every ray test exact in float64, measure in float64
};

// Per-workgroup float64 partial sums of the pruned colouring, summed on the
// host in a fixed order (see PrunedSums in pruned.hip).
constexpr int kPrunedSums = 4;

// Counters gathered when statistics are requested (atomically accumulated).
struct DevStats {
    unsigned long long rays;
    unsigned long long box_tests;
    unsigned long long rechecks;
    unsigned long long fp32_disagree;
    unsigned long long columns;
    unsigned long long slot_tests;
    unsigned long long inside_box;
    unsigned long long t_fallbacks;
    unsigned long long records;
    unsigned long long narrow_tests;
    unsigned long long blocks;          // visible-region blocks classified
    unsigned long long blocks_decided;  // of which decided as a whole
    unsigned long long hull_tests;      // sample x obstacle hull tests of the blocks
    unsigned long long leaves;          // undecided smallest blocks traced at their representative
};

// Everything one brute-force launch needs (passed by value).
struct BruteArgs {
    DevIndex idx;
    TargetDesc tgt;
    GridDesc grid;
    ParamDesc prm;
    uint8_t *bin;
    float *c;
    uint16_t *count;
    DevStats *stats;
    unsigned *counter;  // kXcd work-item range counters (zeroed before the launch)
    uint32_t *gate;     // gate mode: per block, count | N << 10 | fov << 20
    int32_t theta;      // block size in viewpoints (gate mode)
    int32_t full_n[3];  // the viewpoint grid (gate mode)
    int32_t k_begin;    // first z layer of this launch
    uint32_t n_items;   // work items in this launch
    int32_t chunk;      // viewpoints of one grid row per work item (1..64)
    int32_t fill;       // gate mode, theta = 1: trace only the viewpoints whose
                        // gate word is kGateUndecided (the block tree decided
                        // the others)
};

// Gate word of a viewpoint the visible-region blocks left undecided.
constexpr uint32_t kGateUndecided = 0xffffffffu;

// A launch over the work items of many queries.
struct BatchArgs {
    unsigned *counter;  // kXcd range counters
    DevStats *stats;
    int32_t nq;
    uint32_t n_items;
};

// Launch shape of the ray kernels.
struct Tuning {
    int chunk = 0;          // viewpoints per work item; 0: by mode (chunk_for)
    int blocks_per_cu = 8;  // persistent workgroups (4 wavefronts each) per CU
};

// Viewpoints per work item.  FULL-mode viewpoints are cheap and reuse the
// previous viewpoint's blocker, so they take longer runs; FRACTION-mode ones
// balance better in short runs.
inline int chunk_for(const Tuning &t, int mode) {
    if (t.chunk > 0) return t.chunk;
    return mode == VCM_FULL ? 64 : 8;
}

// Host-side index object behind the opaque vcm_index handle.
struct Index {
    int device = 0;
    int dim = 3;
    int64_t n_boxes = 0;
    int64_t n_refs = 0;
    DevIndex dev{};
    int32_t *d_col_start = nullptr;
    BoxRec *d_recs = nullptr;
    double frame[3] = {0, 0, 0};  // world coordinates of the frame origin
    size_t bytes = 0;
    double build_ms = 0.0;
    double build_kernel_ms = 0.0;   // device time of the build kernels
    int32_t longest_list = 0;       // records in the longest column list
    // Host copy of the column lists (same layout as on the device), used to
    // reject targets that meet an obstacle.
    std::vector<int32_t> h_col_start;
    std::vector<BoxRec> h_recs;
};

// Makes `dev` current for the lifetime of the guard.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
    }
};

// Thread-local error reporting.
vcm_status set_error(vcm_status st, const std::string &msg);
void clear_error();

// Validation and translation of a query into kernel descriptors.
vcm_status prepare_query(const Index &ix, const vcm_query &q, TargetDesc *t, GridDesc *g,
                         ParamDesc *p);

// Launch the brute-force kernel over the whole grid of one query on `stream`
// (gate mode: over the representatives of the theta-blocks).  `counter`
// holds kCounterBytes of device memory (the work-item range counters; the
// launch clears them with a kernel first).
vcm_status launch_brute(const Index &ix, const TargetDesc &t, const GridDesc &g,
                        const ParamDesc &p, const vcm_result &r, hipStream_t stream,
                        DevStats *stats, uint32_t *gate, int theta, const Tuning &tune,
                        unsigned *counter, int fill = 0);

// Pieces of a batched launch.
int device_cus(int device);
int slots_for(const TargetDesc &t);
BruteArgs make_brute_args(const Index &ix, const TargetDesc &t, const GridDesc &g,
                          const ParamDesc &p, const vcm_result &r, uint32_t *gate, int theta,
                          int chunk);
void launch_zero_counter(unsigned *c, hipStream_t s);
// d_group_end: per query, the end of its groups of four work items in the
// launch's list (b.n_items counts groups).
vcm_status launch_brute_batch(const Index &ix, bool fp64, int mode, int ns, const BatchArgs &b,
                              const BruteArgs *d_recs, const uint32_t *d_group_end, int blocks,
                              hipStream_t s);

// Visible-region tree of the pruned methods (blocks.hip): blocks of `side`
// viewpoints per edge, from the root side down to the leaf side (the
// largest power of two not above theta), halved at every level.
#ifndef VCM_ROOT_BLOCK_SIDE
#define VCM_ROOT_BLOCK_SIDE 8
#endif
#ifndef VCM_MIN_CLASSIFIED_SIDE
#define VCM_MIN_CLASSIFIED_SIDE 8
#endif
constexpr int kRootBlockSide = VCM_ROOT_BLOCK_SIDE;
// With theta = 1 every viewpoint the tree leaves undecided is traced exactly
// (by the ray kernel over the grid, skipping decided viewpoints), so blocks
// below this side are not classified: tracing their viewpoints costs less
// than classifying them (measured).
constexpr int kMinClassifiedSide = VCM_MIN_CLASSIFIED_SIDE;
constexpr int kMaxBlockLevels = 16;
struct BlockPlan {
    int leaf = 1, root = 1, levels = 0;
    int side[kMaxBlockLevels] = {};
    int64_t count[kMaxBlockLevels] = {};  // blocks of the level over the grid
    int classified = 0;  // levels the block kernel classifies (from the root)
    int leaf_list = 0;   // lists[leaf_list]: the blocks the ray kernel traces
};
int block_leaf_side(int theta);
BlockPlan block_plan(const GridDesc &g, int dim, int theta);
// Classify the tree's blocks level by level.  gate: one word per viewpoint,
// written for the viewpoints of decided blocks; lists[l] (l = 1..levels)
// receive the blocks of level l (lists[levels]: the undecided smallest
// blocks), each with room for bp.count[min(l, levels - 1)] entries; ctr:
// 2 (levels + 1) words (entry counts of the lists at ctr[l], work counters
// after them), cleared by the call.
vcm_status launch_blocks(const Index &ix, const TargetDesc &t, const GridDesc &g, const ParamDesc &p,
                         const BlockPlan &bp, uint32_t *gate, uint32_t *const *lists, unsigned *ctr,
                         hipStream_t s, DevStats *stats);
// The undecided smallest blocks (list, with its entry count at *count):
// each takes its representative viewpoint's traced gate for every viewpoint
// it holds.  claim: a work counter, cleared by launch_blocks.
vcm_status launch_leaves(const Index &ix, const TargetDesc &t, const GridDesc &g, const ParamDesc &p,
                         const BlockPlan &bp, uint32_t *gate, const uint32_t *list, const unsigned *count,
                         unsigned *claim, hipStream_t s, DevStats *stats);
// Before launch_blocks with theta = 1: every gate word set to kGateUndecided.
void launch_gate_clear(uint32_t *gate, int64_t n, hipStream_t s);
// After launch_blocks: the gates of the viewpoints the tree left undecided.
// theta = 1: the ray kernel over the whole grid, tracing only the viewpoints
// whose gate word is still kGateUndecided (work items of consecutive
// viewpoints keep the ray kernel's blocker cache); theta > 1: launch_leaves
// over the undecided smallest blocks.  `counter`: the work-item counters of
// launch_brute.
vcm_status launch_undecided(const Index &ix, const TargetDesc &t, const GridDesc &g, const ParamDesc &p,
                            const BlockPlan &bp, uint32_t *gate, uint32_t *const *lists, unsigned *ctr,
                            unsigned *counter, hipStream_t s, DevStats *stats);

// Pruned colouring (E / M / T) of every viewpoint from its gate word.
// With `sums` non-null (pruned_sum_blocks(g) x kPrunedSums doubles), each
// workgroup also writes its partial sums of the Sec. V-A error and of the
// Sec. IV-A measured error (see pruned.hip).
vcm_status launch_pruned(const Index &ix, const TargetDesc &t, const GridDesc &g,
                         const ParamDesc &p, int method, const uint32_t *gate, const vcm_result &r,
                         hipStream_t stream, unsigned long long *fallback, double *sums);
int64_t pruned_sum_blocks(const GridDesc &g);
int count_rings(double S, double mu, double d0, double *V0);

vcm_status map_error(const float *ce, const float *ca, int64_t n, hipStream_t s, double *out);
void error_bounds(double S, double mu, double d0, int dim, double *out);

// Device scratch memory one query needs beside its inputs and outputs, as
// byte offsets into one buffer: the work-item counters, the pruned methods'
// block gates, and (pruned methods with statistics) the colouring's partial
// sums.
struct WsLayout {
    size_t counter = 0, gate = 0, sums = 0, ctr = 0, bytes = 0;
    size_t lists[kMaxBlockLevels + 1] = {};
    BlockPlan plan;
    int64_t n_sums = 0;  // workgroups writing PrunedSums (0: none)
};
WsLayout query_workspace(const GridDesc &g, int dim, int method, int theta, bool sums);

// One query on one stream: brute force, or the visible-region blocks, their
// undecided smallest blocks' representatives, and the pruned colouring.
// `ws` is device memory laid out as query_workspace(g, dim, method, theta,
// sums), 256-byte aligned; its contents on entry do not matter.  With `sums`
// (pruned methods) the colouring leaves its partial sums there.
vcm_status run_query(const Index &ix, const TargetDesc &t, const GridDesc &g, const ParamDesc &p,
                     int method, int theta, const vcm_result &r, hipStream_t s, DevStats *stats,
                     char *ws, bool sums);

// Pinned host buffers for host-to-device uploads, reused once the copies
// that read them have completed (tracked by an event per buffer).
class Staging {
  public:
    vcm_status acquire(size_t bytes, int device, int *slot, void **ptr);
    vcm_status release(int slot, hipStream_t s);

  private:
    static constexpr size_t kMaxSlotsStaging = 32;
    struct Slot {
        void *h = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
        int device = -1;
        bool busy = false;
        bool pending = false;
    };
    std::mutex m_;
    std::vector<Slot> slots_;
};
Staging &staging();
// Copy `bytes` from host memory to device memory, ordered on `s`; the host
// buffer may be reused as soon as the call returns.
vcm_status upload(const void *src, size_t bytes, void *dst, int device, hipStream_t s);

// One query of a batch, translated.
struct PlanQuery {
    TargetDesc t;
    GridDesc g;
    ParamDesc p;
    int method;
    int theta;
    vcm_result r;
    int ns;
    size_t ws_off;   // pruned methods: byte offset of the query's workspace in the plan's buffer
};

// Queries that share one persistent launch.
struct PlanGroup {
    bool fp64 = false;
    int mode = 0;
    int ns = 1;
    std::vector<int> members;
    size_t rec_off = 0, end_off = 0, ctr_off = 0;
    uint32_t n_items = 0;  // groups of four work items
};

// Device layout and launch sequence of a batch:
//   per group of brute-force queries: BruteArgs[members] | item ends[members]
//   | kXcd counters, then per pruned query its workspace (run_query).
struct BatchPlan {
    const Index *ix = nullptr;
    int device = 0;
    std::vector<PlanQuery> q;
    std::vector<PlanGroup> groups;
    Tuning tune;
    size_t bytes = 0;        // device buffer
    size_t image_bytes = 0;  // uploaded part (records, ends, counters)
    char *d_base = nullptr;
    uint64_t viewpoints = 0, items = 0;

    vcm_status prepare(const Index &ix, const vcm_query *qs, int nq, const vcm_result *rs);
    void layout();
    void image(std::vector<char> &img) const;  // uses d_base
    vcm_status enqueue(hipStream_t s, DevStats *stats) const;
};

// Build the column index on the device.
vcm_status build_index_device(Index *ix, const float *h_lo, const float *h_hi, int64_t n,
                              double cell_size, hipStream_t stream);

}  // namespace vcm

struct vcm_index {
    vcm::Index impl;
};
