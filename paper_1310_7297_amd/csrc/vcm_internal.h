// Internal declarations shared by the HIP sources of libvcm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "vcm.h"

namespace vcm {

// Boxes are inserted into every column their footprint, grown by this much,
// overlaps.  It absorbs the rounding of the float32 corridor walk, whose
// position error is below 2^-9 m for scenes within 2^14 m.
constexpr float kFatMargin = 1.0f / 64.0f;

// Largest number of live samples per viewpoint (64-lane slots x 6).
constexpr int kMaxSamples = 384;
constexpr int kMaxSlots = 6;

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
    float pad;
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
    unsigned *counter;  // work-item counter (zeroed before the launch)
    uint32_t *gate;     // gate mode: per block, count | N << 10 | fov << 20
    int32_t theta;      // block size in viewpoints (gate mode)
    int32_t full_n[3];  // the viewpoint grid (gate mode)
    int32_t k_begin;    // first z layer of this launch
    uint32_t n_items;   // work items in this launch
};

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
    // Host copy of the boxes (float32, exact), used for validation.
    std::string scene_key;
};

// Thread-local error reporting.
vcm_status set_error(vcm_status st, const std::string &msg);
void clear_error();

// Validation and translation of a query into kernel descriptors.
vcm_status prepare_query(const Index &ix, const vcm_query &q, TargetDesc *t, GridDesc *g,
                         ParamDesc *p);

// Launch the brute-force kernel over [vp_begin, vp_end) on `stream`.
vcm_status launch_brute(const Index &ix, const TargetDesc &t, const GridDesc &g,
                        const ParamDesc &p, const vcm_result &r, hipStream_t stream,
                        DevStats *stats, uint32_t *gate = nullptr, int theta = 1);

// Pruned colouring (E / M / T) of every viewpoint from the block gates.
vcm_status launch_pruned(const Index &ix, const TargetDesc &t, const GridDesc &g,
                         const ParamDesc &p, int method, int theta, const uint32_t *gate,
                         const int32_t gn[3], const vcm_result &r, hipStream_t stream,
                         unsigned long long *fallback);
int count_rings(double S, double mu, double d0, double *V0);

vcm_status map_error(const float *ce, const float *ca, int64_t n, hipStream_t s, double *out);
void error_bounds(double S, double mu, double d0, int dim, double *out);

// One query on one stream: brute force, or gates plus pruned colouring.
vcm_status run_query(const Index &ix, const TargetDesc &t, const GridDesc &g, const ParamDesc &p,
                     int method, int theta, const vcm_result &r, hipStream_t s, DevStats *stats);

// Build the column index on the device.
vcm_status build_index_device(Index *ix, const float *h_lo, const float *h_hi, int64_t n,
                              double cell_size, hipStream_t stream);

}  // namespace vcm
