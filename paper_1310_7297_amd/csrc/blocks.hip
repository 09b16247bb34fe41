// Visible-region blocks (Sec. III-C-1) for the pruned constructions.
//
// The paper indexes the visible region with a quad-tree (octree) whose
// blocks are split while they are partly visible, down to a minimum size.
// Here the tree is built level by level over the viewpoint lattice, one
// wavefront per block, its lanes holding the target's live samples (64 per
// slot), so that a block is classified against every obstacle near it at
// once:
//   * the live samples and the field of view must be the same over the whole
//     block (checked at its corners: each live-face condition is a
//     half-space, and the wedge rules are exact for convex sets);
//   * a sample is seen from all of the block when no obstacle meets the
//     convex hull of the block and the sample; it is hidden from all of it
//     when one obstacle meets the segments from every corner of the block to
//     the sample (the points whose segment to a sample meets an obstacle form
//     a convex set); both tests are exact in float64 on the 2^-8 lattice;
//   * FULL mode: one hidden sample decides the block (count 0), all seen
//     decide it (count N); FRACTION mode: every sample seen or hidden decides
//     it (count = seen);
//   * a decided block writes the gate (count | N << 10 | fov << 20) of every
//     one of its viewpoints; an undecided one is split into its octants, or,
//     at the smallest size, listed for the ray kernel, which traces its
//     representative viewpoint (k_leaves in brute.hip).
// A decided block's gate is the traced gate of each of its viewpoints (the
// tests above are exact), so a decided block's sub-blocks would be decided
// alike.  The map is therefore the same when the levels between blocks of 8
// and the smallest blocks are not classified: the undecided blocks of 8 list
// their smallest sub-blocks straight away, and each of those takes its
// representative's traced gate, which a classification could only confirm.
// Tracing a representative costs less than classifying a block (measured),
// so only blocks of edge 8 and more are classified.
// The candidate obstacles are those of the columns crossed by the convex hull
// of the block and the target's box, walked slab by slab along the major
// horizontal axis as for a single viewpoint.
#include <algorithm>
#include <cmath>

#include "trace_common.h"

namespace vcm {
namespace {

// Exact: does the closed box [a, c] meet the convex hull of the box [L, H]
// and the point s?  The hull is the union over lambda in [0, 1] of the boxes
// [s + lambda (L - s), s + lambda (H - s)]; per axis, two linear constraints
// lambda x <= y bound lambda by fractions, compared by cross-multiplication.
// Differences of lattice coordinates are exact in float32, their products in
// float64.
template <int DIM>
__device__ inline bool hull_meets(const float *L, const float *H, const float *s, const float *a,
                                  const float *c) {
    double ln = 0.0, ld = 1.0, un = 1.0, ud = 1.0;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const double x = side ? double(s[k] - H[k]) : double(L[k] - s[k]);
            const double y = side ? double(s[k] - a[k]) : double(c[k] - s[k]);
            if (x > 0.0) {
                if (y * ud < un * x) {
                    un = y;
                    ud = x;
                }
            } else if (x < 0.0) {
                if (-y * ld > ln * -x) {
                    ln = -y;
                    ld = -x;
                }
            } else {
                ok = ok && y >= 0.0;
            }
        }
    return ok && ln * ud <= un * ld;
}

// Float32 filters for the two hull tests: 1 when the hull surely meets the
// box, 0 when it surely misses, -1 when the float32 bounds on lambda lie
// within kHullEps of each other, where the exact test decides.  Each bound
// y / x is y * rcp(x) with x and y exact differences, within 1.5 * 2^-23
// relative (1 ulp for the reciprocal, half an ulp for the product); a bound
// beyond [-2, 2] decides nothing near the margin (min(1, .) and max(0, .)
// clip it, or the gap is then below -1), so every bound that matters is off
// by less than 2^-21, inside kHullEps.
constexpr float kHullEps = 0x1p-20f;

template <int DIM>
__device__ inline int hull_meets_f32(const float *L, const float *H, const float *s, const float *a,
                                     const float *c) {
    float lo = 0.0f, hi = 1.0f;
    bool fail = false;
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const float x = side ? s[k] - H[k] : L[k] - s[k];
            const float y = side ? s[k] - a[k] : c[k] - s[k];
            const float t = y * __builtin_amdgcn_rcpf(x);
            if (x > 0.0f) hi = fminf(hi, t);
            else if (x < 0.0f) lo = fmaxf(lo, t);
            else fail = fail || y < 0.0f;
        }
    if (fail) return 0;
    const float gap = hi - lo;
    return gap > kHullEps ? 1 : (gap < -kHullEps ? 0 : -1);
}

template <int DIM>
__device__ inline int hull2_meets_f32(const float *L, const float *H, const float *F0, const float *F1,
                                      const float *a, const float *c) {
    float lo = 0.0f, hi = 1.0f;
    bool fail = false;
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const float x = side ? H[k] - F1[k] : F0[k] - L[k];
            const float y = side ? H[k] - a[k] : c[k] - L[k];
            const float t = y * __builtin_amdgcn_rcpf(x);
            if (x > 0.0f) hi = fminf(hi, t);
            else if (x < 0.0f) lo = fmaxf(lo, t);
            else fail = fail || y < 0.0f;
        }
    if (fail) return 0;
    const float gap = hi - lo;
    return gap > kHullEps ? 1 : (gap < -kHullEps ? 0 : -1);
}

// Exact: does the closed box [a, c] meet the convex hull of the boxes [L, H]
// and [F0, F1]?  That hull is the union over lambda in [0, 1] of the boxes
// [L + lambda (F0 - L), H + lambda (F1 - H)]; per axis, two linear
// constraints on lambda, as in hull_meets.
template <int DIM>
__device__ inline bool hull2_meets(const float *L, const float *H, const float *F0, const float *F1,
                                   const float *a, const float *c) {
    double ln = 0.0, ld = 1.0, un = 1.0, ud = 1.0;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            // side 0: L + l (F0 - L) <= c;  side 1: H + l (F1 - H) >= a,
            // both written l x <= y
            const double x = side ? double(H[k] - F1[k]) : double(F0[k] - L[k]);
            const double y = side ? double(H[k] - a[k]) : double(c[k] - L[k]);
            if (x > 0.0) {
                if (y * ud < un * x) {
                    un = y;
                    ud = x;
                }
            } else if (x < 0.0) {
                if (-y * ld > ln * -x) {
                    ln = -y;
                    ld = -x;
                }
            } else {
                ok = ok && y >= 0.0;
            }
        }
    return ok && ln * ud <= un * ld;
}

struct BlockLevel {
    DevIndex idx;
    TargetDesc tgt;
    GridDesc grid;
    ParamDesc prm;
    uint32_t *gate;            // per viewpoint: count | N << 10 | fov << 20
    const uint32_t *in_list;   // blocks of this level (index in its block grid); null: all
    const uint32_t *in_count;  // entries of in_list
    uint32_t n_all;            // blocks of this level when in_list is null
    uint32_t *out_list;        // sub-blocks of undecided blocks, or the blocks themselves
    uint32_t *out_count;
    unsigned *claim;           // work counter of this launch
    DevStats *stats;
    int32_t side;              // viewpoints per block edge
    int32_t nb[3];             // blocks per axis at this level
    int32_t child;             // edge of the sub-blocks listed for undecided blocks;
                               // 0: list the undecided blocks themselves
    int32_t nbc[3];            // sub-blocks per axis over the grid
};

// Position of viewpoint index i along axis k (exact).
__device__ inline float vp_pos(const GridDesc &g, int k, int i) {
    return g.o[k] + static_cast<float>(2 * i + 1) * g.h2[k];
}

// Candidate obstacles of a block: the records of the columns crossed by the
// convex hull of the box C = [L, H] and the target's box, slab by slab along
// axis AX from the target end.  `visit(lo, hi)` is called with each
// candidate's corners and returns true to stop the walk.  Float32 with the
// same margins as the viewpoint corridor: the walk never drops a column or
// record the hull reaches (records are inserted with a 2^-6 m margin).
// part / nparts: this wavefront walks slabs part, part + nparts, ...; stop
// (COOP): a flag another wavefront of the workgroup sets when the block is
// decided.
template <int DIM, int AX, bool FAST, bool COOP, class Visit>
__device__ inline void block_walk(const BlockLevel &B, cptr_i32 col_start, cptr_rec recs, const float (&L)[3],
                                  const float (&H)[3], int part, int nparts, const volatile int *stop,
                                  Visit &&visit) {
    const TargetDesc &T = B.tgt;
    const DevIndex &X = B.idx;
    const int lane = threadIdx.x & 63;
    constexpr int BX = 1 - AX;
    const float F0[3] = {T.c[0] - T.half[0], T.c[1] - T.half[1], T.c[2] - T.half[2]};
    const float F1[3] = {T.c[0] + T.half[0], T.c[1] + T.half[1], T.c[2] + T.half[2]};
    const int na = AX == 0 ? X.nx : X.ny, nb = AX == 0 ? X.ny : X.nx;
    // the hull is the union over l in [0, 1] of the boxes
    // [L + l (F0 - L), H + l (F1 - H)]
    const float ua0 = F0[AX] - L[AX], ua1 = F1[AX] - H[AX];
    const float iua0 = ua0 != 0.0f ? __builtin_amdgcn_rcpf(ua0) : 0.0f;
    const float iua1 = ua1 != 0.0f ? __builtin_amdgcn_rcpf(ua1) : 0.0f;
    const float vb0 = F0[BX] - L[BX], vb1 = F1[BX] - H[BX];
    const float wz0 = F0[2] - L[2], wz1 = F1[2] - H[2];
    const float amin = fminf(L[AX], F0[AX]), amax = fmaxf(H[AX], F1[AX]);
    if (!(amax >= 0.0f && amin < na * X.cs)) return;
    const int ia_lo = max(0, min(na - 1, static_cast<int>(floorf(amin * X.inv_cs))));
    const int ia_hi = max(0, min(na - 1, static_cast<int>(floorf(amax * X.inv_cs))));
    const float ca = 0.5f * (L[AX] + H[AX]);
    const int step = (ca <= T.c[AX]) ? -1 : 1;
    for (int s = part; s <= ia_hi - ia_lo; s += nparts) {
        if (COOP && *stop) return;
        const int ia = step < 0 ? ia_hi - s : ia_lo + s;
        const float A0 = ia * X.cs, A1 = A0 + X.cs;
        float l0 = 0.0f, l1 = 1.0f;
        bool ok = true;
        const float r1 = A1 - L[AX], r2 = A0 - H[AX];
        if (ua0 > 0.0f) l1 = fminf(l1, r1 * iua0);
        else if (ua0 < 0.0f) l0 = fmaxf(l0, r1 * iua0);
        else ok = ok && r1 >= 0.0f;
        if (ua1 > 0.0f) l0 = fmaxf(l0, r2 * iua1);
        else if (ua1 < 0.0f) l1 = fminf(l1, r2 * iua1);
        else ok = ok && r2 <= 0.0f;
        l0 = fmaxf(0.0f, l0 - kLambdaMargin);
        l1 = fminf(1.0f, l1 + kLambdaMargin);
        if (!ok || l0 > l1) continue;
        const float bl = fminf(L[BX] + l0 * vb0, L[BX] + l1 * vb0) - kWalkMargin;
        const float bh = fmaxf(H[BX] + l0 * vb1, H[BX] + l1 * vb1) + kWalkMargin;
        const float zf = fminf(L[2] + l0 * wz0, L[2] + l1 * wz0) - kWalkMargin;
        const float zc = fmaxf(H[2] + l0 * wz1, H[2] + l1 * wz1) + kWalkMargin;
        if (!(bh >= 0.0f && bl < nb * X.cs)) continue;
        const int ib0 = max(0, min(nb - 1, static_cast<int>(floorf(bl * X.inv_cs))));
        const int ib1 = max(0, min(nb - 1, static_cast<int>(floorf(bh * X.inv_cs))));
        for (int ib = ib0; ib <= ib1; ++ib) {
            const int col = AX == 0 ? ia + X.nx * ib : ib + X.nx * ia;
            const int cb = col_start[col], ce = col_start[col + 1] - 1;
            for (int base = cb;; base += 64) {
                const BoxRec R = recs[min(base + lane, ce)];
                // lists are sorted by decreasing top and end with a sentinel
                // whose top is -inf: the scan ends below the hull's floor
                const bool above = R.hi[2] >= zf;
                bool cand = above && R.id >= 0 && R.hi[BX] >= bl && R.lo[BX] <= bh && (DIM == 2 || R.lo[2] <= zc);
                // exactly: only a box that meets the hull of the block and the
                // target's box can meet a line of sight from the block
                if (cand) {
                    if constexpr (FAST) {
                        const int f = hull2_meets_f32<DIM>(L, H, F0, F1, R.lo, R.hi);
                        cand = f > 0 || (f < 0 && hull2_meets<DIM>(L, H, F0, F1, R.lo, R.hi));
                    } else {
                        cand = hull2_meets<DIM>(L, H, F0, F1, R.lo, R.hi);
                    }
                }
                unsigned long long cm = __ballot(cand);
                const unsigned long long below = __ballot(!above);
                while (cm) {
                    const int r = __builtin_ctzll(cm);
                    cm &= cm - 1;
                    float lo[3], hi[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        lo[k] = readlane_f(R.lo[k], r);
                        hi[k] = readlane_f(R.hi[k], r);
                    }
                    if (visit(lo, hi)) return;
                }
                if (below) break;
            }
        }
    }
}

// Field of view over the block (corners q[c]): 1 all inside, 0 all outside,
// -1 undecided (see the header comment).
template <int DIM>
__device__ inline int fov_class(const TargetDesc &T, const ParamDesc &P, const float (&L)[3], const float (&H)[3]) {
    // a viewer's ball is convex: corners inside put the block inside; the
    // block is outside when its nearest point to the viewer is beyond rmax
    int region = 1;
    if (T.kind == VCM_VIEWER) {
        bool all_in = true;
        double g2 = 0.0;
#pragma unroll
        for (int c = 0; c < (1 << DIM); ++c) {
            float q[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) q[k] = ((c >> k) & 1) ? H[k] : L[k];
            all_in = all_in && in_region<DIM>(T, q);
        }
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const double x = T.c[k];
            const double gap = x < L[k] ? double(L[k]) - x : (x > H[k] ? x - double(H[k]) : 0.0);
            g2 += gap * gap;
        }
        region = all_in ? 1 : (g2 > double(T.rmax) * double(T.rmax) ? 0 : -1);
        if (region == 0) return 0;
    }
    if (P.fov_kind == kFovAll) return region;
    bool all_in = true, all_out = true, all_front = true, all_back = true;
#pragma unroll
    for (int c = 0; c < (1 << DIM); ++c) {
        float q[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) q[k] = ((c >> k) & 1) ? H[k] : L[k];
        const bool in = in_wedge<DIM>(T, P, q);
        const double dn = P.fov_sign * (double(q[P.fov_axis]) - double(T.c[P.fov_axis]));
        all_in = all_in && in;
        all_out = all_out && !in;
        all_front = all_front && dn >= 0.0;
        all_back = all_back && dn < 0.0;
    }
    // a wedge no wider than a half-space is convex; a wider one has a convex
    // complement and contains the half-space in front of the target
    const int wedge = P.fov_kind != kFovWide ? (all_in ? 1 : (all_back ? 0 : -1))
                                             : (all_front ? 1 : (all_out ? 0 : -1));
    if (wedge == 0) return 0;
    return (region == 1 && wedge == 1) ? 1 : -1;
}

// Live faces over the block: packed face codes (as the ray kernel packs them)
// and their number; false if a face is live for part of the block only.
__device__ inline bool live_faces(const TargetDesc &T, const float (&L)[3], const float (&H)[3], unsigned &faces,
                                  int &nf) {
    faces = 0;
    nf = 0;
    if (T.kind != VCM_CUBE) {
        nf = 1;
        return true;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float up = T.c[k] + T.half[k], dn = T.c[k] - T.half[k];
        // the +k face is live where q_k > up, the -k face where q_k < dn
        const bool up_lo = L[k] > up, up_hi = H[k] > up;
        const bool dn_lo = L[k] < dn, dn_hi = H[k] < dn;
        if (up_lo != up_hi || dn_lo != dn_hi) return false;
        if (up_lo) faces |= static_cast<unsigned>(2 * k + 1) << (4 * nf++);
        if (dn_lo) faces |= static_cast<unsigned>(2 * k) << (4 * nf++);
    }
    return true;
}

// Block-hierarchy statistics of one wavefront.
struct BlockStats {
    unsigned long long blocks = 0, decided = 0, hull_tests = 0, cols = 0;
};

// One level of the tree.  COOP: the four wavefronts of a workgroup classify
// one block together, each walking every fourth slab of its corridor, and
// their seen / hidden masks are combined in LDS (a block's decision does not
// depend on the order of its candidates, so the result is the one-wavefront
// result).  Used for long walks only (FRACTION mode, blocks of 16 and more),
// where a few blocks would otherwise set the launch's length.
template <int DIM, int NS, int MODE, bool COOP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_blocks(
    BlockLevel B, const int32_t *col_start_g, const BoxRec *recs_g) {
    const cptr_i32 col_start = (cptr_i32)col_start_g;
    const cptr_rec recs = (cptr_rec)recs_g;
    __shared__ float4 s_tab[kTableMax];
    build_sample_table<DIM>(B.tgt, s_tab);
    const TargetDesc &T = B.tgt;
    const GridDesc &G = B.grid;
    const int lane = threadIdx.x & 63;
    const uint32_t n_in = B.in_list ? *B.in_count : B.n_all;
    constexpr int kParts = COOP ? 4 : 1;
    const int wave = COOP ? static_cast<int>(threadIdx.x >> 6) : 0;
    const int lead = COOP ? static_cast<int>(threadIdx.x) : lane;  // 0: the block's writer
    __shared__ uint32_t s_item;
    __shared__ int s_stop;
    __shared__ unsigned long long s_seen[kParts][NS], s_hid[kParts][NS];
    BlockStats st;
    for (;;) {
        uint32_t item = 0;
        if constexpr (COOP) {
            __syncthreads();
            if (threadIdx.x == 0) {
                s_item = atomicAdd(B.claim, 1u);
                s_stop = 0;
            }
            __syncthreads();
            item = __builtin_amdgcn_readfirstlane(s_item);
        } else {
            if (lane == 0) item = atomicAdd(B.claim, 1u);
            item = __builtin_amdgcn_readfirstlane(__shfl(item, 0));
        }
        if (item >= n_in) break;
        const uint32_t b = B.in_list ? B.in_list[item] : item;
        int bi[3] = {static_cast<int>(b % static_cast<uint32_t>(B.nb[0])),
                     static_cast<int>((b / static_cast<uint32_t>(B.nb[0])) % static_cast<uint32_t>(B.nb[1])),
                     static_cast<int>(b / (static_cast<uint32_t>(B.nb[0]) * static_cast<uint32_t>(B.nb[1])))};
        int lo[3], hi[3];
        float L[3], H[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lo[k] = bi[k] * B.side;
            hi[k] = min(lo[k] + B.side, G.n[k]) - 1;
            if (k >= DIM) lo[k] = hi[k] = 0;
            L[k] = k < DIM ? vp_pos(G, k, lo[k]) : 0.0f;
            H[k] = k < DIM ? vp_pos(G, k, hi[k]) : 0.0f;
        }
        if (wave == 0) ++st.blocks;
        // ---- classification
        unsigned faces = 0;
        int nf = 0;
        const bool uni = live_faces(T, L, H, faces, nf);
        const int fc = fov_class<DIM>(T, B.prm, L, H);
        const int N = nf * T.per_facet;
        bool decided = false;
        int count = 0;
        if (uni && fc >= 0) {
            if (fc == 0 || N == 0) {
                decided = true;
            } else {
                // lanes hold the live samples
                float sp[NS][3];
                unsigned long long live[NS], seen[NS], hidden[NS];
#pragma unroll
                for (int j = 0; j < NS; ++j) {
                    const int si = j * 64 + lane;
                    live[j] = __ballot(si < N);
                    sample_pos<DIM, kTabBlock>(T, faces, si < N ? si : 0, sp[j], s_tab);
                    seen[j] = live[j];
                    hidden[j] = 0;
                }
                bool stop = false;
                auto visit = [&](const float (&a)[3], const float (&c)[3]) -> bool {
                    bool all_hidden = true;
#pragma unroll
                    for (int j = 0; j < NS; ++j) {
                        const unsigned long long todo = live[j] & ~hidden[j];
                        if (!todo) continue;
                        bool meet = false, hid = false;
                        if ((todo >> lane) & 1) {
                            if constexpr (MODE == VCM_FRACTION) {
                                const int f = hull_meets_f32<DIM>(L, H, sp[j], a, c);
                                meet = f > 0 || (f < 0 && hull_meets<DIM>(L, H, sp[j], a, c));
                            } else {
                                meet = hull_meets<DIM>(L, H, sp[j], a, c);
                            }
                            if (meet) {
                                // hidden from the whole block if the box cuts
                                // the segment from every corner to the sample
                                hid = true;
#pragma unroll 1
                                for (int cn = 0; cn < (1 << DIM) && hid; ++cn) {
                                    float d[3], lq[3], hq[3];
#pragma unroll
                                    for (int k = 0; k < 3; ++k) {
                                        const float qk = ((cn >> k) & 1) ? H[k] : L[k];
                                        d[k] = sp[j][k] - qk;
                                        lq[k] = a[k] - qk;
                                        hq[k] = c[k] - qk;
                                    }
                                    hid = hid && exact_contact<DIM>(d, lq, hq);
                                }
                            }
                        }
                        st.hull_tests += __popcll(todo);
                        seen[j] &= ~__ballot(meet);
                        hidden[j] |= __ballot(hid);
                        if (MODE == VCM_FULL && hidden[j]) {
                            stop = true;
                            if (COOP && lane == 0) s_stop = 1;
                            return true;
                        }
                        all_hidden = all_hidden && hidden[j] == live[j];
                    }
                    // FRACTION mode: nothing left to learn once all are hidden
                    if (MODE == VCM_FRACTION && all_hidden) {
                        stop = true;
                        if (COOP && lane == 0) s_stop = 1;
                        return true;
                    }
                    return false;
                };
                const float dx = fabsf(T.c[0] - 0.5f * (L[0] + H[0])), dy = fabsf(T.c[1] - 0.5f * (L[1] + H[1]));
                if (dx >= dy)
                    block_walk<DIM, 0, MODE == VCM_FRACTION, COOP>(B, col_start, recs, L, H, wave, kParts, &s_stop,
                                                                    visit);
                else
                    block_walk<DIM, 1, MODE == VCM_FRACTION, COOP>(B, col_start, recs, L, H, wave, kParts, &s_stop,
                                                                    visit);
                (void)stop;
                if constexpr (COOP) {
                    // the workgroup's masks: seen from the whole block by
                    // every part, hidden by some part
                    if (lane == 0) {
#pragma unroll
                        for (int j = 0; j < NS; ++j) {
                            s_seen[wave][j] = seen[j];
                            s_hid[wave][j] = hidden[j];
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int j = 0; j < NS; ++j) {
                        unsigned long long sa = ~0ull, ho = 0ull;
#pragma unroll
                        for (int w = 0; w < kParts; ++w) {
                            sa &= s_seen[w][j];
                            ho |= s_hid[w][j];
                        }
                        seen[j] = sa;
                        hidden[j] = ho;
                    }
                }
                int n_seen = 0, n_hidden = 0;
#pragma unroll
                for (int j = 0; j < NS; ++j) {
                    n_seen += __popcll(seen[j]);
                    n_hidden += __popcll(hidden[j]);
                }
                if (MODE == VCM_FULL) {
                    if (n_hidden > 0) {
                        decided = true;
                        count = 0;
                    } else if (n_seen == N) {
                        decided = true;
                        count = N;
                    }
                } else if (n_seen + n_hidden == N) {
                    decided = true;
                    count = n_seen;
                }
            }
        }
        if (decided) {
            // the gate of every viewpoint of the block
            if (wave == 0) ++st.decided;
            const uint32_t word = static_cast<uint32_t>(count) | (static_cast<uint32_t>(N) << 10) |
                                  (fc > 0 ? (1u << 20) : 0u);
            const int e0 = hi[0] - lo[0] + 1, e1 = hi[1] - lo[1] + 1, e2 = hi[2] - lo[2] + 1;
            const int tot = e0 * e1 * e2;
            for (int t = COOP ? static_cast<int>(threadIdx.x) : lane; t < tot; t += COOP ? 256 : 64) {
                const int i = lo[0] + t % e0, j = lo[1] + (t / e0) % e1, k = lo[2] + t / (e0 * e1);
                B.gate[i + static_cast<int64_t>(G.n[0]) * (j + static_cast<int64_t>(G.n[1]) * k)] = word;
            }
        } else if (B.child == 0) {
            if (lead == 0 && B.out_list) B.out_list[atomicAdd(B.out_count, 1u)] = b;
        } else if (wave == 0) {
            // the sub-blocks of edge B.child that hold viewpoints (at most 64:
            // the octants, or the smallest blocks of a block at most 4 of
            // them wide), lane t taking sub-block t
            const int r = B.side / B.child;
            const int tot = DIM == 3 ? r * r * r : r * r;
            int c[3] = {0, 0, 0};
            bool in = lane < tot;
            c[0] = bi[0] * r + lane % r;
            c[1] = bi[1] * r + (lane / r) % r;
            c[2] = DIM == 3 ? bi[2] * r + lane / (r * r) : 0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) in = in && c[k] * B.child < G.n[k];
            const unsigned long long mask = __ballot(in);
            uint32_t base = 0;
            if (lane == 0 && mask) base = atomicAdd(B.out_count, static_cast<uint32_t>(__popcll(mask)));
            base = __shfl(base, 0);
            if (in)
                B.out_list[base + mbcnt(mask)] =
                    static_cast<uint32_t>(c[0]) +
                    static_cast<uint32_t>(B.nbc[0]) *
                        (static_cast<uint32_t>(c[1]) + static_cast<uint32_t>(B.nbc[1]) * static_cast<uint32_t>(c[2]));
        }
    }
    if (B.stats && lane == 0) {
        atomicAdd(&B.stats->blocks, st.blocks);
        atomicAdd(&B.stats->blocks_decided, st.decided);
        atomicAdd(&B.stats->hull_tests, st.hull_tests);
    }
}

__global__ void k_zero_words(unsigned *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

template <int DIM, int MODE, class F>
void dispatch_blocks(int ns, F &&f) {
    if (ns <= 1) f(std::integral_constant<int, 1>{});
    else if (ns == 2) f(std::integral_constant<int, 2>{});
    else if (ns == 3) f(std::integral_constant<int, 3>{});
    else f(std::integral_constant<int, 6>{});
}

}  // namespace

static_assert(kMinClassifiedSide >= 2, "blocks of one viewpoint are traced, not classified");
static_assert(kRootBlockSide >= kMinClassifiedSide, "the root level is classified");

int block_leaf_side(int theta) {
    int s = 1;
    while (2 * s <= theta) s *= 2;
    return s;
}

BlockPlan block_plan(const GridDesc &g, int dim, int theta) {
    BlockPlan bp;
    bp.leaf = block_leaf_side(theta);
    bp.root = std::max(bp.leaf, kRootBlockSide);
    bp.levels = 0;
    for (int s = bp.root; s >= bp.leaf; s /= 2) {
        int64_t n = 1;
        for (int k = 0; k < 3; ++k) n *= k < dim ? (g.n[k] + s - 1) / s : 1;
        bp.side[bp.levels] = s;
        bp.count[bp.levels] = n;
        // classified: blocks of edge kMinClassifiedSide and more, and (theta
        // > 1) those more than 4 smallest blocks wide, whose smallest blocks
        // would not fit one wavefront's list step
        if (s >= kMinClassifiedSide || (bp.leaf > 1 && s > 4 * bp.leaf)) bp.classified = bp.levels + 1;
        ++bp.levels;
    }
    if (bp.classified == 0) bp.classified = 1;
    // the ray kernel's list: theta > 1, the smallest blocks of the undecided
    // blocks of the last classified level (its representatives are traced);
    // theta = 1, none (the viewpoints of those blocks are traced)
    bp.leaf_list = bp.leaf > 1 ? bp.levels : bp.levels - 1;
    return bp;
}

vcm_status launch_blocks(const Index &ix, const TargetDesc &t, const GridDesc &g, const ParamDesc &p,
                         const BlockPlan &bp, uint32_t *gate, uint32_t *const *lists, unsigned *ctr,
                         hipStream_t s, DevStats *stats) {
    // ctr: [0, levels] entry counts of lists[1..levels] (the last is the list
    // of undecided smallest blocks), then one work counter per launch
    const int nctr = 2 * (bp.levels + 1);
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, ctr, nctr);
    const int cus = device_cus(ix.device);
    const int ns = slots_for(t);
    for (int l = 0; l < bp.classified; ++l) {
        BlockLevel B{};
        B.idx = ix.dev;
        B.tgt = t;
        B.grid = g;
        B.prm = p;
        B.gate = gate;
        B.in_list = l == 0 ? nullptr : lists[l];
        B.in_count = l == 0 ? nullptr : ctr + l;
        B.n_all = static_cast<uint32_t>(bp.count[0]);
        const bool last = l == bp.classified - 1;
        // theta = 1: the last classified level lists nothing (the ray kernel
        // traces every viewpoint whose gate is still undecided)
        B.out_list = last ? (bp.leaf > 1 ? lists[bp.leaf_list] : nullptr) : lists[l + 1];
        B.out_count = last ? ctr + bp.leaf_list : ctr + l + 1;
        B.claim = ctr + bp.levels + 1 + l;
        B.stats = stats;
        B.side = bp.side[l];
        // sub-blocks of undecided blocks: the next level's; at the last
        // classified level, theta > 1: its smallest blocks (none when it is
        // the smallest level: the block is listed itself); theta = 1: not
        // listed
        B.child = !last ? bp.side[l] / 2 : (bp.leaf > 1 && bp.leaf < bp.side[l] ? bp.leaf : 0);
        if (B.child > 0) {
            const int r = bp.side[l] / B.child;
            if ((ix.dim == 3 ? r * r * r : r * r) > 64) return set_error(VCM_E_INTERNAL, "block plan: too many sub-blocks");
        }
        const int cs = std::max(1, B.child);
        for (int k = 0; k < 3; ++k) {
            B.nb[k] = k < ix.dim ? (g.n[k] + B.side - 1) / B.side : 1;
            B.nbc[k] = k < ix.dim ? (g.n[k] + cs - 1) / cs : 1;
        }
        const int64_t want = l == 0 ? (bp.count[0] + 3) / 4 : int64_t(cus) * 8;
        const dim3 grid(static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(want, int64_t(cus) * 8))));
        // FRACTION mode with blocks of 16 and more: a workgroup per block
        // (measured: FRACTION VCM_E at theta 16, 1.42 -> 0.83 ms; for blocks
        // of 8, and in FULL mode, one wavefront per block is faster)
        const bool coop = p.mode == VCM_FRACTION && bp.side[l] >= 16;
        auto go = [&](auto nsv) {
            constexpr int NS = decltype(nsv)::value;
            if (ix.dim == 2) {
                if (p.mode == VCM_FULL)
                    hipLaunchKernelGGL((k_blocks<2, NS, VCM_FULL, false>), grid, dim3(256), 0, s, B, ix.dev.col_start,
                                       ix.dev.recs);
                else if (coop)
                    hipLaunchKernelGGL((k_blocks<2, NS, VCM_FRACTION, true>), grid, dim3(256), 0, s, B,
                                       ix.dev.col_start, ix.dev.recs);
                else
                    hipLaunchKernelGGL((k_blocks<2, NS, VCM_FRACTION, false>), grid, dim3(256), 0, s, B,
                                       ix.dev.col_start, ix.dev.recs);
            } else {
                if (p.mode == VCM_FULL)
                    hipLaunchKernelGGL((k_blocks<3, NS, VCM_FULL, false>), grid, dim3(256), 0, s, B, ix.dev.col_start,
                                       ix.dev.recs);
                else if (coop)
                    hipLaunchKernelGGL((k_blocks<3, NS, VCM_FRACTION, true>), grid, dim3(256), 0, s, B,
                                       ix.dev.col_start, ix.dev.recs);
                else
                    hipLaunchKernelGGL((k_blocks<3, NS, VCM_FRACTION, false>), grid, dim3(256), 0, s, B,
                                       ix.dev.col_start, ix.dev.recs);
            }
        };
        dispatch_blocks<3, 0>(ns, go);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return set_error(VCM_E_DEVICE, std::string("block kernel launch: ") + hipGetErrorString(e));
    }
    return VCM_OK;
}

}  // namespace vcm
