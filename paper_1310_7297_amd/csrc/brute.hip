// Brute-force VCM kernel: every viewpoint of the lattice, every live sample
// of the target, every obstacle on the way (the naive map of Sec. III and the
// grid "baseline" of Sec. V-B, computed exactly).
//
// Work decomposition (gfx950, 64-lane wavefronts):
//   * one wavefront per viewpoint q; its lanes hold the rays q -> s to the
//     live samples s of the target (64 per slot, NS slots per lane);
//   * the wavefront walks, column by column, the corridor swept by the rays
//     (the convex hull of q and the target's footprint), starting at the
//     target end where occluders are most likely;
//   * inside a column, the lanes read and cull 64 box records at a time
//     (integer compares), and the list stops at the first box whose top lies
//     below the corridor's lowest point; each candidate box is then tested
//     against all 64 * NS rays;
//   * each lane runs a float32 slab test per ray; a result within `eps` of
//     the decision boundary is settled by the exact float64 predicate;
//   * visibility is reduced with wave ballots and popcounts (integers only).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "trace_common.h"

namespace vcm {
namespace {

struct WaveStats {
    unsigned long long tests = 0, slots = 0, rechecks = 0, cols = 0, rays = 0, inside = 0, recs = 0, narrow = 0,
                       filled = 0;
};

// FRACTION-mode compaction buffer of a wavefront, one entry per ray: with up
// to three slots an entry carries the ray's reciprocal direction beside its
// sample index, so a moved ray needs no new set-up; with more slots it holds
// the index alone (an entry of 16 bytes per ray would cut those kernels'
// occupancy) and the ray is set up again.
template <int NS>
using RaySlot = typename std::conditional<(NS <= 3), float4, int>::type;


// Rays of slot j (among the open ones) that a box blocks: float32 slab test
// with margin eps; results inside the margin, and rays with a zero direction
// component, are settled by the exact predicate.  blq and bhq are the box's
// corners minus q (exact: dyadic coordinates).
template <int DIM, int NS, bool EXACT64, bool STATS, int TAB>
__device__ __attribute__((always_inline)) inline unsigned long long slot_hits(
    int j, const float (&blq)[3], const float (&bhq)[3], const TargetDesc &T, const ParamDesc &P,
    const float *q, unsigned faces, const void *tab, const float (&iv)[NS][3], const int (&sidx)[NS],
    const unsigned long long (&open)[NS], const unsigned long long (&zmask)[NS], WaveStats &ws,
    unsigned long long &n_disagree) {
    const int lane = threadIdx.x & 63;
    unsigned long long hit, unsure;
    float gap = 0.0f;
    if (EXACT64) {
        hit = 0;
        unsure = open[j];
    } else {
        // eps = +inf sends every test to the exact predicate
        gap = slab_gap<DIM>(iv[j], blq, bhq);
        hit = __ballot(gap > P.eps) & open[j];
        unsure = (__ballot(fabsf(gap) <= P.eps) | zmask[j]) & open[j];
    }
    if (__builtin_expect(unsure != 0, 0)) {
        bool ex = false;
        if ((unsure >> lane) & 1) {
            float sp[3], d[3];
            // opaque copy: keeps this rare work out of the hot loops (it is
            // loop-invariant per ray)
            int si = sidx[j];
            asm volatile("" : "+v"(si));
            sample_pos<DIM, TAB>(T, faces, si, sp, tab);
            float lq2[3], hq2[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                d[k] = sp[k] - q[k];
                // keep this rare path's work inside the branch
                lq2[k] = blq[k];
                hq2[k] = bhq[k];
                asm volatile("" : "+v"(lq2[k]), "+v"(hq2[k]));
            }
            ex = exact_contact<DIM>(d, lq2, hq2);
            if (STATS && !EXACT64 && !((zmask[j] >> lane) & 1) && fabsf(gap) > P.eps_ref &&
                (gap > 0.0f) != ex)
                ++n_disagree;
        }
        hit = (hit & ~unsure) | (__ballot(ex) & unsure);
    }
    if (STATS) {
        ws.tests += __popcll(open[j]);
        ws.rechecks += EXACT64 ? 0 : __popcll(unsure);
        ++ws.slots;
    }
    return hit;
}

// Test the open rays against one box (slot by slot) and clear the rays it
// blocks.  Returns 0 when the viewpoint is decided (FULL mode: some ray is
// blocked; FRACTION mode: no ray is left open), else a non-zero mask.
template <int DIM, int NS, bool EXACT64, int MODE, bool STATS, int TAB>
__device__ __attribute__((always_inline)) inline unsigned long long box_test(
    const float (&blq)[3], const float (&bhq)[3], const TargetDesc &T, const ParamDesc &P, const float *q,
    unsigned faces, const void *tab, const float (&iv)[NS][3], const int (&sidx)[NS],
    unsigned long long (&open)[NS], const unsigned long long (&zmask)[NS], WaveStats &ws,
    unsigned long long &n_disagree) {
    unsigned long long open_any = 0;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        if (!open[j]) continue;
        const unsigned long long hit = slot_hits<DIM, NS, EXACT64, STATS, TAB>(j, blq, bhq, T, P, q, faces, tab, iv,
                                                                              sidx, open, zmask, ws, n_disagree);
        open[j] &= ~hit;
        // FULL mode: one blocked ray decides the viewpoint
        if (MODE == VCM_FULL && hit != 0) return 0;
        open_any |= open[j];
    }
    return MODE == VCM_FULL ? ~0ull : open_any;
}

// The corridor walk of one viewpoint (wave-uniform) along major axis AX:
// the columns crossed by the convex hull of q and the target's box, slab by
// slab from the target end, slabs prepared 64 at a time.  Clears the rays
// the boxes met block; returns early when the viewpoint is decided.
template <int DIM, int NS, bool EXACT64, int MODE, bool STATS, int TAB, int AX>
__device__ __attribute__((always_inline)) inline void corridor_walk(
    const BruteArgs &A, cptr_rec recs, cptr_i32 col_start, const float *q, unsigned faces, RaySlot<NS> *lds,
    const void *tab, int &blk, float (&iv)[NS][3], int (&sidx)[NS], unsigned long long (&open)[NS],
    unsigned long long (&zmask)[NS], WaveStats &ws, unsigned long long &n_disagree) {
    const TargetDesc &T = A.tgt;
    const ParamDesc &P = A.prm;
    const DevIndex &X = A.idx;
    const int lane = threadIdx.x & 63;
    const float F0[3] = {T.c[0] - T.half[0], T.c[1] - T.half[1], T.c[2] - T.half[2]};
    const float F1[3] = {T.c[0] + T.half[0], T.c[1] + T.half[1], T.c[2] + T.half[2]};
    constexpr int BX = 1 - AX;  // the other horizontal axis
    const int na = AX == 0 ? X.nx : X.ny, nb = AX == 0 ? X.ny : X.nx;
    const float qa = q[AX], qb = q[BX], qz = q[2];
    const float F0a = F0[AX], F1a = F1[AX];
    const float F0b = F0[BX], F1b = F1[BX];
    const float ca = T.c[AX];
    const float ua0 = F0a - qa, ua1 = F1a - qa;
    const float iua0 = ua0 != 0.0f ? __builtin_amdgcn_rcpf(ua0) : 0.0f;
    const float iua1 = ua1 != 0.0f ? __builtin_amdgcn_rcpf(ua1) : 0.0f;
    const float vb0 = F0b - qb, vb1 = F1b - qb;
    const float wz0 = F0[2] - qz, wz1 = F1[2] - qz;
    const float amin = fminf(qa, F0a), amax = fmaxf(qa, F1a);
    const float gend_a = na * X.cs, gend_b = nb * X.cs;
    if (!(amax >= 0.0f && amin < gend_a)) return;
    {
    const int ia_lo = max(0, min(na - 1, (int)floorf(amin * X.inv_cs)));
    const int ia_hi = max(0, min(na - 1, (int)floorf(amax * X.inv_cs)));
    const int step = (qa <= ca) ? -1 : 1;
    const int ia_first = step < 0 ? ia_hi : ia_lo;
    const int n_slabs = ia_hi - ia_lo + 1;

    for (int base = 0; base < n_slabs; base += 64) {
        // lane l prepares slab base + l: the rectangles (1-l) q + l F meeting
        // the slab [A0, A1] along axis a give the corridor's extent [bl, bh]
        // along b and its lowest point zf there.
        const int ia_l = ia_first + step * (base + lane);
        bool ok = base + lane < n_slabs;
        const float A0 = ia_l * X.cs, A1 = A0 + X.cs;
        float l0 = 0.0f, l1 = 1.0f;
        const float r1 = A1 - qa, r2 = A0 - qa;
        if (ua0 > 0.0f) l1 = fminf(l1, r1 * iua0);
        else if (ua0 < 0.0f) l0 = fmaxf(l0, r1 * iua0);
        else ok = ok && r1 >= 0.0f;
        if (ua1 > 0.0f) l0 = fmaxf(l0, r2 * iua1);
        else if (ua1 < 0.0f) l1 = fminf(l1, r2 * iua1);
        else ok = ok && r2 <= 0.0f;
        l0 = fmaxf(0.0f, l0 - kLambdaMargin);
        l1 = fminf(1.0f, l1 + kLambdaMargin);
        ok = ok && l0 <= l1;
        const float bl = fminf(qb + l0 * vb0, qb + l1 * vb0) - kWalkMargin;
        const float bh = fmaxf(qb + l0 * vb1, qb + l1 * vb1) + kWalkMargin;
        ok = ok && bh >= 0.0f && bl < gend_b;
        const float zf = DIM == 3 ? fminf(qz + l0 * wz0, qz + l1 * wz0) - kWalkMargin : 0.0f;
        const float zc = DIM == 3 ? fmaxf(qz + l0 * wz1, qz + l1 * wz1) + kWalkMargin : 0.0f;
        const int ib0_l = max(0, min(nb - 1, (int)floorf(bl * X.inv_cs)));
        const int ib1_l = max(0, min(nb - 1, (int)floorf(bh * X.inv_cs)));
        // the corridor's slice, in ordered-integer form: its extent along b
        // (along a, every box listed in the slab's columns reaches the slab,
        // up to the insertion margin) and its floor and ceiling
        const unsigned ub0_l = ord(bl), ub1_l = ord(bh);
        const unsigned zf_l = ord(zf), zc_l = DIM == 3 ? ord(zc) : 0x7f800000u;
        const int ibp_l = ib0_l | (ib1_l << 16);
        unsigned long long todo = __ballot(ok);
        while (todo) {
            const int sl = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int ia = ia_first + step * (base + sl);
            const int ibp = __builtin_amdgcn_readlane(ibp_l, sl);
            const int ib0 = ibp & 0xffff, ib1 = static_cast<int>(static_cast<unsigned>(ibp) >> 16);
            const unsigned ub0 = __builtin_amdgcn_readlane(ub0_l, sl);
            const unsigned ub1 = __builtin_amdgcn_readlane(ub1_l, sl);
            const unsigned uzf = __builtin_amdgcn_readlane(zf_l, sl);
            const unsigned uzc = __builtin_amdgcn_readlane(zc_l, sl);
            const float A0s = ia * X.cs, A1s = A0s + X.cs;
            for (int ib = ib0; ib <= ib1; ++ib) {
                const int col = AX == 0 ? ia + X.nx * ib : ib + X.nx * ia;
                if (STATS) ++ws.cols;
                // The column's records, 64 at a time, lane l holding record
                // base + l (the sentinel past the list's end: its top is below
                // every floor).  Every coordinate of the index frame is a
                // non-negative float below 2^31 as an integer, so a signed
                // difference of two of them has the sign of their comparison.
                const int cb = col_start[col], ce = col_start[col + 1] - 1;
                for (int base = cb;; base += 64) {
                    const BoxRec R = recs[min(base + lane, ce)];
                    // not below the corridor's lowest point (the list is
                    // sorted by decreasing top; 2-D boxes have an infinite top)
                    const bool above = static_cast<int>(__float_as_uint(R.hi[2]) - uzf) >= 0;
                    // and neither beside the slice nor above its ceiling
                    const int side = static_cast<int>(__float_as_uint(R.hi[BX]) - ub0) |
                                     static_cast<int>(ub1 - __float_as_uint(R.lo[BX])) |
                                     (DIM == 3 ? static_cast<int>(uzc - __float_as_uint(R.lo[2])) : 0);
                    unsigned long long cand = __ballot(above && side >= 0);
                    const unsigned long long below = __ballot(!above);
                    // the records up to the first one below the floor
                    if (STATS) ws.recs += __popcll(__ballot(above)) + (below ? 1 : 0);
                    if (cand) {
                        if (STATS) ws.narrow += __popcll(cand);
                        // Narrower: the corridor over only the part of the
                        // slab that the box spans along a (the slab's bounds
                        // over a shorter interval).  The rays can meet the
                        // box only there, and a box that misses the slab is
                        // listed in the columns where it lies.
                        const float ca0 = fmaxf(R.lo[AX], A0s), ca1 = fminf(R.hi[AX], A1s);
                        const float s1 = ca1 - qa, s2 = ca0 - qa;
                        float m0 = 0.0f, m1 = 1.0f;
                        bool tight = ca0 <= ca1;
                        if (ua0 > 0.0f) m1 = fminf(m1, s1 * iua0);
                        else if (ua0 < 0.0f) m0 = fmaxf(m0, s1 * iua0);
                        else tight = tight && s1 >= 0.0f;
                        if (ua1 > 0.0f) m0 = fmaxf(m0, s2 * iua1);
                        else if (ua1 < 0.0f) m1 = fminf(m1, s2 * iua1);
                        else tight = tight && s2 <= 0.0f;
                        m0 = fmaxf(0.0f, m0 - kLambdaMargin);
                        m1 = fminf(1.0f, m1 + kLambdaMargin);
                        // every condition evaluated (no divergent branches)
                        const bool e0 = m0 <= m1;
                        const bool e1 = R.hi[BX] >= fminf(qb + m0 * vb0, qb + m1 * vb0) - kWalkMargin;
                        const bool e2 = R.lo[BX] <= fmaxf(qb + m0 * vb1, qb + m1 * vb1) + kWalkMargin;
                        bool e3 = true, e4 = true;
                        if (DIM == 3) {
                            e3 = R.hi[2] >= fminf(qz + m0 * wz0, qz + m1 * wz0) - kWalkMargin;
                            e4 = R.lo[2] <= fmaxf(qz + m0 * wz1, qz + m1 * wz1) + kWalkMargin;
                        }
                        tight = tight & e0 & e1 & e2 & e3 & e4;
                        cand &= __ballot(tight);
                    }
                    if (cand) {
                        float dl[3], dh[3];
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            dl[k] = R.lo[k] - q[k];
                            dh[k] = R.hi[k] - q[k];
                        }
                        // a candidate's corners relative to q, from its
                        // lane through the LDS crossbar (ds_bpermute) rather
                        // than six v_readlane: the vector ALU is the
                        // kernel's limit and the crossbar is idle
                        auto fetch = [&](int r, float (&lq)[3], float (&hq)[3]) {
#pragma unroll
                            for (int k = 0; k < 3; ++k) {
                                lq[k] = __int_as_float(__builtin_amdgcn_ds_bpermute(r << 2, __float_as_int(dl[k])));
                                hq[k] = __int_as_float(__builtin_amdgcn_ds_bpermute(r << 2, __float_as_int(dh[k])));
                            }
                        };
                        // FULL mode fetches one candidate ahead (measured
                        // faster; in FRACTION mode the registers it holds
                        // cost more than the wait it hides)
                        float nlq[3], nhq[3];
                        if constexpr (MODE == VCM_FULL) fetch(__builtin_ctzll(cand), nlq, nhq);
                        do {
                            const int r = __builtin_ctzll(cand);
                            cand &= cand - 1;
                            float blq[3], bhq[3];
                            if constexpr (MODE == VCM_FULL) {
#pragma unroll
                                for (int k = 0; k < 3; ++k) {
                                    blq[k] = nlq[k];
                                    bhq[k] = nhq[k];
                                }
                                if (cand) fetch(__builtin_ctzll(cand), nlq, nhq);
                            } else {
                                fetch(r, blq, bhq);
                            }
                            const unsigned long long rest = box_test<DIM, NS, EXACT64, MODE, STATS, TAB>(
                                blq, bhq, T, P, q, faces, tab, iv, sidx, open, zmask, ws, n_disagree);
                            if (rest == 0) {
                                if (MODE == VCM_FULL) blk = base + r;
                                return;
                            }
                        } while (cand);
                    }
                    if (below) break;
                }
                // FRACTION mode: pack the unresolved rays into fewer slots
                if (NS > 1 && MODE == VCM_FRACTION) {
                    int tot = 0, used = 0;
#pragma unroll
                    for (int j = 0; j < NS; ++j) {
                        tot += __popcll(open[j]);
                        used += open[j] != 0;
                    }
                    if (((tot + 63) >> 6) < used) {
                        int pos = 0;
#pragma unroll
                        for (int j = 0; j < NS; ++j) {
                            if ((open[j] >> lane) & 1) {
                                if constexpr (NS <= 3)
                                    lds[pos + mbcnt(open[j])] =
                                        make_float4(iv[j][0], iv[j][1], iv[j][2], __int_as_float(sidx[j]));
                                else
                                    lds[pos + mbcnt(open[j])] = sidx[j];
                            }
                            pos += __popcll(open[j]);
                        }
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                        for (int j = 0; j < NS; ++j) {
                            const bool live = j * 64 + lane < tot;
                            bool zl = false;
                            if constexpr (NS <= 3) {
                                const float4 r = lds[live ? j * 64 + lane : 0];
                                sidx[j] = __float_as_int(r.w);
                                iv[j][0] = r.x;
                                iv[j][1] = r.y;
                                iv[j][2] = r.z;
                                // a zero direction component has reciprocal 0
#pragma unroll
                                for (int k = 0; k < DIM; ++k) zl = zl || iv[j][k] == 0.0f;
                            } else {
                                sidx[j] = live ? lds[j * 64 + lane] : 0;
                                float sp[3];
                                zl = ray_setup<DIM, TAB>(T, faces, q, sidx[j], sp, iv[j], tab);
                            }
                            open[j] = __ballot(live);
                            zmask[j] = __ballot(zl) & open[j];
                        }
                        __builtin_amdgcn_wave_barrier();
                    }
                }
            }
        }
    }
    }
}

// Is q inside (or on) an obstacle?  Boxes of the index frame have no
// negative coordinate, so the scan of q's column compares ordered bit
// patterns, 64 records at a time; the column's list ends with a sentinel
// (top -inf, lower corner +inf).
template <int DIM, bool STATS>
__device__ __attribute__((always_inline)) inline bool inside_obstacle(const DevIndex &X, cptr_i32 col_start,
                                                                      cptr_rec recs, const float *q,
                                                                      WaveStats &ws) {
    const int lane = threadIdx.x & 63;
    if (!(q[0] >= 0.0f && q[1] >= 0.0f && q[2] >= 0.0f)) return false;
    const int cx = static_cast<int>(floorf(q[0] * X.inv_cs));
    const int cy = static_cast<int>(floorf(q[1] * X.inv_cs));
    if (!(cx < X.nx && cy < X.ny)) return false;
    const unsigned u0 = __builtin_amdgcn_readfirstlane(ord(q[0]));
    const unsigned u1 = __builtin_amdgcn_readfirstlane(ord(q[1]));
    const unsigned u2 = __builtin_amdgcn_readfirstlane(ord(q[2]));
    const int cb = col_start[cx + X.nx * cy], ce = col_start[cx + X.nx * cy + 1] - 1;
    for (int base = cb;; base += 64) {
        const BoxRec R = recs[min(base + lane, ce)];
        // not lower than q (the list is sorted by decreasing top)
        const bool above = static_cast<int>(__float_as_uint(R.hi[2]) - u2) >= 0;
        const int out = static_cast<int>(u0 - __float_as_uint(R.lo[0])) |
                        static_cast<int>(__float_as_uint(R.hi[0]) - u0) |
                        static_cast<int>(u1 - __float_as_uint(R.lo[1])) |
                        static_cast<int>(__float_as_uint(R.hi[1]) - u1) |
                        (DIM == 3 ? static_cast<int>(u2 - __float_as_uint(R.lo[2])) : 0);
        const unsigned long long below = __ballot(!above);
        if (STATS) ws.recs += __popcll(__ballot(above)) + (below ? 1 : 0);
        if (__ballot(above && out >= 0)) {
            if (STATS) ++ws.inside;
            return true;
        }
        if (below) return false;
    }
}

// Visibility of the live samples from q for one wavefront.  Returns the
// number of unblocked live samples (FULL mode: exact only when it equals N).
//
// A column's box records are read 64 at a time, one per lane, and the
// records that cannot meet the corridor (top below its lowest point, beside
// its extent along b, or above its ceiling) are rejected by integer compares
// on the lanes; the candidates are then tested one by one against every ray
// of the wave, their corners handed over by lane reads.
template <int DIM, int NS, bool EXACT64, int MODE, bool STATS, int TAB>
__device__ __attribute__((always_inline)) inline int trace_viewpoint(
    const BruteArgs &A, cptr_i32 col_start, cptr_rec recs, const float *q, unsigned faces,
    int N, RaySlot<NS> *lds, const void *tab, int &blk, WaveStats &ws,
    unsigned long long &n_disagree) {
    const TargetDesc &T = A.tgt;
    const ParamDesc &P = A.prm;
    const DevIndex &X = A.idx;
    const int lane = threadIdx.x & 63;

    // FULL mode: the box that blocked the previous viewpoint of this work
    // item usually blocks this one too, and one blocked ray settles the
    // viewpoint; each slot is tested against it as soon as it is set up, so
    // a viewpoint settled by an early slot sets up no more rays.  A viewpoint
    // inside an obstacle sees nothing, which is also what a blocked ray
    // gives in FULL mode, so with a cached blocker the column scan for it
    // waits until the blocker has failed to settle the viewpoint.
    const bool cached = MODE == VCM_FULL && blk >= 0;
    if (!cached && inside_obstacle<DIM, STATS>(X, col_start, recs, q, ws)) return 0;

    // ---- rays: slot j, lane l holds live sample j*64 + l
    float iv[NS][3];
    int sidx[NS];
    unsigned long long open[NS];
    unsigned long long zmask[NS];  // rays with a zero direction component
    float bl[3] = {0.0f, 0.0f, 0.0f}, bh[3] = {0.0f, 0.0f, 0.0f};
    if (cached) {
        const BoxRec B = recs[blk];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            bl[k] = B.lo[k] - q[k];
            bh[k] = B.hi[k] - q[k];
        }
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        sidx[j] = j * 64 + lane;
        const bool live = sidx[j] < N;
        float sp[3];
        const bool zl = ray_setup<DIM, TAB>(T, faces, q, live ? sidx[j] : 0, sp, iv[j], tab);
        open[j] = __ballot(live);
        zmask[j] = __ballot(zl) & open[j];
        if (cached && open[j] &&
            slot_hits<DIM, NS, EXACT64, STATS, TAB>(j, bl, bh, T, P, q, faces, tab, iv, sidx, open, zmask, ws,
                                                    n_disagree) != 0)
            return 0;
    }
    if (cached && inside_obstacle<DIM, STATS>(X, col_start, recs, q, ws)) return 0;

    // ---- corridor walk along the major horizontal axis of q - c
    if (fabsf(T.c[0] - q[0]) >= fabsf(T.c[1] - q[1]))
        corridor_walk<DIM, NS, EXACT64, MODE, STATS, TAB, 0>(A, recs, col_start, q, faces, lds, tab, blk, iv,
                                                             sidx, open, zmask, ws, n_disagree);
    else
        corridor_walk<DIM, NS, EXACT64, MODE, STATS, TAB, 1>(A, recs, col_start, q, faces, lds, tab, blk, iv,
                                                             sidx, open, zmask, ws, n_disagree);
    int vis = 0;
#pragma unroll
    for (int j = 0; j < NS; ++j) vis += __popcll(open[j]);
    return vis;
}

// Work items are kXcd contiguous ranges of the item list.  Workgroups are
// dispatched to the XCDs in round-robin order, so a wavefront first drains
// the range of its own XCD and then helps the others: neighbouring items are
// then written through the same L2, which merges their partial cache lines
// before they reach HBM.  Every range counter only grows, so each wavefront
// leaves after at most kXcd exhausted ranges.
__device__ inline unsigned range_begin(unsigned n, int r) {
    return static_cast<unsigned>((static_cast<unsigned long long>(n) * r) / kXcd);
}

// Work-item dispenser of one wavefront.  (Issuing the next claim before
// processing the current item, to hide the atomic's latency, measured slower:
// the claim result stays live across the item and the loop's memory waits
// cover it anyway.)
struct Dispenser {
    unsigned *ctr;
    unsigned n;
    int r, left;

    __device__ void init(unsigned *c, unsigned n_items) {
        ctr = c;
        n = n_items;
        r = blockIdx.x % kXcd;
        left = kXcd;
    }
    __device__ bool next(unsigned &item) {
        while (left > 0) {
            unsigned i = 0;
            if ((threadIdx.x & 63) == 0) i = atomicAdd(&ctr[r * kCtrStride], 1u);
            i = __builtin_amdgcn_readfirstlane(__shfl(i, 0));
            const unsigned b = range_begin(n, r), e = range_begin(n, r + 1);
            if (i < e - b) {
                item = b + i;
                return true;
            }
            r = (r + 1) % kXcd;
            --left;
        }
        return false;
    }
};

// One work item of a query: A.chunk consecutive viewpoints of one grid row,
// each traced by the whole wavefront; the results are written by A.chunk
// lanes at once.  `item` counts from the start of the query's items.
template <int DIM, int NS, bool EXACT64, int MODE, bool STATS, int TAB>
__device__ __attribute__((always_inline)) inline void run_item(const BruteArgs &A, cptr_i32 col_start,
                                                               cptr_rec recs, unsigned item, RaySlot<NS> *lds,
                                                               const void *tab, WaveStats &ws,
                                                               unsigned long long &n_disagree) {
    using R = typename std::conditional<EXACT64, double, float>::type;
    const int lane = threadIdx.x & 63;
    const TargetDesc &T = A.tgt;
    const ParamDesc &P = A.prm;
    const int n0 = A.grid.n[0], n1 = A.grid.n[1];
    const int chunk = A.chunk;
    const int cpr = (n0 + chunk - 1) / chunk;
    const int row = static_cast<int>(item / static_cast<unsigned>(cpr));
    const int x0 = static_cast<int>(item - static_cast<unsigned>(row) * cpr) * chunk;
    const int jj = row % n1, kk = A.k_begin + row / n1;
    const int nv = min(chunk, n0 - x0);
    const int64_t v0 = x0 + static_cast<int64_t>(n0) * (jj + static_cast<int64_t>(n1) * kk);
    // lane t keeps the counts of viewpoint t of the item
    int o_cnt = 0, o_n = 0;
    bool o_fov = false;
    int blk = -1;  // record of the last blocking box (FULL mode)
    // fill mode: lane t holds the gate word the block tree left for
    // viewpoint t; only undecided viewpoints are traced and written
    uint32_t pre = kGateUndecided;
    if (A.fill && lane < nv) pre = A.gate[v0 + lane];
    for (int t = 0; t < nv; ++t) {
        if (A.fill && static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(pre), t)) != kGateUndecided)
            continue;
        if (STATS && A.fill) ++ws.filled;
        // grid index; in gate mode the launch grid is the block grid and
        // each block is represented by its lowest-index centre viewpoint
        int ii[3] = {x0 + t, jj, kk};
        if (A.gate) {
#pragma unroll
            for (int k = 0; k < 3; ++k)
                ii[k] = min(ii[k] * A.theta + (A.theta - 1) / 2, A.full_n[k] - 1);
        }
        float q[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            q[k] = (k < DIM) ? A.grid.o[k] + static_cast<float>(2 * ii[k] + 1) * A.grid.h2[k] : 0.0f;
            // FRACTION mode keeps more rays live: q in scalar registers
            // leaves vector registers to them (measured: less spilling)
            if (MODE == VCM_FRACTION) q[k] = uniform_f(q[k]);
        }
        // live facets packed 4 bits each: cube faces whose outer side
        // contains q strictly (code 2k+1 for +k, 2k for -k)
        unsigned faces = 0;
        int nf = 0;
        if (T.kind == VCM_CUBE) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const bool up = q[k] > T.c[k] + T.half[k];
                const bool dn = q[k] < T.c[k] - T.half[k];
                if (up || dn) {
                    faces |= static_cast<unsigned>(2 * k + (up ? 1 : 0)) << (4 * nf);
                    ++nf;
                }
            }
        } else {
            nf = 1;
        }
        const int N = nf * T.per_facet;
        const bool fov = in_fov<DIM>(T, P, q);
        int cnt = 0;
        if (fov && N > 0) {
            if (STATS) ws.rays += N;
            const int vis = trace_viewpoint<DIM, NS, EXACT64, MODE, STATS, TAB>(
                A, col_start, recs, q, faces, N, lds, tab, blk, ws, n_disagree);
            // FRACTION mode: the visible samples; FULL mode: N when all are
            cnt = MODE == VCM_FRACTION ? vis : (vis == N ? N : 0);
        }
        if (lane == t) {
            o_cnt = cnt;
            o_n = N;
            o_fov = fov;
        }
    }
    if (lane < nv) {
        if (A.gate) {
            if (pre == kGateUndecided)
                A.gate[v0 + lane] = static_cast<uint32_t>(o_cnt) | (static_cast<uint32_t>(o_n) << 10) |
                                    (o_fov ? (1u << 20) : 0u);
        } else {
            // measure and bin, one lane per viewpoint of the item (the lane
            // computes its viewpoint's position exactly as the walk did)
            float q[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int ik = k == 0 ? x0 + lane : (k == 1 ? jj : kk);
                q[k] = (k < DIM) ? A.grid.o[k] + static_cast<float>(2 * ik + 1) * A.grid.h2[k] : 0.0f;
            }
            R col;
            int bn;
            colour_and_bin<DIM, R, MODE>(T, P, q, o_cnt, o_n, col, bn);
            A.bin[v0 + lane] = static_cast<uint8_t>(bn);
            if (A.c) A.c[v0 + lane] = static_cast<float>(col);
            if (A.count) A.count[v0 + lane] = static_cast<uint16_t>(o_cnt);
        }
    }
}

template <bool STATS>
__device__ inline void flush_stats(DevStats *st, const WaveStats &ws, unsigned long long n_disagree) {
    if (!STATS) return;
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&st->rays, ws.rays);
        atomicAdd(&st->box_tests, ws.tests);
        atomicAdd(&st->slot_tests, ws.slots);
        atomicAdd(&st->rechecks, ws.rechecks);
        atomicAdd(&st->columns, ws.cols);
        atomicAdd(&st->inside_box, ws.inside);
        atomicAdd(&st->records, ws.recs);
        atomicAdd(&st->narrow_tests, ws.narrow);
        if (ws.filled) atomicAdd(&st->leaves, ws.filled);
    }
    if (n_disagree) atomicAdd(&st->fp32_disagree, n_disagree);  // per lane
}

// Occupancy target of the ray kernels (waves per SIMD): the register budget
// it leaves decides how much the compiler spills.  Six in both modes
// (measured against five and seven: five leaves too few waves to hide the
// walk's latencies, seven spills more than the extra wave gains).  The
// batched kernel, whose FULL-mode queries are mostly small maps, keeps a
// seventh wave in FULL mode (measured: 5.3 G viewpoints/s at six, 5.6 G at
// seven).
template <int MODE>
constexpr int kWaves = 6;
template <int MODE>
constexpr int kBatchWaves = MODE == VCM_FULL ? 7 : 6;

// One query: persistent wavefronts take the query's work items.
template <int DIM, int NS, bool EXACT64, int MODE, bool STATS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kWaves<MODE>, 8))) void k_brute(BruteArgs A, const int32_t *col_start_g,
                                               const BoxRec *recs_g) {
    // same kernel symbol in both compiler passes; constant-space view inside
    const cptr_i32 col_start = (cptr_i32)col_start_g;
    const cptr_rec recs = (cptr_rec)recs_g;
    __shared__ RaySlot<NS> lds_rays[4][NS * 64];
    __shared__ float4 s_tab[kTableMax];
    build_sample_table<DIM>(A.tgt, s_tab);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    RaySlot<NS> *lds = lds_rays[wave];
    WaveStats ws;
    unsigned long long n_disagree = 0;
    Dispenser D;
    D.init(A.counter, A.n_items);
    unsigned item;
    while (D.next(item))
        run_item<DIM, NS, EXACT64, MODE, STATS, kTabBlock>(A, col_start, recs, item, lds, s_tab, ws, n_disagree);
    flush_stats<STATS>(A.stats, ws, n_disagree);
}

// Many queries on one index in one launch.  The work items of all queries
// form one list (query after query) in groups of four items of one query.  A
// workgroup claims a group, one item per wavefront, so that its wavefronts
// share one sample table in LDS, rebuilt when the workgroup moves to another
// query; neighbouring viewpoints cost about the same, so the wavefronts wait
// little for one another at the end of a group.  The query of a group is
// found by binary search over the queries' group ends; its record is read
// from constant memory (scalar loads).
template <int DIM, int NS, bool EXACT64, int MODE, bool STATS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kBatchWaves<MODE>, 8))) void k_brute_batch(
    BatchArgs B, const BruteArgs *qs_g, const uint32_t *group_end_g, const int32_t *col_start_g,
    const BoxRec *recs_g) {
    const cptr_i32 col_start = (cptr_i32)col_start_g;
    const cptr_rec recs = (cptr_rec)recs_g;
    const VCM_CONST BruteArgs *qs = (const VCM_CONST BruteArgs *)qs_g;
    const VCM_CONST uint32_t *group_end = (const VCM_CONST uint32_t *)group_end_g;
    __shared__ RaySlot<NS> lds_rays[4][NS * 64];
    __shared__ float4 s_tab[kTableMax];
    __shared__ unsigned s_group;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    RaySlot<NS> *lds = lds_rays[wave];
    int cur_q = -1;  // query whose samples the table holds (workgroup-uniform)
    WaveStats ws;
    unsigned long long n_disagree = 0;
    Dispenser D;  // claims by wavefront 0 for the workgroup
    D.init(B.counter, B.n_items);
    for (;;) {
        if (wave == 0) {
            unsigned g = 0;
            const bool got = D.next(g);
            if ((threadIdx.x & 63) == 0) s_group = got ? g : 0xffffffffu;
        }
        __syncthreads();
        const unsigned group = __builtin_amdgcn_readfirstlane(s_group);
        if (group == 0xffffffffu) break;
        int lo = 0, hi = B.nq - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (group_end[mid] > group) hi = mid;
            else lo = mid + 1;
        }
        const unsigned begin = lo > 0 ? group_end[lo - 1] : 0u;
        // a generic reference derived from the constant-space pointer: the
        // compiler turns the field reads back into scalar constant loads
        // (a local copy of the record would live in scratch memory)
        const BruteArgs &A = *reinterpret_cast<const BruteArgs *>(qs + lo);
        if (lo != cur_q) {
            build_sample_table<DIM>(A.tgt, s_tab);  // ends with a workgroup barrier
            cur_q = lo;
        }
        const unsigned item = (group - begin) * 4u + static_cast<unsigned>(wave);
        if (item < A.n_items)
            run_item<DIM, NS, EXACT64, MODE, STATS, kTabBlock>(A, col_start, recs, item, lds, s_tab, ws,
                                                                n_disagree);
        __syncthreads();  // the table and s_group are reused next round
    }
    flush_stats<STATS>(B.stats, ws, n_disagree);
}

// The undecided smallest blocks of the visible-region tree (blocks.hip): each
// takes the gate of its representative viewpoint -- the lowest-index centre
// viewpoint of the block -- traced like any viewpoint, for all the
// viewpoints it holds.  One wavefront per block.
constexpr int kLeafRun = 8;

// Every word of p set to v (grid-stride).
__global__ void k_fill_words(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

struct LeafArgs {
    const uint32_t *list;   // blocks (index in the leaf level's block grid)
    const unsigned *count;  // entries of list
    unsigned *claim;        // work counter (cleared)
    int32_t side;           // viewpoints per block edge
    int32_t nb[3];          // blocks per axis
    int32_t run;            // entries a wavefront claims at once
};

template <int DIM, int NS, bool EXACT64, int MODE, bool STATS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kWaves<MODE>, 8))) void k_leaves(
    BruteArgs A, const int32_t *col_start_g, const BoxRec *recs_g, LeafArgs LA) {
    const cptr_i32 col_start = (cptr_i32)col_start_g;
    const cptr_rec recs = (cptr_rec)recs_g;
    __shared__ RaySlot<NS> lds_rays[4][NS * 64];
    __shared__ float4 s_tab[kTableMax];
    build_sample_table<DIM>(A.tgt, s_tab);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    RaySlot<NS> *lds = lds_rays[wave];
    const int lane = threadIdx.x & 63;
    const TargetDesc &T = A.tgt;
    const ParamDesc &P = A.prm;
    WaveStats ws;
    unsigned long long n_disagree = 0, n_leaves = 0;
    const unsigned n_in = *LA.count;
    // A wavefront claims LA.run consecutive entries at once: the sub-blocks
    // an undecided block hands down sit next to each other in the list, so
    // the box that blocked one leaf (FULL mode) is tried first on the next.
    const unsigned run = static_cast<unsigned>(LA.run);
    int blk = -1;
    unsigned item = 0, end = 0;
    for (;;) {
        if (item >= end) {
            unsigned first = 0;
            if (lane == 0) first = atomicAdd(LA.claim, run);
            first = __builtin_amdgcn_readfirstlane(__shfl(first, 0));
            if (first >= n_in) break;
            item = first;
            end = min(n_in, first + run);
        }
        const uint32_t b = LA.list[item++];
        const int bi[3] = {static_cast<int>(b % static_cast<uint32_t>(LA.nb[0])),
                           static_cast<int>((b / static_cast<uint32_t>(LA.nb[0])) % static_cast<uint32_t>(LA.nb[1])),
                           static_cast<int>(b / (static_cast<uint32_t>(LA.nb[0]) * static_cast<uint32_t>(LA.nb[1])))};
        int lo[3], hi[3];
        float q[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lo[k] = k < DIM ? bi[k] * LA.side : 0;
            hi[k] = k < DIM ? min(lo[k] + LA.side, A.grid.n[k]) - 1 : 0;
            const int r = lo[k] + min((LA.side - 1) / 2, hi[k] - lo[k]);
            q[k] = k < DIM ? uniform_f(A.grid.o[k] + static_cast<float>(2 * r + 1) * A.grid.h2[k]) : 0.0f;
        }
        unsigned faces = 0;
        int nf = 0;
        if (T.kind == VCM_CUBE) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const bool up = q[k] > T.c[k] + T.half[k];
                const bool dn = q[k] < T.c[k] - T.half[k];
                if (up || dn) {
                    faces |= static_cast<unsigned>(2 * k + (up ? 1 : 0)) << (4 * nf);
                    ++nf;
                }
            }
        } else {
            nf = 1;
        }
        const int N = nf * T.per_facet;
        const bool fov = in_fov<DIM>(T, P, q);
        int cnt = 0;
        if (fov && N > 0) {
            if (STATS) ws.rays += N;
            const int vis = trace_viewpoint<DIM, NS, EXACT64, MODE, STATS, kTabBlock>(
                A, col_start, recs, q, faces, N, lds, s_tab, blk, ws, n_disagree);
            cnt = MODE == VCM_FRACTION ? vis : (vis == N ? N : 0);
        }
        ++n_leaves;
        const uint32_t word = static_cast<uint32_t>(cnt) | (static_cast<uint32_t>(N) << 10) | (fov ? (1u << 20) : 0u);
        const int e0 = hi[0] - lo[0] + 1, e1 = hi[1] - lo[1] + 1, e2 = hi[2] - lo[2] + 1;
        for (int t = lane; t < e0 * e1 * e2; t += 64) {
            const int i = lo[0] + t % e0, j = lo[1] + (t / e0) % e1, k = lo[2] + t / (e0 * e1);
            A.gate[i + static_cast<int64_t>(A.grid.n[0]) * (j + static_cast<int64_t>(A.grid.n[1]) * k)] = word;
        }
    }
    flush_stats<STATS>(A.stats, ws, n_disagree);
    if (STATS && lane == 0) atomicAdd(&A.stats->leaves, n_leaves);
}

__global__ void k_zero_counter(unsigned *c) {
    if (threadIdx.x < kXcd) c[threadIdx.x * kCtrStride] = 0u;
}

struct Launch {
    dim3 grid;
    bool stats;
    hipStream_t st;
};

// Compile-time variant of the ray kernels.
template <int DIM_, int NS_, bool E_, int MODE_, bool ST_>
struct Variant {
    static constexpr int DIM = DIM_, NS = NS_, MODE = MODE_;
    static constexpr bool E = E_, ST = ST_;
};

template <int DIM, int NS, bool E, int MODE, class F>
void dispatch_stats(bool stats, F &&f) {
    if (stats) f(Variant<DIM, NS, E, MODE, true>{});
    else f(Variant<DIM, NS, E, MODE, false>{});
}
template <int DIM, int NS, bool E, class F>
void dispatch_mode(int mode, bool stats, F &&f) {
    if (mode == VCM_FULL) dispatch_stats<DIM, NS, E, VCM_FULL>(stats, f);
    else dispatch_stats<DIM, NS, E, VCM_FRACTION>(stats, f);
}
// Solo launches: a kernel per slot count.
template <int DIM, bool E, class F>
void dispatch_ns_all(int ns, int mode, bool stats, F &&f) {
    switch (ns) {
        case 1: dispatch_mode<DIM, 1, E>(mode, stats, f); break;
        case 2: dispatch_mode<DIM, 2, E>(mode, stats, f); break;
        case 3: dispatch_mode<DIM, 3, E>(mode, stats, f); break;
        case 4: dispatch_mode<DIM, 4, E>(mode, stats, f); break;
        case 5: dispatch_mode<DIM, 5, E>(mode, stats, f); break;
        default: dispatch_mode<DIM, 6, E>(mode, stats, f); break;
    }
}
// Batched launches: slot counts rounded up to 2, 3 or 6 (empty slots cost a
// scalar branch per box).
template <int DIM, bool E, class F>
void dispatch_ns_batch(int ns, int mode, bool stats, F &&f) {
    if (ns <= 2) dispatch_mode<DIM, 2, E>(mode, stats, f);
    else if (ns == 3) dispatch_mode<DIM, 3, E>(mode, stats, f);
    else dispatch_mode<DIM, 6, E>(mode, stats, f);
}
template <bool BATCH, class F>
void dispatch(int dim, bool fp64, int ns, int mode, bool stats, F &&f) {
    if (dim == 2) {
        if (fp64) BATCH ? dispatch_ns_batch<2, true>(ns, mode, stats, f) : dispatch_ns_all<2, true>(ns, mode, stats, f);
        else BATCH ? dispatch_ns_batch<2, false>(ns, mode, stats, f) : dispatch_ns_all<2, false>(ns, mode, stats, f);
    } else {
        if (fp64) BATCH ? dispatch_ns_batch<3, true>(ns, mode, stats, f) : dispatch_ns_all<3, true>(ns, mode, stats, f);
        else BATCH ? dispatch_ns_batch<3, false>(ns, mode, stats, f) : dispatch_ns_all<3, false>(ns, mode, stats, f);
    }
}

}  // namespace

int device_cus(int device) {
    static int cached[64] = {0};
    if (device < 0 || device >= 64) return 256;
    if (!cached[device]) {
        hipDeviceProp_t prop;
        cached[device] = (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
                             ? prop.multiProcessorCount
                             : 256;
    }
    return cached[device];
}

int slots_for(const TargetDesc &t) {
    const int max_n = t.per_facet * (t.kind == VCM_CUBE ? 3 : 1);
    return (max_n + 63) / 64;
}

BruteArgs make_brute_args(const Index &ix, const TargetDesc &t, const GridDesc &g_in,
                          const ParamDesc &p, const vcm_result &r, uint32_t *gate, int theta,
                          int chunk) {
    BruteArgs a{};
    GridDesc g = g_in;
    a.theta = theta;
    for (int k = 0; k < 3; ++k) a.full_n[k] = g_in.n[k];
    if (gate) {
        // launch over the block grid
        g.count = 1;
        for (int k = 0; k < 3; ++k) {
            g.n[k] = (g_in.n[k] + theta - 1) / theta;
            g.count *= g.n[k];
        }
    }
    a.gate = gate;
    a.idx = ix.dev;
    a.tgt = t;
    a.grid = g;
    a.prm = p;
    a.bin = r.bin;
    a.c = r.c;
    a.count = r.count;
    a.chunk = chunk;
    a.k_begin = 0;
    const uint64_t cpr = (static_cast<uint64_t>(g.n[0]) + chunk - 1) / chunk;
    const uint64_t items = cpr * static_cast<uint64_t>(g.n[1]) * static_cast<uint64_t>(g.n[2]);
    a.n_items = items > 0xffffffffull ? 0xffffffffu : static_cast<uint32_t>(items);
    return a;
}

void launch_zero_counter(unsigned *c, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s, c);
}

vcm_status launch_brute_batch(const Index &ix, bool fp64, int mode, int ns, const BatchArgs &b,
                              const BruteArgs *d_recs, const uint32_t *d_group_end, int blocks,
                              hipStream_t s) {
    if (b.n_items == 0) return VCM_OK;
    launch_zero_counter(b.counter, s);
    const dim3 grid(static_cast<unsigned>(blocks));
    dispatch<true>(ix.dim, fp64, ns, mode, b.stats != nullptr, [&](auto v) {
        using V = decltype(v);
        hipLaunchKernelGGL((k_brute_batch<V::DIM, V::NS, V::E, V::MODE, V::ST>), grid, dim3(256), 0, s, b,
                           d_recs, d_group_end, ix.dev.col_start, ix.dev.recs);
    });
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(VCM_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return VCM_OK;
}

vcm_status launch_leaves(const Index &ix, const TargetDesc &t, const GridDesc &g, const ParamDesc &p,
                         const BlockPlan &bp, uint32_t *gate, const uint32_t *list, const unsigned *count,
                         unsigned *claim, hipStream_t s, DevStats *stats) {
    if (g.count <= 0) return VCM_OK;
    BruteArgs a = make_brute_args(ix, t, g, p, vcm_result{}, nullptr, 1, 1);
    a.gate = gate;
    a.stats = stats;
    const int ns = slots_for(t);
    if (ns < 1 || ns > kMaxSlots) return set_error(VCM_E_INVALID, "too many target samples");
    LeafArgs la{};
    la.list = list;
    la.count = count;
    la.claim = claim;
    la.side = bp.leaf;
    for (int k = 0; k < 3; ++k) la.nb[k] = k < ix.dim ? (g.n[k] + bp.leaf - 1) / bp.leaf : 1;
    // leaves listed with their siblings (the smallest blocks inside an
    // undecided classified block) go in runs, for the blocker cache; leaves
    // that are the classified blocks themselves have no such neighbours and
    // go one by one, which spreads a short list over the device (measured:
    // FRACTION, theta 8: 0.96 -> 0.88 ms; theta 16: 1.78 -> 1.66 ms)
    la.run = bp.leaf < bp.side[bp.classified - 1] ? kLeafRun : 1;
    const int64_t nleaf = bp.count[bp.levels - 1];
    const dim3 grid(static_cast<unsigned>(
        std::max<int64_t>(1, std::min<int64_t>((nleaf + 3) / 4, int64_t(device_cus(ix.device)) * 8))));
    // slot counts rounded up to 2, 3 or 6, as for batches (fewer instances)
    dispatch<true>(ix.dim, p.fp64 != 0, ns, p.mode, stats != nullptr, [&](auto v) {
        using V = decltype(v);
        hipLaunchKernelGGL((k_leaves<V::DIM, V::NS, V::E, V::MODE, V::ST>), grid, dim3(256), 0, s, a,
                           a.idx.col_start, a.idx.recs, la);
    });
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(VCM_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return VCM_OK;
}

void launch_gate_clear(uint32_t *gate, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_words, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, gate, n, kGateUndecided);
}

vcm_status launch_undecided(const Index &ix, const TargetDesc &t, const GridDesc &g, const ParamDesc &p,
                            const BlockPlan &bp, uint32_t *gate, uint32_t *const *lists, unsigned *ctr,
                            unsigned *counter, hipStream_t s, DevStats *stats) {
    if (bp.leaf == 1) return launch_brute(ix, t, g, p, vcm_result{}, s, stats, gate, 1, Tuning{}, counter, 1);
    const int lv = bp.leaf_list;
    return launch_leaves(ix, t, g, p, bp, gate, lists[lv], ctr + lv, ctr + 2 * bp.levels + 1, s, stats);
}

vcm_status launch_brute(const Index &ix, const TargetDesc &t, const GridDesc &g_in,
                        const ParamDesc &p, const vcm_result &r, hipStream_t stream,
                        DevStats *stats, uint32_t *gate, int theta, const Tuning &tune,
                        unsigned *counter, int fill) {
    if (g_in.count <= 0) return VCM_OK;
    const int cus = device_cus(ix.device);
    // viewpoints per work item: the mode's run length, halved while a small
    // map would give fewer work items than the device has SIMDs
    int chunk = chunk_for(tune, p.mode);
    if (tune.chunk <= 0) {
        const int64_t rows = int64_t(g_in.n[1]) * std::max(1, g_in.n[2]);
        while (chunk > 1 && (g_in.n[0] + chunk - 1) / chunk * rows < int64_t(cus) * 4) chunk /= 2;
    }
    BruteArgs a = make_brute_args(ix, t, g_in, p, r, gate, theta, chunk);
    a.stats = stats;
    a.fill = gate && theta == 1 && fill ? 1 : 0;
    const int ns = slots_for(t);
    if (ns < 1 || ns > kMaxSlots) return set_error(VCM_E_INVALID, "too many target samples");
    a.counter = counter;
    const GridDesc &g = a.grid;
    const int64_t cpr = (g.n[0] + a.chunk - 1) / a.chunk;
    const int64_t rows_per_layer = g.n[1];
    // launches over z slabs keep the work-item count within 32 bits
    const int64_t max_layers = std::max<int64_t>(1, (int64_t(1) << 30) / (cpr * rows_per_layer));
    for (int64_t k0 = 0; k0 < g.n[2]; k0 += max_layers) {
        const int64_t nl = std::min<int64_t>(max_layers, g.n[2] - k0);
        a.k_begin = static_cast<int32_t>(k0);
        a.n_items = static_cast<unsigned>(cpr * rows_per_layer * nl);
        const int64_t blocks = std::min<int64_t>((a.n_items + 3) / 4, int64_t(cus) * tune.blocks_per_cu);
        const dim3 grid(static_cast<unsigned>(blocks));
        launch_zero_counter(counter, stream);
        dispatch<false>(ix.dim, p.fp64 != 0, ns, p.mode, stats != nullptr, [&](auto v) {
            using V = decltype(v);
            hipLaunchKernelGGL((k_brute<V::DIM, V::NS, V::E, V::MODE, V::ST>), grid, dim3(256), 0, stream, a,
                               a.idx.col_start, a.idx.recs);
        });
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return set_error(VCM_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    }
    return VCM_OK;
}

}  // namespace vcm
