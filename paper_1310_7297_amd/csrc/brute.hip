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
//   * inside a column, box records are read with wave-uniform (scalar)
//     loads, so one read serves 64 * NS rays, and the list stops at the first
//     box whose top lies below the corridor's lowest point;
//   * each lane runs a float32 slab test per ray; a result within `eps` of
//     the decision boundary is settled by the exact float64 predicate;
//   * visibility is reduced with wave ballots and popcounts (integers only).
#include <cmath>
#include <type_traits>

#include "vcm_internal.h"

namespace vcm {
namespace {

constexpr float kWalkMargin = 1.0f / 128.0f;
constexpr float kLambdaMargin = 1e-6f;

// Exact contact of the closed segment [q, s] with the closed box B.
// All coordinates are multiples of 2^-8 below 2^14, so every difference and
// every product of two differences below is exact in float64.  Along each
// axis the box admits the ray parameters between an entry and an exit
// fraction (numerator / positive denominator); the segment meets the box iff
// no entry exceeds an exit, [0, 1] included, compared by cross-multiplying.
template <int DIM>
__device__ __noinline__ bool exact_contact(float qx, float qy, float qz, float sx, float sy,
                                           float sz, float lx, float ly, float lz, float hx,
                                           float hy, float hz) {
    const double q[3] = {qx, qy, qz}, s[3] = {sx, sy, sz};
    const double lo[3] = {lx, ly, lz}, hi[3] = {hx, hy, hz};
    double en[DIM], ex[DIM], de[DIM];
    bool moving[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const double dk = s[k] - q[k];
        moving[k] = dk != 0.0;
        if (!moving[k]) {
            if (q[k] < lo[k] || q[k] > hi[k]) return false;
            en[k] = 0.0;
            ex[k] = 1.0;
            de[k] = 1.0;
            continue;
        }
        const bool up = dk > 0.0;
        en[k] = up ? lo[k] - q[k] : q[k] - hi[k];
        ex[k] = up ? hi[k] - q[k] : q[k] - lo[k];
        de[k] = fabs(dk);
        if (en[k] > de[k] || ex[k] < 0.0) return false;
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b)
            if (a != b && moving[a] && moving[b] && en[a] * de[b] > ex[b] * de[a]) return false;
    return true;
}

template <int DIM>
__device__ inline bool exact_contact(const float *q, const float *s, const BoxRec &B) {
    return exact_contact<DIM>(q[0], q[1], q[2], s[0], s[1], s[2], B.lo[0], B.lo[1], B.lo[2],
                              B.hi[0], B.hi[1], B.hi[2]);
}

// Lane-private ray data for one slot.
struct Ray {
    float s[3];    // sample position
    float inv[3];  // 1 / (s - q), 0 where the component is 0
    bool zero[3];  // component of s - q is exactly 0
    bool live;
};

// Float32 slab test.  lq = lo - q and hq = hi - q are exact.  Returns the
// entry/exit gap t1 - t0 of the parameter interval the box cuts from [0, 1]:
// the segment meets the box iff the gap is >= 0.  With ZERO the axes whose
// direction component is 0 are handled by containment.
template <int DIM, bool ZERO>
__device__ inline float slab_gap(const Ray &r, const float *lq, const float *hq) {
    float t0 = 0.0f, t1 = 1.0f;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const float a = lq[k] * r.inv[k];
        const float b = hq[k] * r.inv[k];
        float mn = fminf(a, b), mx = fmaxf(a, b);
        if (ZERO) {
            const bool inside = lq[k] <= 0.0f && hq[k] >= 0.0f;
            mn = r.zero[k] ? (inside ? -INFINITY : INFINITY) : mn;
            mx = r.zero[k] ? (inside ? INFINITY : -INFINITY) : mx;
        }
        t0 = fmaxf(t0, mn);
        t1 = fminf(t1, mx);
    }
    return t1 - t0;
}

__device__ inline unsigned long long ballot(bool p) { return __ballot(p); }

template <typename R>
__device__ inline R my_atan2(R y, R x);
template <>
__device__ inline float my_atan2<float>(float y, float x) { return atan2f(y, x); }
template <>
__device__ inline double my_atan2<double>(double y, double x) { return atan2(y, x); }
template <typename R>
__device__ inline R my_atan(R x);
template <>
__device__ inline float my_atan<float>(float x) { return atanf(x); }
template <>
__device__ inline double my_atan<double>(double x) { return atan(x); }

// Visual angle of the target from q (Eq. 1 with the oblique size of Eq. 2),
// divided by its largest value V0.  alpha is measured in the meridian plane:
// h = |Delta . n|, rho = |Delta - (Delta . n) n|, alpha = atan2(h, rho).
template <int DIM, typename R>
__device__ inline R raw_colour(const TargetDesc &T, const ParamDesc &P, const float *q) {
    R dl[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) dl[k] = (k < DIM) ? R(q[k]) - R(T.c[k]) : R(0);
    int nax = T.nax;
    if (T.kind == VCM_CUBE) {
        nax = 0;
        if (fabs(dl[1]) > fabs(dl[nax])) nax = 1;
        if (fabs(dl[2]) > fabs(dl[nax])) nax = 2;
    }
    R h = fabs(dl[nax]);
    R r2 = R(0);
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (k != nax) r2 += dl[k] * dl[k];
    const R rho = sqrt(r2);
    const R D = sqrt(r2 + h * h);
    const R alpha = my_atan2<R>(h, rho);
    const R Sa = alpha * (R(2) / R(M_PI)) * R(T.S);
    const R Dn = D > R(P.d0) ? D : R(P.d0);
    const R V = R(2) * my_atan<R>(Sa / (R(2) * Dn));
    return V / R(P.V0);
}

// Field of view (closed wedge about the normal, apex at the target centre).
// The quantities are exact in float64 for inputs on the 2^-8 lattice.
template <int DIM>
__device__ inline bool in_fov(const TargetDesc &T, const ParamDesc &P, const float *q) {
    if (P.fov_kind == kFovAll) return true;
    double d2 = 0.0, dn = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const double d = double(q[k]) - double(T.c[k]);
        d2 += d * d;
        if (k == T.nax) dn = T.nsign * d;
    }
    if (P.fov_kind == kFovHalf) return dn >= 0.0;
    if (P.fov_kind == kFovNarrow) return dn >= 0.0 && dn * dn >= P.fov_c2 * d2;
    return dn >= 0.0 || dn * dn <= P.fov_c2 * d2;
}

template <int DIM, int NS, bool EXACT64, bool STATS>
__global__ __launch_bounds__(256) void k_brute(BruteArgs A) {
    using R = typename std::conditional<EXACT64, double, float>::type;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t vp = A.vp_begin + static_cast<int64_t>(blockIdx.x) * 4 + wave;
    if (vp >= A.vp_end) return;
    const TargetDesc &T = A.tgt;
    const ParamDesc &P = A.prm;
    const DevIndex &X = A.idx;

    // Viewpoint position (exact).
    const int64_t n0 = A.grid.n[0], n1 = A.grid.n[1];
    const int64_t ii[3] = {vp % n0, (vp / n0) % n1, vp / (n0 * n1)};
    float q[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        q[k] = (k < DIM) ? A.grid.o[k] + static_cast<float>(2 * ii[k] + 1) * A.grid.h2[k] : 0.0f;

    // Live facets: the segment / billboard facet always; cube faces whose
    // outer side contains q strictly.
    int faces[3] = {0, 0, 0};
    int nf = 0;
    if (T.kind == VCM_CUBE) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (q[k] > T.c[k] + T.half[k]) faces[nf++] = 2 * k + 1;
            else if (q[k] < T.c[k] - T.half[k]) faces[nf++] = 2 * k;
        }
    } else {
        nf = 1;
    }
    const int N = nf * T.per_facet;
    const bool fov = in_fov<DIM>(T, P, q);
    const R craw = raw_colour<DIM, R>(T, P, q);

    int visible = 0;
    unsigned long long n_tests = 0, n_rechecks = 0, n_disagree = 0, n_cols = 0;

    if (fov && N > 0) {
        // ---- ray setup: slot j, lane l holds sample j*64 + l
        Ray ray[NS];
        bool blk[NS];
        bool act[NS];   // wave-uniform: some live ray of the slot is unresolved
        bool zro[NS];   // wave-uniform: some ray of the slot has a zero component
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int si = j * 64 + lane;
            Ray &r = ray[j];
            r.live = si < N;
            const int f = r.live ? si / T.per_facet : 0;
            const int w = r.live ? si - f * T.per_facet : 0;
            const int iu = w % T.su, iv = w / T.su;
            const float u = static_cast<float>(2 * iu + 1 - T.su) * T.hu;
            const float v = static_cast<float>(2 * iv + 1 - T.sv) * T.hv;
            float s[3] = {T.c[0], T.c[1], DIM == 3 ? T.c[2] : 0.0f};
            if (T.kind == VCM_CUBE) {
                const int fc = f == 0 ? faces[0] : (f == 1 ? faces[1] : faces[2]);
                const int k = fc >> 1;
                const int ua = (k == 0) ? 1 : 0, vb = (k == 2) ? 1 : 2;
                s[k] = (fc & 1) ? T.c[k] + T.half[k] : T.c[k] - T.half[k];
                s[ua] = T.c[ua] + u;
                s[vb] = T.c[vb] + v;
            } else {
                const int wax = 1 - T.nax;
                s[wax] = T.c[wax] + u;
                if (T.kind == VCM_BILLBOARD) s[2] = T.c[2] + v;
            }
            bool anyzero = false;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                r.s[k] = s[k];
                const float d = s[k] - q[k];
                r.zero[k] = (k < DIM) && d == 0.0f;
                r.inv[k] = (k < DIM && d != 0.0f) ? 1.0f / d : 0.0f;
                anyzero |= r.zero[k];
            }
            blk[j] = false;
            act[j] = ballot(r.live) != 0;
            zro[j] = ballot(r.live && anyzero) != 0;
        }

        // ---- corridor walk over the columns (all wave-uniform)
        const float F0[3] = {T.c[0] - T.half[0], T.c[1] - T.half[1], T.c[2] - T.half[2]};
        const float F1[3] = {T.c[0] + T.half[0], T.c[1] + T.half[1], T.c[2] + T.half[2]};
        const int a = fabsf(T.c[0] - q[0]) >= fabsf(T.c[1] - q[1]) ? 0 : 1;
        const int b = 1 - a;
        const float ga = a == 0 ? X.x0 : X.y0, gb = a == 0 ? X.y0 : X.x0;
        const int na = a == 0 ? X.nx : X.ny, nb = a == 0 ? X.ny : X.nx;
        const float qa = q[a], qb = q[b], qz = q[2];
        const float ua0 = F0[a] - qa, ua1 = F1[a] - qa;
        const float iua0 = ua0 != 0.0f ? 1.0f / ua0 : 0.0f;
        const float iua1 = ua1 != 0.0f ? 1.0f / ua1 : 0.0f;
        const float vb0 = F0[b] - qb, vb1 = F1[b] - qb;
        const float wz0 = F0[2] - qz;
        const float amin = fminf(qa, F0[a]), amax = fmaxf(qa, F1[a]);
        const float gend_a = ga + na * X.cs, gend_b = gb + nb * X.cs;
        bool stop = !(amax >= ga && amin < gend_a);
        int ia_lo = max(0, min(na - 1, (int)floorf((amin - ga) * X.inv_cs)));
        int ia_hi = max(0, min(na - 1, (int)floorf((amax - ga) * X.inv_cs)));
        const int step = (qa <= T.c[a]) ? -1 : 1;
        int ia = step < 0 ? ia_hi : ia_lo;
        const int ia_end = step < 0 ? ia_lo - 1 : ia_hi + 1;
        for (; !stop && ia != ia_end; ia += step) {
            const float A0 = ga + ia * X.cs, A1 = A0 + X.cs;
            float l0 = 0.0f, l1 = 1.0f;
            // rectangle (1-l) q + l F meets the slab [A0, A1] along axis a
            const float r1 = A1 - qa, r2 = A0 - qa;
            if (ua0 > 0.0f) l1 = fminf(l1, r1 * iua0);
            else if (ua0 < 0.0f) l0 = fmaxf(l0, r1 * iua0);
            else if (r1 < 0.0f) continue;
            if (ua1 > 0.0f) l0 = fmaxf(l0, r2 * iua1);
            else if (ua1 < 0.0f) l1 = fminf(l1, r2 * iua1);
            else if (r2 > 0.0f) continue;
            l0 = fmaxf(0.0f, l0 - kLambdaMargin);
            l1 = fminf(1.0f, l1 + kLambdaMargin);
            if (l0 > l1) continue;
            const float bl = fminf(qb + l0 * vb0, qb + l1 * vb0) - kWalkMargin;
            const float bh = fmaxf(qb + l0 * vb1, qb + l1 * vb1) + kWalkMargin;
            if (bh < gb || bl >= gend_b) continue;
            const float zf =
                DIM == 3 ? fminf(qz + l0 * wz0, qz + l1 * wz0) - kWalkMargin : -INFINITY;
            const int ib0 = max(0, min(nb - 1, (int)floorf((bl - gb) * X.inv_cs)));
            const int ib1 = max(0, min(nb - 1, (int)floorf((bh - gb) * X.inv_cs)));
            for (int ib = ib0; !stop && ib <= ib1; ++ib) {
                const int col = a == 0 ? ia + X.nx * ib : ib + X.nx * ia;
                const int rb = X.col_start[col], re = X.col_start[col + 1];
                if (STATS) ++n_cols;
                for (int rr = rb; rr < re; ++rr) {
                    const BoxRec B = X.recs[rr];
                    if (DIM == 3 && B.hi[2] < zf) break;
                    float lq[3], hq[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        lq[k] = B.lo[k] - q[k];
                        hq[k] = B.hi[k] - q[k];
                    }
                    bool any_blk = false, any_act = false;
#pragma unroll
                    for (int j = 0; j < NS; ++j) {
                        if (!act[j]) continue;
                        Ray &r = ray[j];
                        const bool need = r.live && !blk[j];
                        bool hit;
                        if (EXACT64) {
                            hit = need && exact_contact<DIM>(q, r.s, B);
                            if (STATS) n_tests += __popcll(ballot(need));
                        } else {
                            const float gap = zro[j] ? slab_gap<DIM, true>(r, lq, hq)
                                                     : slab_gap<DIM, false>(r, lq, hq);
                            const bool unsure = need && (P.recheck_all || fabsf(gap) <= P.eps);
                            hit = need && gap > P.eps;
                            if (unsure) {
                                const bool ex = exact_contact<DIM>(q, r.s, B);
                                if (STATS && P.recheck_all) {
                                    // float32 decision with the default margin
                                    const bool decided = fabsf(gap) > 0x1p-20f;
                                    if (decided && ((gap > 0.0f) != ex)) ++n_disagree;
                                }
                                hit = ex;
                            }
                            if (STATS) {
                                n_tests += __popcll(ballot(need));
                                n_rechecks += __popcll(ballot(unsure));
                            }
                        }
                        blk[j] = blk[j] || hit;
                        const bool open = r.live && !blk[j];
                        act[j] = ballot(open) != 0;
                        any_act = any_act || act[j];
                        any_blk = any_blk || (ballot(blk[j]) != 0);
                    }
                    if (P.mode == VCM_FULL ? any_blk : !any_act) {
                        stop = true;
                        break;
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < NS; ++j) visible += __popcll(ballot(ray[j].live && !blk[j]));
    }

    // ---- colour, bin, outputs
    int cnt;
    R col;
    if (!fov || N == 0) {
        cnt = 0;
        col = R(0);
    } else if (P.mode == VCM_FRACTION) {
        cnt = visible;
        col = (R(visible) / R(N)) * craw;
    } else {
        cnt = visible == N ? N : 0;
        col = visible == N ? craw : R(0);
    }
    R cb = col;
    if (P.bin_scale == VCM_BIN_LOG) {
        const R veff = col * R(P.V0);
        cb = veff <= R(P.mu) ? R(0) : fmin(R(1), log(veff / R(P.mu)) * R(P.inv_log_V0_mu));
    }
    const int bn = min(P.n_bins - 1, static_cast<int>(floor(cb * R(P.n_bins))));
    if (lane == 0) {
        A.bin[vp] = static_cast<uint8_t>(bn);
        if (A.c) A.c[vp] = static_cast<float>(col);
        if (A.count) A.count[vp] = static_cast<uint16_t>(cnt);
        if (STATS) {
            atomicAdd(&A.stats->rays, (unsigned long long)((fov && N > 0) ? N : 0));
            atomicAdd(&A.stats->box_tests, n_tests);
            atomicAdd(&A.stats->rechecks, n_rechecks);
            atomicAdd(&A.stats->columns, n_cols);
        }
    }
    if (STATS && n_disagree) atomicAdd(&A.stats->fp32_disagree, n_disagree);  // per lane
}

template <int DIM, int NS, bool EXACT64>
void launch_ns(const BruteArgs &a, bool stats, dim3 grid, hipStream_t st) {
    if (stats)
        hipLaunchKernelGGL((k_brute<DIM, NS, EXACT64, true>), grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_brute<DIM, NS, EXACT64, false>), grid, dim3(256), 0, st, a);
}

template <int DIM, bool EXACT64>
void launch_dim(const BruteArgs &a, int ns, bool stats, dim3 grid, hipStream_t st) {
    switch (ns) {
        case 1: launch_ns<DIM, 1, EXACT64>(a, stats, grid, st); break;
        case 2: launch_ns<DIM, 2, EXACT64>(a, stats, grid, st); break;
        case 3: launch_ns<DIM, 3, EXACT64>(a, stats, grid, st); break;
        case 4: launch_ns<DIM, 4, EXACT64>(a, stats, grid, st); break;
        case 5: launch_ns<DIM, 5, EXACT64>(a, stats, grid, st); break;
        default: launch_ns<DIM, 6, EXACT64>(a, stats, grid, st); break;
    }
}

}  // namespace

vcm_status launch_brute(const Index &ix, const TargetDesc &t, const GridDesc &g,
                        const ParamDesc &p, const vcm_result &r, int64_t vp_begin,
                        int64_t vp_end, hipStream_t stream, DevStats *stats) {
    if (vp_end <= vp_begin) return VCM_OK;
    BruteArgs a{};
    a.idx = ix.dev;
    a.tgt = t;
    a.grid = g;
    a.prm = p;
    a.bin = r.bin;
    a.c = r.c;
    a.count = r.count;
    a.stats = stats;
    a.vp_begin = vp_begin;
    a.vp_end = vp_end;
    const int max_n = t.per_facet * (t.kind == VCM_CUBE ? 3 : 1);
    const int ns = (max_n + 63) / 64;
    if (ns < 1 || ns > kMaxSlots) return set_error(VCM_E_INVALID, "too many target samples");
    const int64_t nblk = (vp_end - vp_begin + 3) / 4;
    if (nblk > 0x7fffffff) return set_error(VCM_E_INVALID, "too many viewpoints for one launch");
    dim3 grid(static_cast<unsigned>(nblk));
    const bool st = stats != nullptr;
    if (ix.dim == 2) {
        if (p.fp64)
            launch_dim<2, true>(a, ns, st, grid, stream);
        else
            launch_dim<2, false>(a, ns, st, grid, stream);
    } else {
        if (p.fp64)
            launch_dim<3, true>(a, ns, st, grid, stream);
        else
            launch_dim<3, false>(a, ns, st, grid, stream);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(VCM_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return VCM_OK;
}

}  // namespace vcm
