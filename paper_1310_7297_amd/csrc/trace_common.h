// Device helpers shared by the ray-casting kernels (brute.hip) and the
// visible-region block kernels (blocks.hip): the exact segment/box predicate,
// the visual-angle measure, the field of view, the target's sample table and
// the constant-address-space view of the obstacle index.  Every translation
// unit that includes this header gets its own copy (anonymous namespace).
#pragma once

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "vcm_internal.h"

namespace vcm {
namespace {

constexpr float kWalkMargin = 1.0f / 128.0f;
constexpr float kLambdaMargin = 1e-6f;

// Exact contact of the closed segment [q, s] with the closed box [lo, hi],
// given d = s - q, lq = lo - q and hq = hi - q.  All coordinates are
// multiples of 2^-8 below 2^14, so these differences are exact in float32
// and every product of two of them is exact in float64.  Along each axis the
// box admits the ray parameters between an entry and an exit fraction
// (numerator / positive denominator); the segment meets the box iff no entry
// exceeds an exit, the bounds 0 and 1 included, compared by cross-multiplying.
template <int DIM>
__device__ __attribute__((always_inline)) inline bool exact_contact(const float *d,
                                                                    const float *lq,
                                                                    const float *hq) {
    float en[DIM], ex[DIM], de[DIM];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const bool up = d[k] > 0.0f, down = d[k] < 0.0f;
        en[k] = up ? lq[k] : (down ? -hq[k] : 0.0f);
        ex[k] = up ? hq[k] : (down ? -lq[k] : 1.0f);
        de[k] = up ? d[k] : (down ? -d[k] : 1.0f);
        // a direction component of 0: q itself must lie in the slab
        ok = ok && (up || down || (lq[k] <= 0.0f && hq[k] >= 0.0f));
        ok = ok && en[k] <= de[k] && ex[k] >= 0.0f;
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b)
            if (a != b)
                ok = ok && double(en[a]) * double(de[b]) <= double(ex[b]) * double(de[a]);
    return ok;
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
    // a viewer's points are seen facing (no foreshortening)
    const R alpha = T.kind == VCM_VIEWER ? R(M_PI / 2) : my_atan2<R>(h, rho);
    const R Sa = alpha * (R(2) / R(M_PI)) * R(T.S);
    const R Dn = D > R(P.d0) ? D : R(P.d0);
    const R V = R(2) * my_atan<R>(Sa / (R(2) * Dn));
    return V / R(P.V0);
}

// A viewer-centric map covers the closed ball of radius rmax about the viewer
// (exact in float64 on the 2^-8 lattice); other maps the whole space.
template <int DIM>
__device__ inline bool in_region(const TargetDesc &T, const float *q) {
    if (T.kind != VCM_VIEWER) return true;
    double d2 = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const double d = double(q[k]) - double(T.c[k]);
        d2 += d * d;
    }
    return d2 <= double(T.rmax) * double(T.rmax);
}

// Field of view (closed wedge about the normal, apex at the target centre).
// The quantities are exact in float64 for inputs on the 2^-8 lattice.
template <int DIM>
__device__ inline bool in_wedge(const TargetDesc &T, const ParamDesc &P, const float *q) {
    if (P.fov_kind == kFovAll) return true;
    double d2 = 0.0, dn = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const double d = double(q[k]) - double(T.c[k]);
        d2 += d * d;
        if (k == P.fov_axis) dn = P.fov_sign * d;
    }
    if (P.fov_kind == kFovHalf) return dn >= 0.0;
    if (P.fov_kind == kFovNarrow) return dn >= 0.0 && dn * dn >= P.fov_c2 * d2;
    return dn >= 0.0 || dn * dn <= P.fov_c2 * d2;
}

// Viewpoints outside the field of view or outside the covered region are
// obstructed.  One pass computes both (P.region_r2 is d_max^2 for a
// viewer-centric map, +inf otherwise): the same decisions as in_region and
// in_wedge, with fewer registers live in the ray kernels.
template <int DIM>
__device__ inline bool in_fov(const TargetDesc &T, const ParamDesc &P, const float *q) {
    if (P.fov_kind == kFovAll && !(P.region_r2 < HUGE_VAL)) return true;   // no wedge, no ball
    double d2 = 0.0, dn = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const double d = double(q[k]) - double(T.c[k]);
        d2 += d * d;
        if (k == P.fov_axis) dn = P.fov_sign * d;
    }
    if (!(d2 <= P.region_r2)) return false;
    if (P.fov_kind == kFovAll) return true;
    if (P.fov_kind == kFovHalf) return dn >= 0.0;
    if (P.fov_kind == kFovNarrow) return dn >= 0.0 && dn * dn >= P.fov_c2 * d2;
    return dn >= 0.0 || dn * dn <= P.fov_c2 * d2;
}


// Colour and bin of viewpoint q from its visible count cnt of n live samples
// (0 outside the field of view): the visual angle of Eq. 1 / Eq. 2 over V0,
// scaled by the visible fraction in FRACTION mode, then binned in the
// query's scale.  The ray kernel and the incremental re-colouring share it,
// so that both give the same bits.
template <int DIM, typename R, int MODE>
__device__ __attribute__((always_inline)) inline void colour_and_bin(const TargetDesc &T, const ParamDesc &P,
                                                                     const float *q, int cnt, int n, R &col,
                                                                     int &bin) {
    col = R(0);
    if (cnt > 0) {
        col = raw_colour<DIM, R>(T, P, q);
        if (MODE == VCM_FRACTION) col = (R(cnt) / R(n)) * col;
    }
    R cb = col;
    if (P.bin_scale == VCM_BIN_LOG) {
        const R veff = col * R(P.V0);
        cb = veff <= R(P.mu) ? R(0) : fmin(R(1), log(veff / R(P.mu)) * R(P.inv_log_V0_mu));
    }
    bin = min(P.n_bins - 1, static_cast<int>(floor(cb * R(P.n_bins))));
}

__device__ inline float readlane_f(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline unsigned long long lanes_below() {
    return (1ull << (threadIdx.x & 63)) - 1ull;
}
__device__ inline int mbcnt(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<unsigned>(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<unsigned>(m), 0u));
}

// A wave-uniform float as a scalar-register value.
__device__ inline float uniform_f(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// Position of local sample w (lattice index u fastest) of the facet with face
// code fc (cube: 2k for the face at -k, 2k+1 for +k; other targets: their one
// facet, fc ignored).
template <int DIM>
__device__ __attribute__((always_inline)) inline void sample_pos_face(const TargetDesc &T, unsigned fc_u,
                                                                      unsigned w, float *s) {
    const unsigned iv = static_cast<unsigned>((w * T.m_su) >> 32);
    const unsigned iu = w - iv * T.su;
    const float u = static_cast<float>(2 * static_cast<int>(iu) + 1 - T.su) * T.hu;
    const float v = static_cast<float>(2 * static_cast<int>(iv) + 1 - T.sv) * T.hv;
    s[0] = T.c[0];
    s[1] = T.c[1];
    s[2] = DIM == 3 ? T.c[2] : 0.0f;
    if (T.kind == VCM_CUBE) {
        const int fc = static_cast<int>(fc_u);
        const int k = fc >> 1;
        const int ua = (k == 0) ? 1 : 0;
        // k may differ between lanes: select among scalar copies (values, not
        // loads, so the selection does not become a per-lane memory load)
        const float c0 = uniform_f(T.c[0]), c1 = uniform_f(T.c[1]), c2 = uniform_f(T.c[2]);
        const float h0 = uniform_f(T.half[0]), h1 = uniform_f(T.half[1]), h2 = uniform_f(T.half[2]);
        const float ck = k == 0 ? c0 : (k == 1 ? c1 : c2);
        const float hk = k == 0 ? h0 : (k == 1 ? h1 : h2);
        const float plane = (fc & 1) ? ck + hk : ck - hk;
        s[0] = k == 0 ? plane : (ua == 0 ? c0 + u : s[0]);
        s[1] = k == 1 ? plane : (ua == 1 ? c1 + u : c1 + v);
        s[2] = k == 2 ? plane : c2 + v;
    } else {
        const int wax = 1 - T.nax;
        if (wax == 0) s[0] = T.c[0] + u;
        else s[1] = T.c[1] + u;
        if (T.kind == VCM_BILLBOARD) s[2] = T.c[2] + v;
    }
}

// Sample table of a launch: every sample of every facet (the cube's six faces
// or the one facet), indexed by face code * per_facet + local index, in LDS.
// A cube has at most 128 samples per face (three faces of live samples fit
// the 384 ray slots), other targets at most 384: 768 entries.
constexpr int kTableMax = 768;

template <int DIM>
__device__ void build_sample_table(const TargetDesc &T, float4 *tab) {
    const int n = (T.kind == VCM_CUBE ? 6 : 1) * T.per_facet;
    for (int t = threadIdx.x; t < n && t < kTableMax; t += blockDim.x) {
        const unsigned fc = static_cast<unsigned>((static_cast<unsigned>(t) * T.m_pf) >> 32);
        const unsigned w = static_cast<unsigned>(t) - fc * T.per_facet;
        float sp[3];
        sample_pos_face<DIM>(T, fc, w, sp);
        tab[t] = make_float4(sp[0], sp[1], sp[2], 0.0f);
    }
    __syncthreads();
}

// Sample sources: lattice arithmetic, or the workgroup's table.
constexpr int kTabNone = 0, kTabBlock = 1;

// Position of sample `si` among the live samples of a viewpoint whose live
// facets are `faces` (cube, packed 4 bits per live face) or the single facet
// (segment, billboard); from the sample table when one is given.
template <int DIM, int TAB>
__device__ __attribute__((always_inline)) inline void sample_pos(const TargetDesc &T, unsigned faces, unsigned si,
                                                                 float *s, const void *tab) {
    const unsigned f = static_cast<unsigned>((si * T.m_pf) >> 32);
    const unsigned w = si - f * T.per_facet;
    const unsigned fc = T.kind == VCM_CUBE ? (faces >> (4 * f)) & 7u : 0u;
    if (TAB == kTabBlock) {
        const float4 p = static_cast<const float4 *>(tab)[fc * T.per_facet + w];
        s[0] = p.x;
        s[1] = p.y;
        s[2] = p.z;
    } else {
        sample_pos_face<DIM>(T, fc, w, s);
    }
}

// Rays of one slot: sample position and reciprocal direction per lane.  A
// zero direction component gets reciprocal 0 and sends the lane's tests to
// the exact predicate (zero_lane).
template <int DIM, int TAB>
__device__ __attribute__((always_inline)) inline bool ray_setup(const TargetDesc &T, unsigned faces, const float *q,
                                                               unsigned si, float *s, float *inv,
                                                               const void *tab) {
    sample_pos<DIM, TAB>(T, faces, si, s, tab);
    bool zero = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float d = s[k] - q[k];
        // v_rcp_f32 is accurate to 1 ulp; with the exact numerator lo - q the
        // slab parameter carries at most 1.5 * 2^-23 relative error.
        inv[k] = (k < DIM && d != 0.0f) ? __builtin_amdgcn_rcpf(d) : 0.0f;
        zero = zero || (k < DIM && d == 0.0f);
    }
    return zero;
}

// Float32 slab test: gap t1 - t0 of the parameter interval [t0, t1] that the
// box cuts from [0, 1]; the segment meets the box iff gap >= 0.
template <int DIM>
__device__ inline float slab_gap(const float *inv, const float *lq, const float *hq) {
    float t0 = 0.0f, t1 = 1.0f;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const float a = lq[k] * inv[k];
        const float b = hq[k] * inv[k];
        t0 = fmaxf(t0, fminf(a, b));
        t1 = fminf(t1, fmaxf(a, b));
    }
    return t1 - t0;
}

// A non-negative float as an unsigned integer with the same order; negative
// values (and -0) map to 0, below every box coordinate of the index frame.
__device__ inline unsigned ord(float x) { return x > 0.0f ? __float_as_uint(x) : 0u; }

// The index is immutable while kernels run: read it through the constant
// address space, so that wave-uniform reads (column offsets, the blocker
// cache's record) become scalar loads.
// (The host pass of the compiler only needs the declarations.)
#if defined(__HIP_DEVICE_COMPILE__)
#define VCM_CONST __attribute__((address_space(4)))
#else
#define VCM_CONST
#endif
typedef const VCM_CONST int32_t *cptr_i32;
typedef const VCM_CONST BoxRec *cptr_rec;

}  // namespace
}  // namespace vcm
