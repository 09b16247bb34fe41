// Pruned VCM construction: equi-visible cells (Sec. III-A) joined with the
// visibility gate, exactly (VCM_E) or through the MBR and tangential cell
// approximations of Sec. IV-A (VCM_M, VCM_T).
//
// The paper builds a colour tree of cells and joins it with a quad-tree of
// visible regions.  On the GPU every viewpoint instead finds its cell in
// closed form: ring i satisfies V(d_i) = V0 - i mu at the facing angle, so
// i = floor((V0 - V(D)) / mu) up to rounding, and the band likewise from the
// visual angle at the ring's middle distance.  Each guess is then settled by
// comparing against the boundary values themselves, which are evaluated in
// float64 with the same expressions that define them.  One thread per
// viewpoint; the gate (visible count, live samples, field of view) comes
// from the visible-region blocks (blocks.hip) or, for the undecided
// smallest blocks, from the ray kernel at their representatives.
#include <cmath>

#include "vcm_internal.h"

namespace vcm {
namespace {

struct CellFrame {
    double S, mu, d0, V0, dmax;
    int K;           // rings 0..K; ring K ends at dmax
    int rings_only;  // viewer-centric maps: one band per ring, colour facing
};

// Boundary radius d_i (d_0 = near point, d_{K+1} = d_max).
__device__ inline double ring_d(const CellFrame &F, int i) {
    if (i <= 0) return F.d0;
    if (i > F.K) return F.dmax;
    const double V = F.V0 - i * F.mu;
    return F.S / (2.0 * tan(V / 2.0));
}

__device__ inline double vis_angle(double S, double D, double alpha) {
    return 2.0 * atan((alpha / (M_PI / 2.0)) * S / (2.0 * D));
}

// Ring of distance D, or -1 at or beyond d_max.
__device__ inline int ring_of(const CellFrame &F, double D) {
    if (D >= F.dmax) return -1;
    const double Dn = D > F.d0 ? D : F.d0;
    const double V90 = 2.0 * atan(F.S / (2.0 * Dn));
    int i = static_cast<int>(floor((F.V0 - V90) / F.mu));
    i = max(0, min(F.K, i));
    while (i > 0 && D < ring_d(F, i)) --i;
    while (i < F.K && D >= ring_d(F, i + 1)) ++i;
    return i;
}

// Bands of one ring: gamma_0 = pi/2 > gamma_1 > ... > gamma_L > gamma_{L+1} = 0.
struct Ring {
    double dl, dh, dp, W0;
    int L;
};

// An upper bound on the angular width of every band of every ring whose
// middle distance d' lies in [a, b].  Band edges are (pi/2)(2d'/S) tan(W/2)
// with W stepping by mu, and tan is convex, so a ring's widest regular band
// is its first, of width (pi/2) t (x + 1/x) / (1 + x t) with x = S/(2d'),
// t = tan(mu/2); its last band is narrower than (pi/2)(2d'/S) tan(mu); a ring
// with W0 < 2 mu is one band of pi/2.  The bound decreases and then increases
// with d', so on an interval it is largest at an end.
__device__ inline double band_bound(const CellFrame &F, double d) {
    const double W0 = 2.0 * atan(F.S / (2.0 * d));
    if (W0 < 2.0 * F.mu) return M_PI / 2.0;
    const double x = F.S / (2.0 * d), t = tan(F.mu / 2.0);
    const double first = (M_PI / 2.0) * t * (x + 1.0 / x) / (1.0 + x * t);
    const double last = (M_PI / 2.0) * (2.0 * d / F.S) * tan(F.mu);
    return fmax(first, last);
}
__device__ inline double widest_band(const CellFrame &F, double a, double b) {
    return fmin(M_PI / 2.0, 1.000001 * fmax(band_bound(F, a), band_bound(F, b)) + 1e-12);
}

__device__ inline Ring make_ring(const CellFrame &F, int i) {
    Ring r;
    r.dl = ring_d(F, i);
    r.dh = ring_d(F, i + 1);
    r.dp = 0.5 * (r.dl + r.dh);
    r.W0 = 2.0 * atan(F.S / (2.0 * r.dp));
    int L = max(0, static_cast<int>(floor((r.W0 - F.mu) / F.mu)));
    while (r.W0 - (L + 1) * F.mu >= F.mu) ++L;
    while (L > 0 && r.W0 - L * F.mu < F.mu) --L;
    r.L = F.rings_only ? 0 : L;
    return r;
}

__device__ inline double gamma_of(const CellFrame &F, const Ring &r, int j) {
    if (j <= 0) return M_PI / 2.0;
    if (j > r.L) return 0.0;
    const double W = r.W0 - j * F.mu;
    const double Sj = 2.0 * r.dp * tan(W / 2.0);
    return (M_PI / 2.0) * Sj / F.S;
}

// Band of viewing angle alpha: (gamma_{j+1}, gamma_j]; the last one closed at 0.
__device__ inline int band_of(const CellFrame &F, const Ring &r, double alpha) {
    const double V = vis_angle(F.S, r.dp, alpha);
    int j = static_cast<int>(floor((r.W0 - V) / F.mu));
    j = max(0, min(r.L, j));
    while (j > 0 && alpha > gamma_of(F, r, j)) --j;
    while (j < r.L && alpha <= gamma_of(F, r, j + 1)) ++j;
    return j;
}

__device__ inline double cell_colour(const CellFrame &F, const Ring &r, int j) {
    const double gm = F.rings_only ? M_PI / 2.0 : 0.5 * (gamma_of(F, r, j) + gamma_of(F, r, j + 1));
    return vis_angle(F.S, r.dp, gm) / F.V0;
}

// Smallest j in [0, L] with pred(j) true for a predicate that is false then
// true as j grows; L + 1 if none.  Starts from a guess.
template <typename P>
__device__ inline int first_true(int guess, int L, P pred) {
    int j = max(0, min(L + 1, guess));
    while (j > 0 && pred(j - 1)) --j;
    while (j <= L && !pred(j)) ++j;
    return j;
}

// Band index whose boundary gamma_k first drops to <= theta (k in 0..L+1).
__device__ inline int first_gamma_below(const CellFrame &F, const Ring &r, double theta) {
    const double V = vis_angle(F.S, r.dp, fmax(theta, 0.0));
    const int guess = static_cast<int>(ceil((r.W0 - V) / F.mu));
    int k = max(0, min(r.L + 1, guess));
    while (k > 0 && gamma_of(F, r, k - 1) <= theta) --k;
    while (k <= r.L && gamma_of(F, r, k) > theta) ++k;
    return k;
}

// Sums of one pruned map, when statistics are requested (float64, one set per
// workgroup, added on the host in workgroup order):
//   [0] sum of (c_ref - c), [1] sum of |c_ref - c|, [2] sum of c_ref, where c
//       is the map's colour and c_ref, under the same visibility gate, the
//       brute-force colour (VCM_E) or the VCM_E colour (VCM_M, VCM_T): the
//       error measure of Sec. V-A;
//   [3] VCM_M / VCM_T: sum of |c_approx - c_E| over the viewpoints within
//       d_max, without the visibility gate: the error the bounds of Sec. IV-A
//       bound (they ignore obstacles), in colour units.
struct PrunedSums {
    double d[kPrunedSums];
};

struct PrunedArgs {
    CellFrame F;
    TargetDesc tgt;
    GridDesc grid;
    ParamDesc prm;
    const uint32_t *gate;  // per viewpoint: count | N << 10 | fov << 20
    int32_t method;        // VCM_PRUNED_E / M / T
    int32_t dim;
    uint8_t *bin;
    float *c;
    uint16_t *count;
    unsigned long long *fallback;  // tangent lookups that fell back (optional)
    double *sums;                  // per-workgroup PrunedSums (optional)
};

// Workgroup sum of the PrunedSums of its threads, written by thread 0.
__device__ void write_sums(double *out, const PrunedSums &v) {
    __shared__ double s[kPrunedSums][256];
    for (int k = 0; k < kPrunedSums; ++k) s[k][threadIdx.x] = v.d[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w)
            for (int k = 0; k < kPrunedSums; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < kPrunedSums; ++k) out[kPrunedSums * blockIdx.x + k] = s[k][0];
}

// VCM_M: the colour of the lowest ring, then lowest band, whose closed MBR
// in the (rho, h) quadrant contains q; q's own cell (ring iq, colour ce)
// holds it, so the search ends there.
__device__ double m_colour(const CellFrame &F, double D, double rho, double hh, int iq, double ce) {
    // a ring's MBRs lie within sqrt(2) d_{i+1} of the centre
    int i0 = ring_of(F, D / sqrt(2.0));
    i0 = i0 < 0 ? 0 : i0;
    while (i0 > 0 && sqrt(2.0) * ring_d(F, i0) >= D) --i0;
    // tighter: with u = sin g_j, v = cos g_{j+1} of a band of width w,
    // u^2 + v^2 <= 1 + 2w, so a ring whose MBR holds q has
    // D^2 <= d_{i+1}^2 (1 + 2w)
    {
        const double w = widest_band(F, ring_d(F, i0), ring_d(F, iq + 1));
        const int i1 = ring_of(F, D / sqrt(1.0 + 2.0 * w)) - 1;
        if (i1 > i0) i0 = i1;
    }
    for (int i = i0; i <= iq; ++i) {
        if (sqrt(2.0) * ring_d(F, i + 1) < D) continue;
        const Ring r = make_ring(F, i);
        // rho <= d_{i+1} cos(gamma_{j+1})  <=>  gamma_{j+1} <= acos(rho / d_{i+1})
        int jB = rho <= r.dh ? first_gamma_below(F, r, acos(rho / r.dh)) - 1 : r.L + 1;
        // d_i sin(gamma_{j+1}) <= h  <=>  gamma_{j+1} <= asin(h / d_i)
        int jC = hh >= r.dl ? 0 : first_gamma_below(F, r, asin(hh / r.dl)) - 1;
        jB = max(jB, 0);
        jC = max(jC, 0);
        const int j = max(jB, jC);
        if (j > r.L) continue;
        const double g0 = gamma_of(F, r, j), g1 = gamma_of(F, r, j + 1);
        if (rho >= r.dl * cos(g0) && rho <= r.dh * cos(g1) && hh >= r.dl * sin(g1) && hh <= r.dh * sin(g0))
            return cell_colour(F, r, j);
    }
    return ce;
}

// VCM_T: the colour of the lowest ring whose tangent trapezoid (band of
// alpha, projection on the band's middle direction in [d_i, d_{i+1}))
// contains q; q's own cell if none does (*fell_back set).
__device__ double t_colour(const CellFrame &F, double D, double alpha, int iq, double ce, bool *fell_back) {
    // the projection is at least D cos(45 deg)
    int i0 = ring_of(F, D * sqrt(0.5));
    i0 = i0 < 0 ? 0 : i0;
    while (i0 > 0 && ring_d(F, i0) > D * sqrt(0.5)) --i0;
    // tighter: alpha lies in the band, within half a band width of its
    // middle, so the projection is at least D cos(w / 2)
    {
        const double w = widest_band(F, ring_d(F, i0), ring_d(F, iq + 1));
        const int i1 = ring_of(F, D * cos(0.5 * w)) - 1;
        if (i1 > i0) i0 = i1;
    }
    for (int i = i0; i <= iq; ++i) {
        const Ring r = make_ring(F, i);
        const int j = band_of(F, r, alpha);
        const double gm = 0.5 * (gamma_of(F, r, j) + gamma_of(F, r, j + 1));
        const double p = D * cos(alpha - gm);
        if (p >= r.dl && p < r.dh) {
            *fell_back = false;
            return cell_colour(F, r, j);
        }
    }
    *fell_back = true;
    return ce;
}

__device__ void colour_viewpoint(const PrunedArgs &A, int64_t vp, PrunedSums &sum) {
    // the viewpoint's gate: from its decided block, or its smallest block's
    // representative
    const uint32_t gw = A.gate[vp];
    const int vis = static_cast<int>(gw & 1023u), N = static_cast<int>((gw >> 10) & 1023u);
    const bool fov = (gw >> 20) & 1u;
    const bool shown = fov && N > 0 && vis > 0;   // some colour survives the gate
    if (!shown && !A.sums) {
        // colour 0, bin 0: no cell lookup (most viewpoints of a city map)
        A.bin[vp] = 0;
        if (A.c) A.c[vp] = 0.0f;
        if (A.count) A.count[vp] = static_cast<uint16_t>(vis);
        return;
    }
    const int n0 = A.grid.n[0], n1 = A.grid.n[1];
    const int ii[3] = {static_cast<int>(vp % n0), static_cast<int>((vp / n0) % n1),
                       static_cast<int>(vp / (static_cast<int64_t>(n0) * n1))};
    // viewpoint, relative to the target centre (exact)
    double dl[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < A.dim; ++k)
        dl[k] = (double(A.grid.o[k]) + double(2 * ii[k] + 1) * double(A.grid.h2[k])) -
                double(A.tgt.c[k]);
    int nax = A.tgt.nax;
    if (A.tgt.kind == VCM_CUBE) {
        nax = 0;
        if (fabs(dl[1]) > fabs(dl[nax])) nax = 1;
        if (fabs(dl[2]) > fabs(dl[nax])) nax = 2;
    }
    const double h = fabs(dl[nax]);
    double r2 = 0.0;
    for (int k = 0; k < 3; ++k)
        if (k != nax) r2 += dl[k] * dl[k];
    const double D = sqrt(r2 + h * h);
    const double alpha = atan2(h, sqrt(r2));
    const double rho = D * cos(alpha), hh = D * sin(alpha);

    const CellFrame &F = A.F;
    double craw = 0.0, ce = 0.0;
    bool fell_back = false;
    const int iq = ring_of(F, D);
    if (iq >= 0 && (shown || A.sums)) {
        const Ring rq = make_ring(F, iq);
        ce = cell_colour(F, rq, band_of(F, rq, alpha));
        craw = ce;
        if (A.method == VCM_PRUNED_M) craw = m_colour(F, D, rho, hh, iq, ce);
        else if (A.method == VCM_PRUNED_T) craw = t_colour(F, D, alpha, iq, ce, &fell_back);
    }
    double gatef = 0.0;
    if (fov && N > 0) gatef = A.prm.mode == VCM_FRACTION ? double(vis) / double(N) : (vis == N ? 1.0 : 0.0);
    const double col = gatef * craw;
    if (A.sums) {
        // reference colour under the same gate: the brute-force measure for
        // VCM_E, q's own cell for VCM_M and VCM_T
        const double am = F.rings_only ? M_PI / 2.0 : alpha;  // a viewer's points face it
        const double ref_raw = A.method == VCM_PRUNED_E ? vis_angle(F.S, D > F.d0 ? D : F.d0, am) / F.V0 : ce;
        const double ref = gatef * ref_raw;
        sum.d[0] += ref - col;
        sum.d[1] += fabs(ref - col);
        sum.d[2] += ref;
        if (A.method != VCM_PRUNED_E) sum.d[3] += fabs(craw - ce);
    }
    double cb = col;
    if (A.prm.bin_scale == VCM_BIN_LOG) {
        const double veff = col * F.V0;
        const double mu = F.mu;
        cb = veff <= mu ? 0.0 : fmin(1.0, log(veff / mu) / log(F.V0 / mu));
    }
    const int bn = min(A.prm.n_bins - 1, static_cast<int>(floor(cb * A.prm.n_bins)));
    A.bin[vp] = static_cast<uint8_t>(bn);
    if (A.c) A.c[vp] = static_cast<float>(col);
    if (A.count) A.count[vp] = static_cast<uint16_t>(vis);
    if (A.fallback && fell_back && shown) atomicAdd(A.fallback, 1ull);
}

__global__ __launch_bounds__(256) void k_pruned(PrunedArgs A) {
    const int64_t vp = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    PrunedSums sum{};
    if (vp < A.grid.count) colour_viewpoint(A, vp, sum);
    if (A.sums) write_sums(A.sums, sum);
}

}  // namespace

int64_t pruned_sum_blocks(const GridDesc &g) { return (g.count + 255) / 256; }

int count_rings(double S, double mu, double d0, double *V0) {
    *V0 = 2.0 * std::atan(S / (2.0 * d0));
    int K = 0;
    for (int k = 1;; ++k) {
        if (*V0 - k * mu < mu) break;
        K = k;
    }
    return K;
}

vcm_status launch_pruned(const Index &ix, const TargetDesc &t, const GridDesc &g,
                         const ParamDesc &p, int method, const uint32_t *gate, const vcm_result &r,
                         hipStream_t stream, unsigned long long *fallback, double *sums) {
    PrunedArgs a{};
    double V0;
    const double mu = p.mu_d;
    a.F.S = t.S;
    a.F.mu = mu;
    a.F.d0 = p.d0_d;
    a.F.K = count_rings(t.S, mu, p.d0_d, &V0);
    a.F.V0 = V0;
    a.F.dmax = t.S / (2.0 * std::tan(mu / 2.0));
    a.F.rings_only = t.kind == VCM_VIEWER ? 1 : 0;
    a.tgt = t;
    a.grid = g;
    a.prm = p;
    a.gate = gate;
    a.method = method;
    a.dim = ix.dim;
    a.bin = r.bin;
    a.c = r.c;
    a.count = r.count;
    a.fallback = fallback;
    a.sums = sums;
    const int64_t nblk = pruned_sum_blocks(g);
    if (nblk <= 0) return VCM_OK;
    hipLaunchKernelGGL(k_pruned, dim3(static_cast<unsigned>(nblk)), dim3(256), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(VCM_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return VCM_OK;
}

}  // namespace vcm
