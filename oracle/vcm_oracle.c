/*
 * vcm_oracle.c -- plain, slow, exact CPU reference for target-centric
 * visibility color maps (VCM).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The HIP library
 * shares no code with it and never calls it.
 *
 * What it computes, with the passage each part follows:
 *   - VCM (Def. 2.1): one colour c in [0,1] per viewpoint of a discretised
 *     space, for a given target T and obstacle set O.
 *   - Point-to-point visibility (Def. 2.2): p and p' see each other iff the
 *     segment pp' meets no obstacle.  Obstacles are closed axis-aligned boxes
 *     and touching counts as meeting (Def. 3.1 says a segment that touches an
 *     obstacle is shadowed).  The test is exact: every input is a multiple of
 *     2^-8 below 2^14 in magnitude, so it runs in 64-bit integers.
 *   - Obstructed region (Def. 2.3): a viewpoint that does not see *all* points
 *     of T is obstructed and coloured 0 (Sec. III-B, last paragraph; Sec.
 *     III-C).  T is represented by a lattice of sample points per facet.
 *   - Visual angle (Eq. 1) with oblique foreshortening (Eq. 2):
 *     V = 2 arctan(S_alpha / 2D), S_alpha = (alpha / 90 deg) S.
 *   - Field of view (Sec. III-B): viewpoints outside the FOV wedge around the
 *     target normal are obstructed.
 *   - Viewer-centric VCM (Sec. IV-B): a viewer q instead of a target; the map
 *     covers the ball of radius d_max about q, and S is the size whose visual
 *     angle is mu at d_max, S = 2 d_max tan(mu / 2).  Read as a point target
 *     at q of that size, seen facing (no foreshortening), by the symmetry of
 *     visibility (Sec. III-A).
 *   - Pruned construction: equi-visible cells (Sec. III-A), visible-region
 *     blocks split down to a minimum size (Sec. III-C-1), the MBR and
 *     tangential approximations and their error bounds (Sec. IV-A), the
 *     error measure (Sec. V-A).
 *
 * Readings taken where the paper is silent:
 *   - S is the largest target dimension; D is the distance from the viewpoint
 *     to the target centre, floored at the near point d0; alpha is the angle
 *     between the line of sight and the target plane, measured in the
 *     meridian plane (h = |Delta . n|, rho = |Delta - (Delta . n) n|).
 *   - c = V / V0 with V0 = 2 arctan(S / 2 d0), the largest visual angle.
 *   - Cube targets: n is the axis of largest |Delta_k|; only faces facing the
 *     viewpoint (strictly) carry live samples.
 *   - FULL mode is the paper's complete-visibility rule; FRACTION mode scales
 *     the colour by the visible fraction of live samples (an extension).
 *   - Linear colour bins: bin = min(B-1, floor(c B)); the log scale is a test
 *     aid that spreads visual angles between mu and V0 over the bins.
 *
 * Every function is pinned by tests against closed forms, invariants, brute
 * force on tiny inputs or the paper's worked example.  The error bounds of
 * Sec. IV-A (vo_error_bounds) are pinned only from below: they must exceed
 * the error measured over the whole region of distinguishable visibility
 * (vo_bound_measured); the paper prints no value of either bound that could
 * pin them exactly.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { VO_SEGMENT = 0, VO_BILLBOARD = 1, VO_CUBE = 2, VO_VIEWER = 3 };
enum { VO_FULL = 0, VO_FRACTION = 1 };
enum { VO_BIN_LINEAR = 0, VO_BIN_LOG = 1 };

typedef struct {
    int kind;
    int normal_axis;
    int normal_sign;
    int su, sv;
    double center[3];
    double size[2];
} vo_target;

typedef struct {
    double origin[3];
    double extent[3];
    int64_t n[3];
} vo_grid;

typedef struct {
    double mu_arcmin;
    double d0;
    double fov_deg;
    int n_bins;
    int bin_scale;
    int mode;
    int gaze;   /* field-of-view axis: 0 = the target's normal, +-(1 + k) = +-axis k */
} vo_params;

#define VO_PI 3.14159265358979323846

/* ------------------------------------------------------------ exactness -- */

/* x as an integer count of 2^-8 quanta; -1 if x is not such a multiple or
 * is out of range. */
static int to_quanta(double x, int64_t *out)
{
    double y = x * 256.0;
    if (!(fabs(y) < 4194304.0) || y != floor(y))
        return -1;
    *out = (int64_t)y;
    return 0;
}

/* ------------------------------------------ point-to-point visibility ---- */

/* Does the closed segment [q, s] meet the closed box [lo, hi]?  All values in
 * quanta.  The segment is q + t (s - q), t in [0, 1].  Along each axis the
 * box admits an interval of t; the segment meets the box iff the largest
 * lower end is not above the smallest upper end (together with [0, 1]).
 * Every interval end is a fraction num/den with den > 0, so each comparison
 * is done by cross-multiplication, exactly. */
static int seg_meets_box(int dim, const int64_t *q, const int64_t *s,
                         const int64_t *lo, const int64_t *hi)
{
    int64_t lnum[3], unum[3], den[3];
    int m = 0;
    for (int k = 0; k < dim; ++k) {
        int64_t d = s[k] - q[k];
        if (d == 0) {
            if (q[k] < lo[k] || q[k] > hi[k])
                return 0;
            continue;
        }
        int64_t a, b, e;
        if (d > 0) {
            a = lo[k] - q[k];
            b = hi[k] - q[k];
            e = d;
        } else {
            a = q[k] - hi[k];
            b = q[k] - lo[k];
            e = -d;
        }
        /* lower end a/e must not exceed 1; upper end b/e must not be below 0 */
        if (a > e || b < 0)
            return 0;
        lnum[m] = a;
        unum[m] = b;
        den[m] = e;
        ++m;
    }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j)
            if (i != j && lnum[i] * den[j] > unum[j] * den[i])
                return 0;
    return 1;
}

/* Public wrapper on doubles (inputs must be multiples of 2^-8).
 * Returns 1 (meets), 0 (misses), -1 (invalid input). */
int vo_segment_meets_box(int dim, const double *q, const double *s,
                         const double *lo, const double *hi)
{
    int64_t Q[3] = {0, 0, 0}, S[3] = {0, 0, 0}, L[3] = {0, 0, 0}, H[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) {
        if (to_quanta(q[k], &Q[k]) || to_quanta(s[k], &S[k]) ||
            to_quanta(lo[k], &L[k]) || to_quanta(hi[k], &H[k]))
            return -1;
        if (L[k] > H[k])
            return -1;
    }
    return seg_meets_box(dim, Q, S, L, H);
}

/* --------------------------------------------------------- target side -- */

static double mu_rad(const vo_params *p) { return p->mu_arcmin * VO_PI / (180.0 * 60.0); }

/* Size S entering Eq. 1: the largest target dimension; for the viewer of a
 * viewer-centric map (size[0] = d_max), the size whose visual angle at d_max
 * is mu (Sec. IV-B): 2 arctan(S / (2 d_max)) = mu. */
static double target_size(const vo_target *t, const vo_params *p)
{
    if (t->kind == VO_BILLBOARD)
        return t->size[0] > t->size[1] ? t->size[0] : t->size[1];
    if (t->kind == VO_VIEWER)
        return 2.0 * t->size[0] * tan(mu_rad(p) / 2.0);
    return t->size[0];
}

/* Live samples of T seen from q: facet-lattice cell centres
 * (k + 1/2) / N along each facet direction.  Segment: N_u points along the
 * axis orthogonal to the normal.  Billboard: N_u (horizontal) x N_v
 * (vertical) on the plane orthogonal to the normal axis.  Cube: N_u x N_v per
 * face, faces in the order (-x, +x, -y, +y, -z, +z), a face being live only
 * when q lies strictly on its outer side.  Returns N(q). */
int vo_live_samples(const vo_target *t, const double *q, double *out)
{
    int n = 0;
    const double *c = t->center;
    if (t->kind == VO_VIEWER) {
        if (out) {
            out[0] = c[0];
            out[1] = c[1];
            out[2] = c[2];
        }
        return 1;
    }
    if (t->kind == VO_SEGMENT || t->kind == VO_BILLBOARD) {
        int a = t->normal_axis;
        int w = 1 - a;
        double W = t->size[0];
        double H = t->kind == VO_BILLBOARD ? t->size[1] : 0.0;
        int nv = t->kind == VO_BILLBOARD ? t->sv : 1;
        for (int iv = 0; iv < nv; ++iv)
            for (int iu = 0; iu < t->su; ++iu) {
                double p[3];
                p[a] = c[a];
                p[w] = c[w] - W / 2.0 + (iu + 0.5) * (W / t->su);
                p[2] = t->kind == VO_BILLBOARD ? c[2] - H / 2.0 + (iv + 0.5) * (H / nv) : 0.0;
                if (out) {
                    out[3 * n + 0] = p[0];
                    out[3 * n + 1] = p[1];
                    out[3 * n + 2] = p[2];
                }
                ++n;
            }
        return n;
    }
    /* cube */
    double E = t->size[0];
    for (int f = 0; f < 6; ++f) {
        int k = f / 2;
        int sgn = (f % 2) ? 1 : -1;
        double plane = c[k] + sgn * E / 2.0;
        if (!(sgn * (q[k] - plane) > 0.0))
            continue;
        int ua = (k == 0) ? 1 : 0;
        int vb = (k == 2) ? 1 : 2;
        for (int iv = 0; iv < t->sv; ++iv)
            for (int iu = 0; iu < t->su; ++iu) {
                double p[3];
                p[k] = plane;
                p[ua] = c[ua] - E / 2.0 + (iu + 0.5) * (E / t->su);
                p[vb] = c[vb] - E / 2.0 + (iv + 0.5) * (E / t->sv);
                if (out) {
                    out[3 * n + 0] = p[0];
                    out[3 * n + 1] = p[1];
                    out[3 * n + 2] = p[2];
                }
                ++n;
            }
    }
    return n;
}

/* ----------------------------------------------------------- measure ----- */

/* Visual angle of T from q (Eq. 1 with the oblique size of Eq. 2).
 * out = {D, alpha (rad), V (rad), V0 (rad)}. */
void vo_measure(const vo_target *t, const vo_params *p, const double *q, double *out)
{
    double dl[3];
    for (int k = 0; k < 3; ++k)
        dl[k] = q[k] - t->center[k];
    if (t->kind == VO_SEGMENT)
        dl[2] = 0.0; /* the 2-D plane */
    int nax;
    if (t->kind == VO_CUBE) {
        nax = 0;
        for (int k = 1; k < 3; ++k)
            if (fabs(dl[k]) > fabs(dl[nax]))
                nax = k;
    } else {
        nax = t->normal_axis;
    }
    double h = fabs(dl[nax]);
    double r2 = 0.0;
    for (int k = 0; k < 3; ++k)
        if (k != nax)
            r2 += dl[k] * dl[k];
    double rho = sqrt(r2);
    double D = sqrt(r2 + h * h);
    double alpha = atan2(h, rho);                 /* 90 deg facing, 0 edge-on */
    if (t->kind == VO_VIEWER)
        alpha = VO_PI / 2.0;                      /* a point seen facing */
    double S = target_size(t, p);
    double s_alpha = (alpha / (VO_PI / 2.0)) * S; /* Eq. 2 */
    double Dn = D > p->d0 ? D : p->d0;            /* no closer than the near point */
    double V = 2.0 * atan(s_alpha / (2.0 * Dn));  /* Eq. 1 */
    double V0 = 2.0 * atan(S / (2.0 * p->d0));
    out[0] = D;
    out[1] = alpha;
    out[2] = V;
    out[3] = V0;
}

/* ----------------------------------------------------------- FOV --------- */

/* Axis and orientation of the field-of-view wedge: the target's normal,
 * or the gaze direction the query names (incremental processing, Sec. IV-C,
 * turns the gaze without moving the target). */
static void wedge_axis(const vo_target *t, const vo_params *p, int *axis, int *sign)
{
    if (p->gaze == 0) {
        *axis = t->normal_axis;
        *sign = t->normal_sign;
    } else {
        *axis = (p->gaze > 0 ? p->gaze : -p->gaze) - 1;
        *sign = p->gaze > 0 ? 1 : -1;
    }
}

/* Is q inside the field of view?  The wedge has its apex at the target
 * centre and is symmetric about the wedge axis n, the target normal or the
 * gaze (viewer-at-target symmetry, Sec. III-A): angle(q - m, n) <= FOV / 2,
 * closed.  The test
 * compares (Delta.n)^2 with cos^2(FOV/2) |Delta|^2; cos^2 is an exact rational
 * for the half-angles 30/45/60/120/135/150 degrees (the table's FOVs and 90 /
 * 270 degrees), which makes the comparison exact on the 2^-8 lattice: a point
 * on the wedge's boundary is inside. */
static int in_wedge(const vo_target *t, const vo_params *p, const double *q)
{
    double half = p->fov_deg / 2.0;
    if (half >= 180.0)
        return 1;
    double dl[3], d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        dl[k] = (t->kind == VO_SEGMENT && k == 2) ? 0.0 : q[k] - t->center[k];
        d2 += dl[k] * dl[k];
    }
    int ax, sg;
    wedge_axis(t, p, &ax, &sg);
    double dn = sg * dl[ax];
    if (half == 90.0)
        return dn >= 0.0;
    double c2;
    if (half == 30.0 || half == 150.0)
        c2 = 0.75;
    else if (half == 45.0 || half == 135.0)
        c2 = 0.5;
    else if (half == 60.0 || half == 120.0)
        c2 = 0.25;
    else {
        double cs = cos(half * VO_PI / 180.0);
        c2 = cs * cs;
    }
    if (half < 90.0)
        return dn >= 0.0 && dn * dn >= c2 * d2;
    return dn >= 0.0 || dn * dn <= c2 * d2;
}

/* A viewer-centric map covers the closed ball of radius d_max about the
 * viewer (Sec. IV-B); every other map covers the whole space.  Exact on the
 * 2^-8 lattice. */
static int in_region(const vo_target *t, const double *q)
{
    if (t->kind != VO_VIEWER)
        return 1;
    double r2 = 0.0;
    for (int k = 0; k < 3; ++k)
        r2 += (q[k] - t->center[k]) * (q[k] - t->center[k]);
    return r2 <= t->size[0] * t->size[0];
}

/* Viewpoints outside the field of view, or outside the region a
 * viewer-centric map covers, are obstructed. */
int vo_in_fov(const vo_target *t, const vo_params *p, const double *q)
{
    return in_region(t, q) && in_wedge(t, p, q);
}

/* ----------------------------------------------------------- colour ------ */

/* Colour in the bin's scale and the bin index. */
static void to_bin(const vo_params *p, double c, double V0, double *cb, uint8_t *bin)
{
    double v;
    if (p->bin_scale == VO_BIN_LOG) {
        double mu = p->mu_arcmin * VO_PI / (180.0 * 60.0);
        double Veff = c * V0;
        if (Veff <= mu)
            v = 0.0;
        else {
            v = log(Veff / mu) / log(V0 / mu);
            if (v > 1.0)
                v = 1.0;
        }
    } else {
        v = c;
    }
    double f = floor(v * p->n_bins);
    int b = (int)f;
    if (b > p->n_bins - 1)
        b = p->n_bins - 1;
    if (b < 0)
        b = 0;
    *cb = v;
    *bin = (uint8_t)b;
}

/* ----------------------------------------------------------- the map ----- */

typedef struct {
    int dim;
    int64_t nbox;
    int64_t *blo, *bhi; /* quanta, [box][3] */
    const vo_target *t;
    const vo_grid *g;
    const vo_params *p;
    const int64_t *vp;
    int64_t nvp;
    uint16_t *count, *nlive;
    uint8_t *infov, *bin;
    double *c, *cb;
    int64_t first, last;
} vo_job;

static void eval_range(vo_job *J)
{
    const vo_target *t = J->t;
    const vo_grid *g = J->g;
    const vo_params *p = J->p;
    int maxs = 6 * t->su * (t->sv > 0 ? t->sv : 1);
    double *smp = (double *)malloc(sizeof(double) * 3 * (size_t)maxs);
    int64_t *sq = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)maxs);
    for (int64_t v = J->first; v < J->last; ++v) {
        int64_t idx = J->vp[v];
        int64_t i = idx % g->n[0];
        int64_t j = (idx / g->n[0]) % g->n[1];
        int64_t k = idx / (g->n[0] * g->n[1]);
        int64_t ii[3] = {i, j, k};
        double q[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < J->dim; ++a)
            q[a] = g->origin[a] + (double)(2 * ii[a] + 1) * (g->extent[a] / (2.0 * (double)g->n[a]));
        int n = vo_live_samples(t, q, smp);
        int inf = vo_in_fov(t, p, q);
        double m[4];
        vo_measure(t, p, q, m);
        double craw = m[2] / m[3];
        int vis = 0;
        if (inf && n > 0) {
            int64_t Q[3] = {0, 0, 0};
            for (int a = 0; a < J->dim; ++a)
                to_quanta(q[a], &Q[a]);
            for (int s = 0; s < n; ++s)
                for (int a = 0; a < 3; ++a)
                    sq[3 * s + a] = 0;
            for (int s = 0; s < n; ++s)
                for (int a = 0; a < J->dim; ++a)
                    to_quanta(smp[3 * s + a], &sq[3 * s + a]);
            for (int s = 0; s < n; ++s) {
                int blocked = 0;
                for (int64_t b = 0; b < J->nbox && !blocked; ++b)
                    blocked = seg_meets_box(J->dim, Q, &sq[3 * s], &J->blo[3 * b], &J->bhi[3 * b]);
                vis += !blocked;
            }
        }
        int cnt;
        double col;
        if (!inf || n == 0) {
            cnt = 0;
            col = 0.0;
        } else if (p->mode == VO_FRACTION) {
            cnt = vis;
            col = ((double)vis / (double)n) * craw;
        } else {
            cnt = (vis == n) ? n : 0;
            col = (vis == n) ? craw : 0.0;
        }
        double cbv;
        uint8_t bn;
        to_bin(p, col, m[3], &cbv, &bn);
        if (J->count) J->count[v] = (uint16_t)cnt;
        if (J->nlive) J->nlive[v] = (uint16_t)n;
        if (J->infov) J->infov[v] = (uint8_t)inf;
        if (J->c) J->c[v] = col;
        if (J->cb) J->cb[v] = cbv;
        if (J->bin) J->bin[v] = bn;
    }
    free(smp);
    free(sq);
}

static void *eval_thread(void *arg)
{
    eval_range((vo_job *)arg);
    return NULL;
}

/* Checks that every coordinate the map touches is a multiple of 2^-8. */
static int check_query(int dim, const vo_target *t, const vo_grid *g, const vo_params *p)
{
    int64_t dummy;
    if (dim != 2 && dim != 3) return -1;
    if (p->n_bins < 2 || p->n_bins > 256) return -1;
    if (t->su <= 0 || t->sv <= 0) return -1;
    if (t->kind == VO_VIEWER) {
        int64_t r;
        if (t->su != 1 || t->sv != 1 || !(t->size[0] > 0.0) || to_quanta(t->size[0], &r)) return -1;
        if (dim == 2 && t->center[2] != 0.0) return -1;
        if (!(2.0 * atan(target_size(t, p) / (2.0 * p->d0)) > mu_rad(p))) return -1;
    } else if ((t->kind == VO_SEGMENT) != (dim == 2)) {
        return -1;
    }
    if (t->kind != VO_CUBE && t->normal_axis != 0 && t->normal_axis != 1) return -1;
    if (t->kind == VO_CUBE && p->fov_deg < 360.0 && p->gaze == 0) return -1;
    if (p->gaze < -dim || p->gaze > dim) return -1;
    if (!(p->fov_deg > 0.0 && p->fov_deg <= 360.0)) return -1;
    if (!(p->mu_arcmin > 0.0) || !(p->d0 > 0.0)) return -1;
    for (int a = 0; a < dim; ++a) {
        if (g->n[a] <= 0) return -1;
        if (to_quanta(g->origin[a], &dummy)) return -1;
        if (to_quanta(g->extent[a] / (2.0 * (double)g->n[a]), &dummy)) return -1;
    }
    double q[3] = {1e300, 1e300, 1e300};
    int maxs = 6 * t->su * t->sv;
    double *smp = (double *)malloc(sizeof(double) * 3 * (size_t)maxs);
    int n = vo_live_samples(t, q, smp);
    /* a far viewpoint sees at most 3 cube faces; check all faces from both sides */
    int bad = 0;
    for (int s = 0; s < n; ++s)
        for (int a = 0; a < dim; ++a)
            if (to_quanta(smp[3 * s + a], &dummy)) bad = 1;
    double q2[3] = {-1e300, -1e300, -1e300};
    n = vo_live_samples(t, q2, smp);
    for (int s = 0; s < n; ++s)
        for (int a = 0; a < dim; ++a)
            if (to_quanta(smp[3 * s + a], &dummy)) bad = 1;
    free(smp);
    return bad ? -1 : 0;
}

/* Closed bounding box of the target (its extent along each axis). */
static void target_box(const vo_target *t, double *lo, double *hi)
{
    double half[3] = {0.0, 0.0, 0.0};
    if (t->kind == VO_VIEWER) {
        /* a point */
    } else if (t->kind == VO_CUBE) {
        half[0] = half[1] = half[2] = t->size[0] / 2.0;
    } else {
        half[1 - t->normal_axis] = t->size[0] / 2.0;
        if (t->kind == VO_BILLBOARD)
            half[2] = t->size[1] / 2.0;
    }
    for (int k = 0; k < 3; ++k) {
        lo[k] = t->center[k] - half[k];
        hi[k] = t->center[k] + half[k];
    }
}

/* Boxes in quanta, [box][3] (zeros beyond dim), in *blo_out / *bhi_out
 * (to be freed).  -1 if a coordinate is off the lattice, a box has lo > hi,
 * or a box meets the target's box: the target is not an obstacle (Def. 2.1
 * keeps them apart), so such a query is rejected. */
static int load_boxes(int dim, int64_t nbox, const double *lo, const double *hi, const vo_target *t,
                      int64_t **blo_out, int64_t **bhi_out)
{
    int64_t *blo = (int64_t *)calloc((size_t)(nbox > 0 ? nbox : 1) * 3, sizeof(int64_t));
    int64_t *bhi = (int64_t *)calloc((size_t)(nbox > 0 ? nbox : 1) * 3, sizeof(int64_t));
    int bad = 0;
    for (int64_t b = 0; b < nbox && !bad; ++b)
        for (int a = 0; a < dim; ++a)
            if (to_quanta(lo[a * nbox + b], &blo[3 * b + a]) || to_quanta(hi[a * nbox + b], &bhi[3 * b + a]) ||
                blo[3 * b + a] > bhi[3 * b + a])
                bad = 1;
    double tl[3], th[3];
    int64_t TL[3] = {0, 0, 0}, TH[3] = {0, 0, 0};
    target_box(t, tl, th);
    for (int a = 0; a < dim && !bad; ++a)
        if (to_quanta(tl[a], &TL[a]) || to_quanta(th[a], &TH[a]))
            bad = 1;
    for (int64_t b = 0; b < nbox && !bad; ++b) {
        int meet = 1;
        for (int a = 0; a < dim; ++a)
            meet = meet && blo[3 * b + a] <= TH[a] && bhi[3 * b + a] >= TL[a];
        bad = meet;
    }
    if (bad) {
        free(blo);
        free(bhi);
        return -1;
    }
    *blo_out = blo;
    *bhi_out = bhi;
    return 0;
}

/* Evaluate the VCM at the listed viewpoints (linear index, x fastest).
 * lo/hi: [3][nbox] SoA, multiples of 2^-8.  Any output pointer may be NULL.
 * count: FRACTION mode: visible live samples; FULL mode: N(q) when all are
 * visible, else 0; 0 outside the FOV.  c: colour; cb: colour in the bin's
 * scale.  Returns 0, or -1 on invalid input. */
int vo_eval(int dim, int64_t nbox, const double *lo, const double *hi,
            const vo_target *t, const vo_grid *g, const vo_params *p,
            const int64_t *vp, int64_t nvp, int nthreads,
            uint16_t *count, uint16_t *nlive, uint8_t *infov,
            double *c, double *cb, uint8_t *bin)
{
    if (check_query(dim, t, g, p))
        return -1;
    int64_t *blo, *bhi;
    if (load_boxes(dim, nbox, lo, hi, t, &blo, &bhi))
        return -1;
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    vo_job base = {dim, nbox, blo, bhi, t, g, p, vp, nvp, count, nlive, infov, bin, c, cb, 0, nvp};
    if (nthreads == 1) {
        eval_range(&base);
    } else {
        vo_job jobs[256];
        pthread_t th[256];
        for (int i = 0; i < nthreads; ++i) {
            jobs[i] = base;
            jobs[i].first = nvp * i / nthreads;
            jobs[i].last = nvp * (i + 1) / nthreads;
            pthread_create(&th[i], NULL, eval_thread, &jobs[i]);
        }
        for (int i = 0; i < nthreads; ++i)
            pthread_join(th[i], NULL);
    }
    free(blo);
    free(bhi);
    return 0;
}

/* ===================================================================== */
/* Pruned construction: equi-visible cells (Sec. III-A), MBR and tangent  */
/* approximations (Sec. IV-A), error metric (Sec. V-A).                   */
/* ===================================================================== */

typedef struct {
    int nring;          /* rings i = 0 .. nring-1                              */
    double *d;          /* d[0..nring]: ring i is [d[i], d[i+1]); d[nring] = d_max */
    int64_t *boff;      /* boff[0..nring]: bands of ring i are gam[boff[i] .. boff[i+1]-1] */
    double *gam;        /* per ring: gamma_0 = pi/2 > gamma_1 > ... > gamma_{L+1} = 0 (radians);
                           band j of the ring is (gamma_{j+1}, gamma_j]                   */
    double S, mu, d0, V0;
    int rings_only;     /* viewer-centric maps: one band per ring, colour facing */
} vo_cells;

/* Distance-based partition (Sec. III-A-1) followed by the angle-based
 * partition of every ring (Sec. III-A-2), in the paper's order.
 *
 * Rings: starting at the near point d0 with V0 = 2 arctan(S / 2 d0) (Eq. 1,
 * facing the target), the visual angle is lowered by mu per step and the
 * distance at which it is reached is the next ring boundary, while the
 * angle stays >= mu.  The last boundary is d_max, where V = mu (the
 * distance beyond which no difference is perceivable; Sec. IV-B uses the
 * same relation).  The k-th angle is computed as V0 - k mu.
 *
 * Bands of a ring: at the ring's middle distance d' the facing angle
 * W_0 = 2 arctan(S / 2 d') is lowered by mu per step; each W_j is the visual
 * angle of a perceived size S_j = 2 d' tan(W_j / 2), which Eq. 2 attributes
 * to the viewing angle gamma_j = 90 deg * S_j / S.  The band boundaries are
 * these angles, from 90 deg down, while W_j >= mu; the last band reaches 0. */
static int partition(double S, double mu, double d0, int rings_only, vo_cells *out)
{
    memset(out, 0, sizeof(*out));
    if (!(S > 0) || !(mu > 0) || !(d0 > 0))
        return -1;
    double V0 = 2.0 * atan(S / (2.0 * d0));
    if (!(V0 > mu))
        return -1;
    int cap = 1024, nr = 0;
    double *d = (double *)malloc(sizeof(double) * (size_t)cap);
    d[0] = d0;
    for (int k = 1;; ++k) {
        double V = V0 - k * mu;
        if (V < mu)
            break;
        if (k + 1 >= cap) {
            cap *= 2;
            d = (double *)realloc(d, sizeof(double) * (size_t)cap);
        }
        d[k] = S / (2.0 * tan(V / 2.0));
        nr = k;
    }
    /* nr = K: boundaries d[0..K]; ring K ends at d_max */
    if (nr + 2 >= cap)
        d = (double *)realloc(d, sizeof(double) * (size_t)(nr + 2));
    d[nr + 1] = S / (2.0 * tan(mu / 2.0));
    int nring = nr + 1;
    int64_t *boff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nring + 1));
    int64_t gcap = 4096, gn = 0;
    double *gam = (double *)malloc(sizeof(double) * (size_t)gcap);
    for (int i = 0; i < nring; ++i) {
        boff[i] = gn;
        double dp = 0.5 * (d[i] + d[i + 1]);
        double W0 = 2.0 * atan(S / (2.0 * dp));
        if (gn + 2 >= gcap) {
            gcap *= 2;
            gam = (double *)realloc(gam, sizeof(double) * (size_t)gcap);
        }
        gam[gn++] = VO_PI / 2.0;
        for (int j = 1; !rings_only; ++j) {
            double W = W0 - j * mu;
            if (W < mu)
                break;
            double Sj = 2.0 * dp * tan(W / 2.0);
            if (gn + 2 >= gcap) {
                gcap *= 2;
                gam = (double *)realloc(gam, sizeof(double) * (size_t)gcap);
            }
            gam[gn++] = (VO_PI / 2.0) * Sj / S;
        }
        gam[gn++] = 0.0;
    }
    boff[nring] = gn;
    out->nring = nring;
    out->d = d;
    out->boff = boff;
    out->gam = gam;
    out->S = S;
    out->mu = mu;
    out->d0 = d0;
    out->V0 = V0;
    out->rings_only = rings_only;
    return 0;
}

int vo_partition(double S, double mu, double d0, vo_cells *out) { return partition(S, mu, d0, 0, out); }

/* The partition of a viewer-centric map (Sec. IV-B): a point seen facing
 * has no viewing angle to tell apart, so its equi-visible cells are the
 * distance rings of Sec. III-A-1 alone, one band from 90 degrees to 0 each,
 * coloured by the facing visual angle at the ring's middle distance. */
int vo_partition_rings(double S, double mu, double d0, vo_cells *out) { return partition(S, mu, d0, 1, out); }

void vo_free_cells(vo_cells *c)
{
    free(c->d);
    free(c->boff);
    free(c->gam);
    memset(c, 0, sizeof(*c));
}

int vo_cells_size(const vo_cells *c, int64_t *n_bands_total) { *n_bands_total = c->boff[c->nring]; return c->nring; }
void vo_cells_copy(const vo_cells *c, double *d, int64_t *boff, double *gam)
{
    memcpy(d, c->d, sizeof(double) * (size_t)(c->nring + 1));
    memcpy(boff, c->boff, sizeof(int64_t) * (size_t)(c->nring + 1));
    memcpy(gam, c->gam, sizeof(double) * (size_t)c->boff[c->nring]);
}

/* Visual angle at distance D and viewing angle alpha (Eq. 1 with Eq. 2). */
static double vis_angle(double S, double D, double alpha)
{
    return 2.0 * atan((alpha / (VO_PI / 2.0)) * S / (2.0 * D));
}

/* Colour of cell (i, j): the visual angle at the cell's centre (Sec.
 * III-A, after the partitioning steps), taken in parameter space as the
 * ring's middle distance and the band's middle angle, divided by V0. */
static double cell_colour(const vo_cells *c, int i, int j)
{
    const double *g = c->gam + c->boff[i];
    double dp = 0.5 * (c->d[i] + c->d[i + 1]);
    double gm = 0.5 * (g[j] + g[j + 1]);
    if (c->rings_only)
        gm = VO_PI / 2.0;
    return vis_angle(c->S, dp, gm) / c->V0;
}

static int n_bands(const vo_cells *c, int i) { return (int)(c->boff[i + 1] - c->boff[i]) - 1; }

/* Band of viewing angle alpha in ring i: (gamma_{j+1}, gamma_j], the last
 * band closed at 0. */
static int band_of(const vo_cells *c, int i, double alpha)
{
    const double *g = c->gam + c->boff[i];
    int L = n_bands(c, i);
    for (int j = 0; j < L; ++j)
        if (alpha > g[j + 1])
            return j;
    return L - 1;
}

/* Ring of distance D: [d_i, d_{i+1}); below d0 counts as ring 0; -1 at or
 * beyond d_max. */
static int ring_of(const vo_cells *c, double D)
{
    if (D >= c->d[c->nring])
        return -1;
    int i = 0;
    while (i + 1 < c->nring && D >= c->d[i + 1])
        ++i;
    return i;
}

/* Per-viewpoint colours of the three pruned constructions from the
 * meridian coordinates (D, alpha) of q (first quadrant, Sec. III-A-2):
 *   E: colour of q's own cell;
 *   M: colour of the first cell, lowest ring then lowest band, whose closed
 *      MBR in the (rho, h) plane contains q (Sec. IV-A, MBR approximation);
 *   T: colour of the first ring whose tangent trapezoid, the band of alpha
 *      bounded by the tangents of the ring's arcs at the band's middle
 *      angle, contains q (Sec. IV-A, tangential approximation); when no
 *      trapezoid contains q the exact cell is used and *t_fallback set.
 * Beyond d_max all three are 0.  out = {cE, cM, cT}; ring/band of E too. */
void vo_pruned_colours(const vo_cells *c, double D, double alpha, double *out, int *cell,
                       int *t_fallback)
{
    out[0] = out[1] = out[2] = 0.0;
    cell[0] = cell[1] = -1;
    *t_fallback = 0;
    int ir = ring_of(c, D);
    if (ir < 0)
        return;
    int jb = band_of(c, ir, alpha);
    cell[0] = ir;
    cell[1] = jb;
    out[0] = cell_colour(c, ir, jb);
    double rho = D * cos(alpha), h = D * sin(alpha);
    /* MBR: the cell is the annular sector d in [d_i, d_{i+1}], angle in
     * [gamma_{j+1}, gamma_j]; its bounding box in the (rho, h) quadrant. */
    int found = 0;
    for (int i = 0; i < c->nring && !found; ++i) {
        /* a ring's MBRs lie within sqrt(2) d_{i+1} of the centre */
        if (sqrt(2.0) * c->d[i + 1] < D)
            continue;
        const double *g = c->gam + c->boff[i];
        int L = n_bands(c, i);
        for (int j = 0; j < L; ++j) {
            double r0 = c->d[i] * cos(g[j]), r1 = c->d[i + 1] * cos(g[j + 1]);
            double h0 = c->d[i] * sin(g[j + 1]), h1 = c->d[i + 1] * sin(g[j]);
            if (rho >= r0 && rho <= r1 && h >= h0 && h <= h1) {
                out[1] = cell_colour(c, i, j);
                found = 1;
                break;
            }
        }
    }
    if (!found)
        out[1] = out[0];
    /* Tangents: for each ring, the band containing alpha and the projection
     * of q on the direction of the band's middle angle. */
    found = 0;
    for (int i = 0; i < c->nring; ++i) {
        int j = band_of(c, i, alpha);
        const double *g = c->gam + c->boff[i];
        double gm = 0.5 * (g[j] + g[j + 1]);
        double p = D * cos(alpha - gm);
        if (p >= c->d[i] && p < c->d[i + 1]) {
            out[2] = cell_colour(c, i, j);
            found = 1;
            break;
        }
    }
    if (!found) {
        out[2] = out[0];
        *t_fallback = 1;
    }
}

/* Meridian coordinates of q relative to the target: D and alpha as in the
 * measure (h along the normal axis, rho the rest). */
static void meridian(const vo_target *t, const double *q, double *D, double *alpha)
{
    double dl[3];
    for (int k = 0; k < 3; ++k)
        dl[k] = q[k] - t->center[k];
    if (t->kind == VO_SEGMENT)
        dl[2] = 0.0;
    int nax;
    if (t->kind == VO_CUBE) {
        nax = 0;
        for (int k = 1; k < 3; ++k)
            if (fabs(dl[k]) > fabs(dl[nax]))
                nax = k;
    } else {
        nax = t->normal_axis;
    }
    double h = fabs(dl[nax]), r2 = 0.0;
    for (int k = 0; k < 3; ++k)
        if (k != nax)
            r2 += dl[k] * dl[k];
    *D = sqrt(r2 + h * h);
    *alpha = atan2(h, sqrt(r2));
}

void vo_meridian(const vo_target *t, const double *q, double *out)
{
    meridian(t, q, &out[0], &out[1]);
}

/* ===================================================================== */
/* Visible-region blocks (Sec. III-C-1, "Indexing Visible Regions"): a    */
/* block of viewpoints is decided when the target is seen completely from  */
/* all of it or from none of it; otherwise it is split, down to the        */
/* minimum block size.                                                     */
/* ===================================================================== */

/* Does the closed box [a, c] meet the convex hull of the box [L, H] and the
 * point s?  That hull is the union over lambda in [0, 1] of the boxes
 * [s + lambda (L - s), s + lambda (H - s)], so the box meets it iff some
 * lambda in [0, 1] satisfies, along every axis k,
 *   s_k + lambda (L_k - s_k) <= c_k   and   s_k + lambda (H_k - s_k) >= a_k,
 * each a bound on lambda of the form lambda x <= y.  Bounds are fractions
 * compared by cross-multiplication: exact in quanta. */
static int hull_meets_box(int dim, const int64_t *L, const int64_t *H, const int64_t *s,
                          const int64_t *a, const int64_t *c)
{
    int64_t ln = 0, ld = 1, un = 1, ud = 1; /* lambda in [ln/ld, un/ud] */
    for (int k = 0; k < dim; ++k)
        for (int side = 0; side < 2; ++side) {
            int64_t x = side ? s[k] - H[k] : L[k] - s[k];
            int64_t y = side ? s[k] - a[k] : c[k] - s[k];
            if (x > 0) {
                if (y * ud < un * x) { /* lambda <= y / x is tighter */
                    un = y;
                    ud = x;
                }
            } else if (x < 0) {
                if (-y * ld > ln * -x) { /* lambda >= (-y) / (-x) is tighter */
                    ln = -y;
                    ld = -x;
                }
            } else if (y < 0) {
                return 0;
            }
        }
    return ln * ud <= un * ld;
}

/* Field of view over a box of viewpoints given by its corners: 1 if every
 * viewpoint of the box is inside, 0 if every one is outside, -1 if that
 * cannot be told from the corners.  A set that is convex contains the box
 * when it contains the corners: the wedge itself when it is no wider than a
 * half-space, else the half-space in front of the target; the half-space
 * behind the target, else the complement of a wide wedge (a convex cone). */
static int fov_class(const vo_target *t, const vo_params *p, int nc, const double (*cq)[3])
{
    /* the region of a viewer-centric map: the ball is convex, so corners
     * inside put the box inside; the box is outside when its nearest point
     * to the viewer is farther than d_max */
    int region = 1;
    if (t->kind == VO_VIEWER) {
        int all_in = 1;
        double g2 = 0.0;
        for (int c = 0; c < nc; ++c)
            all_in = all_in && in_region(t, cq[c]);
        for (int k = 0; k < 3; ++k) {
            double lo = cq[0][k], hi = cq[nc - 1][k], x = t->center[k];
            double gap = x < lo ? lo - x : (x > hi ? x - hi : 0.0);
            g2 += gap * gap;
        }
        region = all_in ? 1 : (g2 > t->size[0] * t->size[0] ? 0 : -1);
        if (region == 0)
            return 0;
    }
    int wedge;
    double half = p->fov_deg / 2.0;
    if (half >= 180.0) {
        wedge = 1;
    } else {
        int all_in = 1, all_out = 1, all_front = 1, all_back = 1;
        int ax, sg;
        wedge_axis(t, p, &ax, &sg);
        for (int c = 0; c < nc; ++c) {
            int in = in_wedge(t, p, cq[c]);
            double dn = sg * (cq[c][ax] - t->center[ax]);
            all_in = all_in && in;
            all_out = all_out && !in;
            all_front = all_front && dn >= 0.0;
            all_back = all_back && dn < 0.0;
        }
        if (half <= 90.0)
            wedge = all_in ? 1 : (all_back ? 0 : -1);
        else
            wedge = all_front ? 1 : (all_out ? 0 : -1);
    }
    if (wedge == 0)
        return 0;
    return (region == 1 && wedge == 1) ? 1 : -1;
}

/* Classify the block of viewpoints with grid indices lo[a] .. hi[a]
 * (inclusive) as a whole.  Its viewpoints lie in the box spanned by the
 * block's extreme viewpoints; C denotes that box.
 *   - The live samples and the field of view must be the same for all of C
 *     (each live-face condition is a half-space; the field of view by
 *     fov_class), else the block is undecided.
 *   - Outside the field of view, or with no live sample: decided, count 0.
 *   - A live sample s is seen from all of C when no obstacle meets the
 *     convex hull of C and s (every line of sight lies in it); it is hidden
 *     from all of C when one obstacle o meets the segments from every
 *     corner of C to s (the points whose segment to s meets o form a convex
 *     set, so it holds C).
 *   - FULL mode: some live sample hidden from all of C: decided, count 0;
 *     every live sample seen from all of C: decided, count N; else
 *     undecided.
 *   - FRACTION mode: every live sample either seen from or hidden from all
 *     of C: decided, count = the samples seen; else undecided.
 * A decided block gives every one of its viewpoints the count, live count
 * and field of view the brute force gives it.  Returns 1 (decided) with
 * out = {count, N, in FOV}, else 0.  Boxes in quanta, [box][3]. */
static int classify_block(int dim, int64_t nbox, const int64_t *blo, const int64_t *bhi,
                          const vo_target *t, const vo_grid *g, const vo_params *p,
                          const int64_t *lo, const int64_t *hi, int *out)
{
    int nc = 1 << dim;
    double cq[8][3];
    int64_t CQ[8][3], L[3] = {0, 0, 0}, H[3] = {0, 0, 0};
    for (int c = 0; c < nc; ++c)
        for (int a = 0; a < 3; ++a) {
            cq[c][a] = 0.0;
            CQ[c][a] = 0;
            if (a < dim) {
                int64_t i = ((c >> a) & 1) ? hi[a] : lo[a];
                cq[c][a] = g->origin[a] + (double)(2 * i + 1) * (g->extent[a] / (2.0 * (double)g->n[a]));
                to_quanta(cq[c][a], &CQ[c][a]);
            }
        }
    for (int a = 0; a < dim; ++a) {
        L[a] = CQ[0][a];
        H[a] = CQ[nc - 1][a];
    }
    /* live samples: the same set at every corner */
    int maxs = 6 * t->su * t->sv;
    double *smp = (double *)malloc(sizeof(double) * 3 * (size_t)maxs);
    double *tmp = (double *)malloc(sizeof(double) * 3 * (size_t)maxs);
    int n = vo_live_samples(t, cq[0], smp);
    int uniform = 1;
    for (int c = 1; c < nc && uniform; ++c) {
        int m = vo_live_samples(t, cq[c], tmp);
        uniform = m == n && memcmp(smp, tmp, sizeof(double) * 3 * (size_t)n) == 0;
    }
    free(tmp);
    int fc = fov_class(t, p, nc, cq);
    if (!uniform || fc < 0) {
        free(smp);
        return 0;
    }
    out[1] = n;
    out[2] = fc;
    if (fc == 0 || n == 0) {
        out[0] = 0;
        free(smp);
        return 1;
    }
    int seen = 0, hidden = 0;
    for (int s = 0; s < n; ++s) {
        int64_t S[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a)
            to_quanta(smp[3 * s + a], &S[a]);
        int vis = 1, hid = 0;
        for (int64_t b = 0; b < nbox && !hid; ++b) {
            if (!hull_meets_box(dim, L, H, S, &blo[3 * b], &bhi[3 * b]))
                continue;
            vis = 0;
            int all = 1;
            for (int c = 0; c < nc && all; ++c)
                all = seg_meets_box(dim, CQ[c], S, &blo[3 * b], &bhi[3 * b]);
            hid = all;
        }
        seen += vis;
        hidden += hid;
        if (p->mode == VO_FULL && hid)
            break;
    }
    free(smp);
    if (p->mode == VO_FULL) {
        if (hidden) {
            out[0] = 0;
            return 1;
        }
        if (seen == n) {
            out[0] = n;
            return 1;
        }
        return 0;
    }
    if (seen + hidden == n) {
        out[0] = seen;
        return 1;
    }
    return 0;
}

/* Side of the smallest blocks for a minimum block size theta (viewpoints):
 * blocks are halved, so it is the largest power of two not above theta. */
static int64_t leaf_side(int theta)
{
    int64_t s = 1;
    while (2 * s <= theta)
        s *= 2;
    return s;
}

/* The smallest block holding viewpoint idx: aligned blocks of `side`
 * viewpoints per axis, cut by the grid's end; its index ranges and its
 * representative, the lowest-index viewpoint of its centre. */
static void leaf_block(const vo_grid *g, int dim, int64_t side, int64_t idx, int64_t *lo, int64_t *hi,
                       int64_t *rep, int64_t *key)
{
    int64_t ii[3] = {idx % g->n[0], (idx / g->n[0]) % g->n[1], idx / (g->n[0] * g->n[1])};
    int64_t r[3] = {0, 0, 0}, b[3] = {0, 0, 0}, nb[3] = {1, 1, 1};
    for (int a = 0; a < 3; ++a) {
        lo[a] = hi[a] = 0;
        if (a >= dim)
            continue;
        b[a] = ii[a] / side;
        nb[a] = (g->n[a] + side - 1) / side;
        lo[a] = b[a] * side;
        hi[a] = lo[a] + side - 1 < g->n[a] - 1 ? lo[a] + side - 1 : g->n[a] - 1;
        int64_t off = (side - 1) / 2;
        r[a] = lo[a] + (off < hi[a] - lo[a] ? off : hi[a] - lo[a]);
    }
    *rep = r[0] + g->n[0] * (r[1] + g->n[1] * r[2]);
    *key = b[0] + nb[0] * (b[1] + nb[1] * b[2]);
}

/* Public wrappers (pins).  vo_hull_meets_box: 1 if the closed box [a, c]
 * meets the convex hull of the box [L, H] and the point s, 0 if not, -1 on
 * input off the lattice. */
int vo_hull_meets_box(int dim, const double *L, const double *H, const double *s, const double *a,
                      const double *c)
{
    int64_t l[3] = {0, 0, 0}, h[3] = {0, 0, 0}, S[3] = {0, 0, 0}, A[3] = {0, 0, 0}, C[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k)
        if (to_quanta(L[k], &l[k]) || to_quanta(H[k], &h[k]) || to_quanta(s[k], &S[k]) ||
            to_quanta(a[k], &A[k]) || to_quanta(c[k], &C[k]) || l[k] > h[k] || A[k] > C[k])
            return -1;
    return hull_meets_box(dim, l, h, S, A, C);
}

/* vo_classify_block: the classification of the block of viewpoints with
 * grid indices lo[a] .. hi[a]: 1 (decided, out = {count, N, in FOV}),
 * 0 (undecided), -1 (invalid input). */
int vo_classify_block(int dim, int64_t nbox, const double *lo, const double *hi, const vo_target *t,
                      const vo_grid *g, const vo_params *p, const int64_t *ilo, const int64_t *ihi, int *out)
{
    if (check_query(dim, t, g, p))
        return -1;
    for (int a = 0; a < dim; ++a)
        if (ilo[a] < 0 || ihi[a] < ilo[a] || ihi[a] >= g->n[a])
            return -1;
    int64_t *blo, *bhi;
    if (load_boxes(dim, nbox, lo, hi, t, &blo, &bhi))
        return -1;
    int r = classify_block(dim, nbox, blo, bhi, t, g, p, ilo, ihi, out);
    free(blo);
    free(bhi);
    return r;
}

/* Representative viewpoint of q for a minimum block size theta: the
 * lowest-index centre viewpoint of q's smallest block (side: the largest
 * power of two not above theta; cut by the grid's end).  A smallest block
 * that is not decided takes its representative's visibility (Sec. III-C-1
 * stops splitting there; the baseline of Sec. V-B likewise uses one point
 * per grid cell).  theta = 1 gives q itself. */
int64_t vo_block_rep(const vo_grid *g, int dim, int theta, int64_t idx)
{
    int64_t lo[3], hi[3], rep, key;
    leaf_block(g, dim, leaf_side(theta), idx, lo, hi, &rep, &key);
    return rep;
}

typedef struct {
    int dim;
    int64_t nbox;
    const int64_t *blo, *bhi;
    const vo_target *t;
    const vo_grid *g;
    const vo_params *p;
    int64_t side;
    const int64_t *leaf_vp; /* one viewpoint of each leaf */
    int *decided, *gate;    /* per leaf: decided, {count, N, in FOV} */
    int64_t first, last;
} vo_leaf_job;

static void *classify_thread(void *arg)
{
    vo_leaf_job *J = (vo_leaf_job *)arg;
    for (int64_t u = J->first; u < J->last; ++u) {
        int64_t lo[3], hi[3], rep, key;
        leaf_block(J->g, J->dim, J->side, J->leaf_vp[u], lo, hi, &rep, &key);
        J->decided[u] = classify_block(J->dim, J->nbox, J->blo, J->bhi, J->t, J->g, J->p, lo, hi, &J->gate[3 * u]);
    }
    return NULL;
}

typedef struct {
    int64_t key, v;
} vo_keyed;

static int cmp_keyed(const void *a, const void *b)
{
    const vo_keyed *x = (const vo_keyed *)a, *y = (const vo_keyed *)b;
    if (x->key != y->key)
        return x->key < y->key ? -1 : 1;
    return x->v < y->v ? -1 : (x->v > y->v);
}

/* Pruned VCM at the listed viewpoints: method 1 = E, 2 = M, 3 = T.
 * The gate (visible count, N(q), FOV) of q comes from q's smallest block
 * (side: the largest power of two not above theta): if that block is
 * decided as a whole (classify_block), its count; otherwise the brute-force
 * oracle at the block's representative.  (A block that is decided keeps
 * every sub-block decided, so the blocks above the smallest ones do not
 * change the map: the quad-/oct-tree only saves work.)  The colour comes
 * from the cell lookups at q.  count/c/cb/bin as in vo_eval; cell_out:
 * ring, band of q's own cell; decided_out: 1 where q's block was decided. */
int vo_eval_pruned(int dim, int64_t nbox, const double *lo, const double *hi,
                   const vo_target *t, const vo_grid *g, const vo_params *p,
                   int method, int theta, const int64_t *vp, int64_t nvp, int nthreads,
                   uint16_t *count, double *c, double *cb, uint8_t *bin, int32_t *cell_out,
                   uint8_t *t_fallback, uint8_t *decided_out)
{
    if (method < 1 || method > 3 || theta < 1)
        return -1;
    if (check_query(dim, t, g, p))
        return -1;
    int64_t *blo, *bhi;
    if (load_boxes(dim, nbox, lo, hi, t, &blo, &bhi))
        return -1;
    vo_cells cells;
    double mu = mu_rad(p);
    if (partition(target_size(t, p), mu, p->d0, t->kind == VO_VIEWER, &cells)) {
        free(blo);
        free(bhi);
        return -1;
    }
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    int64_t side = leaf_side(theta);
    size_t nv = (size_t)(nvp > 0 ? nvp : 1);
    /* the smallest block of every viewpoint, each distinct block once */
    vo_keyed *kv = (vo_keyed *)malloc(sizeof(vo_keyed) * nv);
    int64_t *rep_of = (int64_t *)malloc(sizeof(int64_t) * nv);
    for (int64_t v = 0; v < nvp; ++v) {
        int64_t l[3], h[3];
        leaf_block(g, dim, side, vp[v], l, h, &rep_of[v], &kv[v].key);
        kv[v].v = v;
    }
    qsort(kv, (size_t)nvp, sizeof(vo_keyed), cmp_keyed);
    int64_t *leaf_of = (int64_t *)malloc(sizeof(int64_t) * nv); /* viewpoint -> distinct block */
    int64_t *leaf_vp = (int64_t *)malloc(sizeof(int64_t) * nv);
    int64_t nleaf = 0;
    for (int64_t k = 0; k < nvp; ++k) {
        if (k == 0 || kv[k].key != kv[k - 1].key)
            leaf_vp[nleaf++] = vp[kv[k].v];
        leaf_of[kv[k].v] = nleaf - 1;
    }
    int *decided = (int *)calloc((size_t)(nleaf > 0 ? nleaf : 1), sizeof(int));
    int *lgate = (int *)calloc((size_t)(nleaf > 0 ? nleaf : 1) * 3, sizeof(int));
    {
        vo_leaf_job base = {dim, nbox, blo, bhi, t, g, p, side, leaf_vp, decided, lgate, 0, nleaf};
        vo_leaf_job jobs[256];
        pthread_t th[256];
        int nt = nleaf < nthreads ? (int)(nleaf > 0 ? nleaf : 1) : nthreads;
        for (int i = 0; i < nt; ++i) {
            jobs[i] = base;
            jobs[i].first = nleaf * i / nt;
            jobs[i].last = nleaf * (i + 1) / nt;
            if (nt == 1)
                classify_thread(&jobs[i]);
            else
                pthread_create(&th[i], NULL, classify_thread, &jobs[i]);
        }
        if (nt > 1)
            for (int i = 0; i < nt; ++i)
                pthread_join(th[i], NULL);
    }
    /* representatives of the undecided blocks, by the brute-force oracle */
    int64_t *reps = (int64_t *)malloc(sizeof(int64_t) * nv);
    int64_t nrep = 0;
    for (int64_t v = 0; v < nvp; ++v)
        if (!decided[leaf_of[v]])
            reps[nrep++] = rep_of[v];
    size_t nr = (size_t)(nrep > 0 ? nrep : 1);
    uint16_t *rc = (uint16_t *)malloc(sizeof(uint16_t) * nr);
    uint16_t *rn = (uint16_t *)malloc(sizeof(uint16_t) * nr);
    uint8_t *rf = (uint8_t *)malloc(nr);
    int r = nrep > 0 ? vo_eval(dim, nbox, lo, hi, t, g, p, reps, nrep, nthreads, rc, rn, rf, NULL, NULL, NULL) : 0;
    if (r == 0) {
        int64_t k = 0;
        for (int64_t v = 0; v < nvp; ++v) {
            int64_t idx = vp[v];
            int64_t ii[3] = {idx % g->n[0], (idx / g->n[0]) % g->n[1], idx / (g->n[0] * g->n[1])};
            double q[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < dim; ++a)
                q[a] = g->origin[a] + (double)(2 * ii[a] + 1) * (g->extent[a] / (2.0 * (double)g->n[a]));
            double D, al, cols[3];
            int cl[2], tf;
            meridian(t, q, &D, &al);
            vo_pruned_colours(&cells, D, al, cols, cl, &tf);
            double craw = cols[method - 1];
            int u = (int)leaf_of[v];
            int vis, n, inf;
            if (decided[u]) {
                vis = lgate[3 * u];
                n = lgate[3 * u + 1];
                inf = lgate[3 * u + 2];
            } else {
                vis = rc[k];
                n = rn[k];
                inf = rf[k];
                ++k;
            }
            double col;
            if (!inf || n == 0)
                col = 0.0;
            else if (p->mode == VO_FRACTION)
                col = ((double)vis / (double)n) * craw;
            else
                col = (vis == n) ? craw : 0.0;
            double cbv;
            uint8_t bn;
            to_bin(p, col, cells.V0, &cbv, &bn);
            if (count) count[v] = (uint16_t)vis;
            if (c) c[v] = col;
            if (cb) cb[v] = cbv;
            if (bin) bin[v] = bn;
            if (cell_out) {
                cell_out[2 * v] = cl[0];
                cell_out[2 * v + 1] = cl[1];
            }
            if (t_fallback) t_fallback[v] = (uint8_t)tf;
            if (decided_out) decided_out[v] = (uint8_t)decided[u];
        }
    }
    free(kv);
    free(rep_of);
    free(leaf_of);
    free(leaf_vp);
    free(decided);
    free(lgate);
    free(reps);
    free(rc);
    free(rn);
    free(rf);
    free(blo);
    free(bhi);
    vo_free_cells(&cells);
    return r;
}

/* Approximation error of Sec. V-A: sum_i (c_e A - c_a A) / sum_i c_e A over
 * equal-size viewpoint cells, and the same with |c_e - c_a|. */
void vo_map_error(const double *ce, const double *ca, int64_t n, double *signed_err, double *abs_err)
{
    double num = 0.0, den = 0.0, ab = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        num += ce[i] - ca[i];
        ab += fabs(ce[i] - ca[i]);
        den += ce[i];
    }
    *signed_err = den > 0 ? num / den : 0.0;
    *abs_err = den > 0 ? ab / den : 0.0;
}

/* Measured approximation error in the units of the Sec. IV-A bounds.  Each
 * of the n viewpoints, given by its meridian coordinates (D[k], alpha[k]),
 * stands for a region of size A (an area in 2-D, a volume in 3-D); the sums
 * over the viewpoints of |V_M - V_E| A and |V_T - V_E| A are returned in
 * out[0] and out[1], visual angles in radians (colours times V0). */
void vo_bound_measured(const vo_cells *c, int64_t n, const double *D, const double *alpha,
                       double A, double *out)
{
    double m = 0.0, t = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double col[3];
        int cell[2], tf;
        vo_pruned_colours(c, D[k], alpha[k], col, cell, &tf);
        m += fabs(col[1] - col[0]) * c->V0 * A;
        t += fabs(col[2] - col[0]) * c->V0 * A;
    }
    out[0] = m;
    out[1] = t;
}

/* Error bounds of Sec. IV-A, evaluated as printed, per ring i with radii
 * r_i = d_i, r_{i+1} = d_{i+1}:
 *   MBR:     dr = sqrt(2) r_{i+1};             bands counted below
 *            arctan(r_{i+1} / (S/2));
 *   tangent: dr = sqrt(r_{i+1}^2 + (r_{i+1} - r_i)^2); bands counted below
 *            arctan(r_{i+1} / (S/2 + r_i));
 *   n = (dr - r_{i+1}) / (r_{i+1} - r_i), a_i = number of such bands,
 *   dc = n a_i mu, E = sum over the ring's cells of dc * A_cell,
 * A_cell the cell's area in the (rho, h) quadrant (2-D) or its volume of
 * revolution about the normal axis (3-D).  out = {E_MBR, E_Tangent}.
 * Pinned only from below (they must exceed the measured error of
 * vo_bound_measured over the whole region, for one quadrant in 2-D and one
 * half-space in 3-D) and by 0 < E_Tangent < E_MBR: the paper prints no value
 * of either bound for a scene that can be rebuilt here. */
void vo_error_bounds(const vo_cells *c, int dim, double *out)
{
    double E[2] = {0.0, 0.0};
    for (int i = 0; i < c->nring; ++i) {
        double r0 = c->d[i], r1 = c->d[i + 1];
        if (!(r1 > r0))
            continue;
        const double *g = c->gam + c->boff[i];
        int L = n_bands(c, i);
        double drs[2] = {sqrt(2.0) * r1, sqrt(r1 * r1 + (r1 - r0) * (r1 - r0))};
        double lim[2] = {atan(r1 / (c->S / 2.0)), atan(r1 / (c->S / 2.0 + r0))};
        for (int m = 0; m < 2; ++m) {
            double n = (drs[m] - r1) / (r1 - r0);
            int a = 0;
            for (int j = 0; j < L; ++j)
                if (g[j + 1] < lim[m])
                    ++a;
            double dc = n * a * c->mu;
            double area = 0.0;
            for (int j = 0; j < L; ++j) {
                double g0 = g[j + 1], g1 = g[j];
                if (dim == 2)
                    area += 0.5 * (g1 - g0) * (r1 * r1 - r0 * r0);
                else /* revolve the sector about the h axis: 2 pi * int rho dA */
                    area += 2.0 * VO_PI * (r1 * r1 * r1 - r0 * r0 * r0) / 3.0 * (sin(g1) - sin(g0));
            }
            E[m] += dc * area;
        }
    }
    out[0] = E[0];
    out[1] = E[1];
}
