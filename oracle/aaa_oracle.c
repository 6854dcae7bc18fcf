/*
 * aaa_oracle.c -- plain, slow FP64 CPU reference of the AAA-Gaussians
 * rasterisation path (arXiv 2504.12811).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP path.
 *
 * Everything is computed in double precision from the definitions:
 *   - Gaussian primitive, Sec. 3.1 Eq.(1)-(3).
 *   - Response = maximum of the Gaussian along the pixel's line (Sec. 3.1,
 *     "Evaluation in 3D", Eq.(4)-(5)).  The oracle writes the maximum out as
 *     the closed-form minimum over t of the Mahalanobis distance of o + t r,
 *     i.e. the ray form, not the screen-plane form used by the kernels.
 *   - Adaptive 3D filter, Sec. 3.2 Eq.(6), (10)-(13); volume-normalised
 *     variant Eq.(7)-(8) behind a flag.
 *   - Camera-inside discard, Sec. 3.3.
 *   - 3D frustum culling, Sec. 3.4 Eq.(18): exact minimum of rho^2 over a
 *     pyramid by enumeration of every active set (faces, edges, apex).
 *   - Hierarchical ordering (Sec. 3.1 "Blending Sort Order", Sec. 4 impl.
 *     details): tile list ordered by a per-tile 3D depth, then a bounded
 *     per-ray window keyed by the per-pixel depth of maximum response.
 *   - Front-to-back alpha blending with early termination (3DGS lineage).
 *
 * Where the paper is silent, the reading taken is stated at its use below.
 * Candidate lists are a conservative bounding sphere (its own acceleration);
 * extra candidates are filtered out by the per-pixel test and cannot change
 * the result.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_TILE 16

typedef struct {
    int64_t n;
    int32_t sh_degree;
    int32_t _pad;
    /* double precision so that finite differences can perturb inputs;
     * float32 scenes convert exactly */
    const double *means;          /* [3][n] */
    const double *log_scales;     /* [3][n] */
    const double *quats;          /* [4][n] (w,x,y,z) */
    const double *opacity_logits; /* [n] */
    const double *sh;             /* [(deg+1)^2][3][n] */
    const double *v_train;        /* [n] or NULL */
} or_scene;

typedef struct {
    double viewmat[16]; /* world -> view, row-major; +x right, +y down, +z forward */
    double fx, fy, cx, cy;
    int32_t width, height;
    double znear;
    double bg[3];
} or_camera;

typedef struct {
    double filter_k;
    int32_t ray_window;  /* K; 0 = blend in tile order */
    int32_t filter_mode; /* 0 adaptive (Eq.12), 1 off, 2 volume-normalised (Eq.8) */
    double alpha_min, alpha_max, t_min;
    /* relative bands inside which an FP32 decision may legitimately differ */
    double band_alpha, band_z, band_tie, band_T;
    /* 1: the middle level of the hierarchical sort, an exact re-sort of each
     * 8x8 sub-tile's entries by the depth on the sub-tile-centre line */
    int32_t subtile_sort;
    int32_t pad_;
} or_settings;

enum { OR_VISIBLE = 0, OR_INVALID = 1, OR_LOW_OPACITY = 2, OR_CAM_INSIDE = 3, OR_OUTSIDE = 4 };

typedef struct {
    int32_t status;
    int32_t ambiguous; /* camera-inside decision within band: pixels it would touch are flagged */
    double alpha, alpha_t, tau, filter_a;
    double s[3], s_t[3];
    double R[9];   /* row-major; world offset = R * diag(s) * g */
    double mu[3], mu_v[3], o[3];
    double o_g[3]; /* camera centre in normalised (filtered) Gaussian space */
    double A[9];   /* view-space direction -> normalised Gaussian space: S~^-1 R^T R_V^T */
    double M[9];   /* normalised Gaussian space -> view space: R_V R S~ (row-major) */
    double color[3];
    double dir[3]; /* unit direction camera -> mean (world) */
} or_gauss;

/* ------------------------------------------------------------------------ */
/* small linear algebra                                                       */

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static void matvec3(const double *m, const double *v, double *out)
{
    for (int i = 0; i < 3; ++i) out[i] = m[3 * i] * v[0] + m[3 * i + 1] * v[1] + m[3 * i + 2] * v[2];
}

static void matTvec3(const double *m, const double *v, double *out)
{
    for (int i = 0; i < 3; ++i) out[i] = m[i] * v[0] + m[3 + i] * v[1] + m[6 + i] * v[2];
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.1 Eq.(3): rotation matrix of a quaternion q = (w, x, y, z).        */
void or_rotation(const double *q_in, double *R)
{
    double n = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3]);
    double w = q_in[0] / n, x = q_in[1] / n, y = q_in[2] / n, z = q_in[3] / n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* ------------------------------------------------------------------------ */
/* View-dependent colour (Sec. 5 mentions a view-dependent encoding; reading:
 * real spherical harmonics of degree <= 3).  Written from the textbook
 * definition: Y_l^m = N_l^|m| P_l^|m|(cos theta) * {sqrt2 cos(m phi), 1,
 * sqrt2 sin(|m| phi)} with the Condon-Shortley phase inside P_l^m, theta the
 * polar angle from +z and phi the azimuth from +x towards +y.  Index l*l+l+m. */
static double fact(int k) { double r = 1; for (int i = 2; i <= k; ++i) r *= i; return r; }

static double assoc_legendre(int l, int m, double x) /* P_l^m(x), m >= 0, with (-1)^m phase */
{
    /* Standard recurrences (Abramowitz & Stegun 8.5.3, 8.6.x). */
    double pmm = 1.0;
    if (m > 0) {
        double somx2 = sqrt((1.0 - x) * (1.0 + x));
        double f = 1.0;
        for (int i = 1; i <= m; ++i) { pmm *= -f * somx2; f += 2.0; }
    }
    if (l == m) return pmm;
    double pmmp1 = x * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return pmmp1;
    double pll = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pll = ((2.0 * ll - 1.0) * x * pmmp1 - (ll + m - 1.0) * pmm) / (ll - m);
        pmm = pmmp1;
        pmmp1 = pll;
    }
    return pll;
}

void or_sh_basis(int degree, const double *dir, double *Y)
{
    double r = sqrt(dot3(dir, dir));
    double ct = dir[2] / r;
    if (ct > 1) ct = 1;
    if (ct < -1) ct = -1;
    double phi = atan2(dir[1], dir[0]);
    for (int l = 0; l <= degree; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double N = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * fact(l - am) / fact(l + am));
            double P = assoc_legendre(l, am, ct);
            double v;
            if (m > 0) v = sqrt(2.0) * N * P * cos(m * phi);
            else if (m < 0) v = sqrt(2.0) * N * P * sin(am * phi);
            else v = N * P;
            Y[l * l + l + m] = v;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Per-Gaussian preparation: Sec. 3.1 Eq.(1)-(3), Sec. 3.2 Eq.(6)-(13),
 * Sec. 3.3 camera-inside discard, Sec. 3.4 whole-frustum cull.            */

static void camera_parts(const or_camera *cam, double *RV, double *tV, double *o)
{
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) RV[3 * i + j] = cam->viewmat[4 * i + j];
        tV[i] = cam->viewmat[4 * i + 3];
    }
    /* camera centre o = -R_V^T t_V (rigid view matrix) */
    matTvec3(RV, tV, o);
    o[0] = -o[0]; o[1] = -o[1]; o[2] = -o[2];
}

double or_cone_min_rho2(const or_gauss *g, const or_camera *cam, double x0, double x1, double y0, double y1);

static int finite_all(const double *v, int n)
{
    for (int i = 0; i < n; ++i) if (!isfinite(v[i])) return 0;
    return 1;
}

void or_prepare(const or_scene *sc, const or_camera *cam, const or_settings *st, int64_t i, or_gauss *g)
{
    memset(g, 0, sizeof(*g));
    const int64_t n = sc->n;
    double RV[9], tV[3], o[3];
    camera_parts(cam, RV, tV, o);
    double q[4], ls[3], logit;
    for (int k = 0; k < 3; ++k) {
        g->mu[k] = sc->means[k * n + i];
        ls[k] = sc->log_scales[k * n + i];
    }
    for (int k = 0; k < 4; ++k) q[k] = sc->quats[k * n + i];
    logit = sc->opacity_logits[i];
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!finite_all(g->mu, 3) || !finite_all(ls, 3) || !finite_all(q, 4) || !isfinite(logit) || !(qn > 0)) {
        g->status = OR_INVALID;
        return;
    }
    /* O1: activations (Eq.1-3). */
    for (int k = 0; k < 3; ++k) g->s[k] = exp(ls[k]);
    g->alpha = 1.0 / (1.0 + exp(-logit));
    or_rotation(q, g->R);
    /* O2: view transform. */
    matvec3(RV, g->mu, g->mu_v);
    for (int k = 0; k < 3; ++k) { g->mu_v[k] += tV[k]; g->o[k] = o[k]; }
    /* O3: filter.  v = f/d (Eq.6) with d the view depth of the mean, read as
     * max(z, znear) so that it exists behind the camera; f = fx.  Eq.(13):
     * v' = min(v_train, v).  Filter variance a = k / v'^2 (Sec. 3.1). */
    double dz = g->mu_v[2] > cam->znear ? g->mu_v[2] : cam->znear;
    double v = cam->fx / dz;
    if (sc->v_train) {
        double vt = sc->v_train[i];
        if (vt < v) v = vt;
    }
    double a = st->filter_mode == 1 ? 0.0 : st->filter_k / (v * v);
    g->filter_a = a;
    double s2[3], sh_[3];
    for (int k = 0; k < 3; ++k) {
        s2[k] = g->s[k] * g->s[k];
        sh_[k] = s2[k] + a; /* hat s_k = s_k^2 + k/v'^2 */
        g->s_t[k] = sqrt(sh_[k]);
    }
    /* unit direction from the camera centre to the mean */
    double d[3] = {g->mu[0] - o[0], g->mu[1] - o[1], g->mu[2] - o[2]};
    double dn = sqrt(dot3(d, d));
    for (int k = 0; k < 3; ++k) { d[k] /= dn; g->dir[k] = d[k]; }
    if (st->filter_mode == 1) {
        g->alpha_t = g->alpha;
    } else if (st->filter_mode == 2) {
        /* Eq.(8): volume ratio sqrt(prod s^2 / prod (s^2 + a)). */
        g->alpha_t = g->alpha * sqrt((s2[0] * s2[1] * s2[2]) / (sh_[0] * sh_[1] * sh_[2]));
    } else {
        /* Eq.(12): perpendicular ratio with d' = R^T d. */
        double dp[3];
        matTvec3(g->R, d, dp);
        double num = dp[0] * dp[0] * s2[1] * s2[2] + dp[1] * dp[1] * s2[0] * s2[2] + dp[2] * dp[2] * s2[0] * s2[1];
        double den = dp[0] * dp[0] * sh_[1] * sh_[2] + dp[1] * dp[1] * sh_[0] * sh_[2] + dp[2] * dp[2] * sh_[0] * sh_[1];
        g->alpha_t = g->alpha * sqrt(num / den);
    }
    /* normalised-space maps: g = S~^-1 R^T (x - mu) in world; view dir r_v -> A r_v */
    double RtRVt[9]; /* R^T R_V^T */
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += g->R[3 * k + r] * RV[3 * c + k];
            RtRVt[3 * r + c] = acc;
        }
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) g->A[3 * r + c] = RtRVt[3 * r + c] / g->s_t[r];
    for (int r = 0; r < 3; ++r) /* M = R_V R S~ */
        for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += RV[3 * r + k] * g->R[3 * k + c];
            g->M[3 * r + c] = acc * g->s_t[c];
        }
    {
        double om[3] = {o[0] - g->mu[0], o[1] - g->mu[1], o[2] - g->mu[2]}, t[3];
        matTvec3(g->R, om, t);
        for (int k = 0; k < 3; ++k) g->o_g[k] = t[k] / g->s_t[k];
    }
    /* O6: colour, c = max(0, 0.5 + sum_lm Y_lm(d) c_lm) per channel. */
    {
        double Y[16];
        int nb = (sc->sh_degree + 1) * (sc->sh_degree + 1);
        or_sh_basis(sc->sh_degree, d, Y);
        for (int ch = 0; ch < 3; ++ch) {
            double acc = 0.5;
            for (int b = 0; b < nb; ++b) acc += Y[b] * sc->sh[((int64_t)b * 3 + ch) * n + i];
            g->color[ch] = acc > 0 ? acc : 0;
        }
    }
    /* O4: opacity cull; tau = 2 ln(alpha~ / alpha_min) is the rho^2 level at
     * which alpha~ exp(-rho^2/2) equals alpha_min (reading of tau_rho). */
    if (!(g->alpha_t >= st->alpha_min)) {
        g->status = OR_LOW_OPACITY;
        return;
    }
    g->tau = 2.0 * log(g->alpha_t / st->alpha_min);
    /* O5: camera inside the level-tau ellipsoid -> discard (Sec. 3.3). */
    double og2 = dot3(g->o_g, g->o_g);
    if (fabs(og2 - g->tau) <= st->band_alpha * g->tau) g->ambiguous = 1;
    if (og2 < g->tau) {
        g->status = OR_CAM_INSIDE;
        return;
    }
    /* Whole-frustum cull (Sec. 3.4 last paragraph): same test as a tile, with
     * the image borders as the pyramid. */
    double m = or_cone_min_rho2(g, cam, 0.0, (double)cam->width, 0.0, (double)cam->height);
    if (!(m < g->tau)) {
        g->status = OR_OUTSIDE;
        return;
    }
    g->status = OR_VISIBLE;
}

/* ------------------------------------------------------------------------ */
/* Response of one Gaussian on the line through pixel position (x, y).
 * Sec. 3.1 Eq.(4)-(5): the maximum along the line of G equals exp(-rho^2/2)
 * with rho^2 the squared distance from the origin to the line in normalised
 * Gaussian space.  Line: o_g + t r_g with r_g = A (u, v, 1); the view depth of
 * the point at parameter t is t, because the view direction has z = 1.     */
void or_response(const or_gauss *g, const or_camera *cam, double x, double y, double *rho2, double *zstar)
{
    double rv[3] = {(x - cam->cx) / cam->fx, (y - cam->cy) / cam->fy, 1.0};
    double rg[3];
    matvec3(g->A, rv, rg);
    double rr = dot3(rg, rg);
    double orr = dot3(g->o_g, rg);
    double t = -orr / rr;
    double p[3] = {g->o_g[0] + t * rg[0], g->o_g[1] + t * rg[1], g->o_g[2] + t * rg[2]};
    *rho2 = dot3(p, p);
    *zstar = t;
}

/* p satisfies every half-space except skip1/skip2, up to a relative 1e-12. */
static int feasible(double ng[4][3], const double *dg, const double *p, int skip1, int skip2)
{
    for (int j = 0; j < 4; ++j) {
        if (j == skip1 || j == skip2) continue;
        double s = dot3(ng[j], p) + dg[j];
        double scale = sqrt(dot3(ng[j], ng[j])) * sqrt(dot3(p, p)) + fabs(dg[j]) + 1e-300;
        if (s < -1e-12 * scale) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Exact minimum of rho^2 over the pyramid spanned by the camera centre and the
 * screen rectangle [x0,x1] x [y0,y1] (Sec. 3.4, Eq.(18)).  The pyramid is the
 * intersection of four half-spaces through the camera centre; rho^2 is a
 * strictly convex quadratic, so its minimum over the pyramid is attained at
 * the feasible stationary point of some active set.  Every active set is
 * enumerated: none (the mean itself), one plane, two planes (a line through
 * the apex), three or more (the apex).                                       */
double or_cone_min_rho2(const or_gauss *g, const or_camera *cam, double x0, double x1, double y0, double y1)
{
    /* view-space half-spaces n . X >= 0 */
    double nv[4][3] = {
        {cam->fx, 0.0, cam->cx - x0},   /* x >= x0 */
        {-cam->fx, 0.0, x1 - cam->cx},  /* x <= x1 */
        {0.0, cam->fy, cam->cy - y0},   /* y >= y0 */
        {0.0, -cam->fy, y1 - cam->cy},  /* y <= y1 */
    };
    /* transform to normalised Gaussian space: X = M p + mu_v,
     * n.X = (M^T n).p + n.mu_v (Eq.(5): planes move with T'^T). */
    double ng[4][3], dg[4];
    for (int k = 0; k < 4; ++k) {
        double nn = sqrt(dot3(nv[k], nv[k]));
        double nk[3] = {nv[k][0] / nn, nv[k][1] / nn, nv[k][2] / nn};
        matTvec3(g->M, nk, ng[k]);
        dg[k] = dot3(nk, g->mu_v);
    }
    /* empty active set: the mean (p = 0) */
    {
        int inside = 1;
        for (int k = 0; k < 4; ++k) if (dg[k] < 0) inside = 0;
        if (inside) return 0.0;
    }
    double best = INFINITY;
    /* apex: the camera centre, always in the closed pyramid */
    best = dot3(g->o_g, g->o_g);
    /* one active plane */
    for (int k = 0; k < 4; ++k) {
        double nn = dot3(ng[k], ng[k]);
        double p[3] = {-dg[k] * ng[k][0] / nn, -dg[k] * ng[k][1] / nn, -dg[k] * ng[k][2] / nn};
        if (feasible(ng, dg, p, k, k)) {
            double v = dot3(p, p);
            if (v < best) best = v;
        }
    }
    /* two active planes: their intersection line passes through the apex */
    for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b) {
            double dir[3];
            cross3(ng[a], ng[b], dir);
            double dd = dot3(dir, dir);
            if (!(dd > 0)) continue;
            double t = -dot3(g->o_g, dir) / dd;
            double p[3] = {g->o_g[0] + t * dir[0], g->o_g[1] + t * dir[1], g->o_g[2] + t * dir[2]};
            if (feasible(ng, dg, p, a, b)) {
                double v = dot3(p, p);
                if (v < best) best = v;
            }
        }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Conservative candidate tiles: sphere of radius sqrt(tau) * max s~ around the
 * mean (contains the level-tau ellipsoid).  Tile column tx is a candidate if
 * the sphere reaches both half-spaces of the column's side planes; same for
 * rows; and the sphere must reach depth znear.                              */
static int sphere_rect(const or_gauss *g, const or_camera *cam, int tiles_x, int tiles_y, int *rect)
{
    double smax = g->s_t[0];
    if (g->s_t[1] > smax) smax = g->s_t[1];
    if (g->s_t[2] > smax) smax = g->s_t[2];
    double rad = sqrt(g->tau) * smax * (1.0 + 1e-9) + 1e-12;
    if (g->mu_v[2] + rad < cam->znear) return 0;
    int lo = tiles_x, hi = -1;
    for (int tx = 0; tx < tiles_x; ++tx) {
        double x0 = tx * OR_TILE, x1 = x0 + OR_TILE;
        double nl[3] = {cam->fx, 0, cam->cx - x0}, nr[3] = {-cam->fx, 0, x1 - cam->cx};
        double dl = dot3(nl, g->mu_v) / sqrt(dot3(nl, nl));
        double dr = dot3(nr, g->mu_v) / sqrt(dot3(nr, nr));
        if (dl >= -rad && dr >= -rad) {
            if (tx < lo) lo = tx;
            hi = tx;
        }
    }
    if (hi < 0) return 0;
    int lo_y = tiles_y, hi_y = -1;
    for (int ty = 0; ty < tiles_y; ++ty) {
        double y0 = ty * OR_TILE, y1 = y0 + OR_TILE;
        double nt[3] = {0, cam->fy, cam->cy - y0}, nb[3] = {0, -cam->fy, y1 - cam->cy};
        double dt = dot3(nt, g->mu_v) / sqrt(dot3(nt, nt));
        double db = dot3(nb, g->mu_v) / sqrt(dot3(nb, nb));
        if (dt >= -rad && db >= -rad) {
            if (ty < lo_y) lo_y = ty;
            hi_y = ty;
        }
    }
    if (hi_y < 0) return 0;
    rect[0] = lo; rect[1] = hi + 1; rect[2] = lo_y; rect[3] = hi_y + 1;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Rendering. */

typedef struct {
    double dtile;
    int64_t id;
    double z, a;
    const double *c;
    double tat; /* transmittance just before this entry was blended; -1 if never blended */
    double r2;  /* rho^2 on the pixel line */
    int clamped;/* alpha hit alpha_max */
} or_contrib;

static int cmp_tile_order(const void *pa, const void *pb)
{
    const or_contrib *a = (const or_contrib *)pa, *b = (const or_contrib *)pb;
    if (a->dtile < b->dtile) return -1;
    if (a->dtile > b->dtile) return 1;
    return (a->id > b->id) - (a->id < b->id);
}

typedef struct {
    double T, C[3];
    int done;
    int flag;
    int64_t nblend;
    double errT; /* relative error bound of a float32 T after the entries blended so far */
    int flip_at; /* termination test (counted from 0) taken the other way; -1: none */
    int ncall;   /* termination tests so far */
    int nterm;   /* termination tests within their band (flag 4), recorded in term_at */
    int term_at[4];
} or_pixel_state;

static or_pixel_state pixel_state_init(int flip_at)
{
    or_pixel_state ps;
    memset(&ps, 0, sizeof ps);
    ps.T = 1.0;
    ps.flip_at = flip_at;
    return ps;
}

static double max3(const double *c)
{
    double m = c[0] > c[1] ? c[0] : c[1];
    return c[2] > m ? c[2] : m;
}

/* O12: front-to-back blending with early termination: stop, without blending
 * it, at the first entry that would take T below t_min (3DGS lineage).
 *
 * Flag 4 marks a termination test that a float32 implementation may take the
 * other way.  Its band is an error bound of a float32 T: every blended entry
 * multiplies T by 1 - alpha, where alpha has a relative error of at most
 * band_alpha (the band of the alpha test; zero when alpha is clamped at
 * alpha_max, a value both sides hit exactly), which gives 1 - alpha a
 * relative error of band_alpha * alpha / (1 - alpha), plus two roundings
 * (the subtraction and the product) of 2^-24 each.  These add up over the
 * entries blended; band_T is a floor. */
static void blend_one(or_pixel_state *ps, const or_settings *st, or_contrib *e)
{
    if (ps->done) return;
    double Tn = ps->T * (1.0 - e->a);
    double cm = max3(e->c);
    double errTn = ps->errT + (e->clamped ? 0.0 : st->band_alpha * e->a / (1.0 - e->a)) + 2.0 * 0x1p-24;
    double band = errTn > st->band_T ? errTn : st->band_T;
    if (fabs(Tn - st->t_min) <= band * st->t_min && ps->T * e->a * (cm > 1 ? cm : 1) > 5e-5) {
        ps->flag |= 4;
        if (ps->nterm < 4) ps->term_at[ps->nterm++] = ps->ncall;
    }
    int stop = Tn < st->t_min;
    if (ps->ncall == ps->flip_at) stop = !stop; /* an alternative outcome of a flagged test */
    ps->ncall++;
    if (stop) {
        ps->done = 1;
        return;
    }
    e->tat = ps->T;
    for (int k = 0; k < 3; ++k) ps->C[k] += ps->T * e->a * e->c[k];
    ps->T = Tn;
    ps->errT = errTn;
    ps->nblend++;
}

/* O11: per-ray window of capacity K keyed by (z*, id): each contributor is
 * inserted; when the window holds more than K entries its minimum is popped
 * and blended; at the end of the list the rest is popped in ascending order.
 * K = 0 blends in list order. */
static int win_less(const or_contrib *a, const or_contrib *b)
{
    if (a->z < b->z) return 1;
    if (a->z > b->z) return 0;
    return a->id < b->id;
}

static void window_blend(or_contrib *seq, int64_t ns, int K, or_pixel_state *ps, const or_settings *st, int64_t *win)
{
    if (K <= 0) {
        for (int64_t i = 0; i < ns && !ps->done; ++i) blend_one(ps, st, &seq[i]);
        return;
    }
    int nw = 0;
    for (int64_t i = 0; i < ns && !ps->done; ++i) {
        win[nw++] = i;
        if (nw > K) {
            int mi = 0;
            for (int j = 1; j < nw; ++j) if (win_less(&seq[win[j]], &seq[win[mi]])) mi = j;
            int64_t e = win[mi];
            win[mi] = win[nw - 1];
            nw--;
            blend_one(ps, st, &seq[e]);
        }
    }
    while (nw > 0 && !ps->done) {
        int mi = 0;
        for (int j = 1; j < nw; ++j) if (win_less(&seq[win[j]], &seq[win[mi]])) mi = j;
        int64_t e = win[mi];
        win[mi] = win[nw - 1];
        nw--;
        blend_one(ps, st, &seq[e]);
    }
}

/* Largest change of the pixel if the blend order of entries i and j were
 * swapped: T_before * a_i * a_j * |c_i - c_j| (both blended), or T_before *
 * max(a) * max(c) when only one of them was blended (termination between). */
static double swap_impact(const or_contrib *p, const or_contrib *q)
{
    double tp = p->tat, tq = q->tat;
    if (tp < 0 && tq < 0) return 0.0;
    if (tp >= 0 && tq >= 0) {
        double t = tp > tq ? tp : tq, d = 0;
        for (int k = 0; k < 3; ++k) {
            double x = fabs(p->c[k] - q->c[k]);
            if (x > d) d = x;
        }
        return t * p->a * q->a * d;
    }
    double t = tp >= 0 ? tp : tq;
    double am = p->a > q->a ? p->a : q->a;
    double cm = max3(p->c) > max3(q->c) ? max3(p->c) : max3(q->c);
    return t * am * cm;
}

/* indices of seq ordered by the window key (insertion sort; lists are short) */
static void sort_idx_by_key(int64_t *idx, int64_t n, const or_contrib *seq)
{
    for (int64_t i = 1; i < n; ++i) {
        int64_t v = idx[i], j = i - 1;
        while (j >= 0 && win_less(&seq[v], &seq[idx[j]])) {
            idx[j + 1] = idx[j];
            --j;
        }
        idx[j + 1] = v;
    }
}

typedef struct {
    int64_t n_visible, n_candidates_total;
    int64_t n_contrib_total, n_blended_total;
    int64_t n_flagged;
} or_stats;

/*
 * Render.  out_rgb [3][H][W], out_T [H][W], out_flags [H][W] (bit 0: a
 * contribution test within band, bit 1: depth near-tie, bit 2: termination
 * within band, bit 3: ambiguous camera-inside Gaussian touches the pixel),
 * out_ncontrib [H][W] (may be NULL).  tile_sel [tiles] selects the tiles to
 * render (NULL = all); unselected pixels are left untouched.
 */
/* Reverse pass of one pixel (plain reverse-mode recursion over the blended
 * entries, in the order they were blended: decreasing T).  Accumulates into
 * per-Gaussian intermediate gradients gi[16 * id]: o_g (3), A (9), alpha~ (1),
 * colour (3). */
#define OR_GI 16
static void pixel_reverse(or_contrib *seq, int64_t ns, int64_t *idx, const or_gauss *gs, const or_camera *cam,
                          const double *gC, double x, double y, double *gi)
{
    int64_t m = 0;
    for (int64_t j = 0; j < ns; ++j)
        if (seq[j].tat >= 0) idx[m++] = j;
    for (int64_t i = 1; i < m; ++i) { /* sort by decreasing T (= blend order) */
        int64_t v = idx[i], j = i - 1;
        while (j >= 0 && seq[idx[j]].tat < seq[v].tat) { idx[j + 1] = idx[j]; --j; }
        idx[j + 1] = v;
    }
    double gT = cam->bg[0] * gC[0] + cam->bg[1] * gC[1] + cam->bg[2] * gC[2];
    double rv[3] = {(x - cam->cx) / cam->fx, (y - cam->cy) / cam->fy, 1.0};
    for (int64_t k = m - 1; k >= 0; --k) {
        const or_contrib *e = &seq[idx[k]];
        const or_gauss *g = &gs[e->id];
        double Tk = e->tat, a = e->a;
        double cg = e->c[0] * gC[0] + e->c[1] * gC[1] + e->c[2] * gC[2];
        double ga = Tk * cg - Tk * gT;
        double *G = gi + OR_GI * e->id;
        for (int c = 0; c < 3; ++c) {
#pragma omp atomic
            G[13 + c] += Tk * a * gC[c];
        }
        gT = a * cg + (1.0 - a) * gT;
        if (e->clamped) continue;
        double ex = exp(-0.5 * e->r2);
#pragma omp atomic
        G[12] += ga * ex;
        double gr2 = -0.5 * ga * a;
        double r[3];
        matvec3(g->A, rv, r);
        double rr = dot3(r, r), orr = dot3(g->o_g, r);
        for (int c = 0; c < 3; ++c) {
            double dro = 2.0 * g->o_g[c] - 2.0 * orr / rr * r[c];
            double drr = -2.0 * orr / rr * g->o_g[c] + 2.0 * orr * orr / (rr * rr) * r[c];
#pragma omp atomic
            G[c] += gr2 * dro;
            for (int j = 0; j < 3; ++j) {
#pragma omp atomic
                G[3 + 3 * c + j] += gr2 * drr * rv[j];
            }
        }
    }
}

/* Alternative outcomes of a flagged pixel.  Each flagged decision (a
 * membership test within its band, an ambiguous camera-inside Gaussian, a
 * near-tie in either ordering key, a termination test within its band) is
 * taken the other way, one at a time, and the pixel blended again; an FP32
 * implementation may legitimately produce any of these results. */
#define OR_MAX_ALT 16
typedef struct {
    or_contrib e; /* the entry as it would contribute */
    int in_seq;   /* it is in the sequence (the alternative removes it) */
} or_near;
typedef struct {
    int kind;     /* 0: tile-order neighbours i, j swapped; 1: window-order q moved in front of p */
    int64_t i, j;
} or_tie;

static void blend_alternative(const or_contrib *s2, int64_t ns2, or_contrib *buf, int K, const or_settings *st,
                              const or_camera *cam, int flip_at, int64_t *win, double *out)
{
    memcpy(buf, s2, sizeof(or_contrib) * (size_t)ns2);
    or_pixel_state ps = pixel_state_init(flip_at);
    window_blend(buf, ns2, K, &ps, st, win);
    for (int k = 0; k < 3; ++k) out[k] = ps.C[k] + ps.T * cam->bg[k];
    out[3] = ps.T;
}

static int pixel_alternatives(const or_contrib *seq, int64_t ns, const or_near *nr, int nnear, const or_tie *ties,
                              int nties, const or_pixel_state *ps, int K, const or_settings *st, const or_camera *cam,
                              or_contrib *s2, or_contrib *buf, int64_t *win, double *out)
{
    int na = 0;
    for (int q = 0; q < nnear && na < OR_MAX_ALT; ++q) {
        int64_t n2 = 0;
        for (int64_t j = 0; j < ns; ++j)
            if (!(nr[q].in_seq && seq[j].id == nr[q].e.id)) s2[n2++] = seq[j];
        if (!nr[q].in_seq) {
            s2[n2++] = nr[q].e;
            qsort(s2, n2, sizeof(or_contrib), cmp_tile_order);
        }
        blend_alternative(s2, n2, buf, K, st, cam, -1, win, out + 4 * na++);
    }
    for (int q = 0; q < nties && na < OR_MAX_ALT; ++q) {
        memcpy(s2, seq, sizeof(or_contrib) * (size_t)ns);
        if (ties[q].kind == 0) {
            or_contrib t = s2[ties[q].i];
            s2[ties[q].i] = s2[ties[q].j];
            s2[ties[q].j] = t;
        } else {
            s2[ties[q].j].z = nextafter(s2[ties[q].i].z, -INFINITY);
        }
        blend_alternative(s2, ns, buf, K, st, cam, -1, win, out + 4 * na++);
    }
    for (int q = 0; q < ps->nterm && na < OR_MAX_ALT; ++q)
        blend_alternative(seq, ns, buf, K, st, cam, ps->term_at[q], win, out + 4 * na++);
    return na;
}

static int render_impl(const or_scene *sc, const or_camera *cam, const or_settings *st, const uint8_t *tile_sel,
                       double *out_rgb, double *out_T, uint8_t *out_flags, int32_t *out_ncontrib, or_stats *stats,
                       const double *dL_drgb, double *gi, const int32_t *alt_slot, double *alt_out, int32_t *alt_n)
{
    const int64_t n = sc->n;
    const int W = cam->width, H = cam->height;
    const int tiles_x = (W + OR_TILE - 1) / OR_TILE, tiles_y = (H + OR_TILE - 1) / OR_TILE;
    const int ntiles = tiles_x * tiles_y;
    or_gauss *gs = (or_gauss *)malloc(sizeof(or_gauss) * (n > 0 ? n : 1));
    int *rects = (int *)malloc(sizeof(int) * 4 * (n > 0 ? n : 1));
    unsigned char *use = (unsigned char *)calloc(n > 0 ? n : 1, 1);
    if (!gs || !rects || !use) return 1;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        or_prepare(sc, cam, st, i, &gs[i]);
        int cand = gs[i].status == OR_VISIBLE;
        if (gs[i].status == OR_CAM_INSIDE && gs[i].ambiguous) {
            /* would be visible if the FP32 decision went the other way */
            cand = 1;
        }
        if (cand && sphere_rect(&gs[i], cam, tiles_x, tiles_y, &rects[4 * i])) use[i] = cand;
    }
    /* bucket candidates per tile */
    int64_t *cnt = (int64_t *)calloc(ntiles + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        if (!use[i]) continue;
        for (int ty = rects[4 * i + 2]; ty < rects[4 * i + 3]; ++ty)
            for (int tx = rects[4 * i]; tx < rects[4 * i + 1]; ++tx) cnt[ty * tiles_x + tx + 1]++;
    }
    for (int t = 0; t < ntiles; ++t) cnt[t + 1] += cnt[t];
    int64_t total = cnt[ntiles];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (ntiles + 1));
    memcpy(fill, cnt, sizeof(int64_t) * (ntiles + 1));
    int64_t *lists = (int64_t *)malloc(sizeof(int64_t) * (total > 0 ? total : 1));
    for (int64_t i = 0; i < n; ++i) {
        if (!use[i]) continue;
        for (int ty = rects[4 * i + 2]; ty < rects[4 * i + 3]; ++ty)
            for (int tx = rects[4 * i]; tx < rects[4 * i + 1]; ++tx) lists[fill[ty * tiles_x + tx]++] = i;
    }
    int64_t nvis = 0;
    for (int64_t i = 0; i < n; ++i) nvis += gs[i].status == OR_VISIBLE;
    int64_t tot_contrib = 0, tot_blend = 0, tot_flag = 0;
    const int K = st->ray_window;

#pragma omp parallel reduction(+ : tot_contrib, tot_blend, tot_flag)
    {
        or_contrib *seq = NULL, *s2 = NULL, *s3 = NULL;
        or_near nr[OR_MAX_ALT];
        or_tie ties[OR_MAX_ALT];
        int64_t *win = (int64_t *)malloc(sizeof(int64_t) * (K + 2));
        int64_t *ridx = NULL;
        double *dt = NULL;
        int64_t *zi = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 1)
        for (int t = 0; t < ntiles; ++t) {
            if (tile_sel && !tile_sel[t]) continue;
            int tx = t % tiles_x, ty = t / tiles_x;
            int64_t b = cnt[t], e = cnt[t + 1], m = e - b;
            if (m > cap) {
                cap = m;
                seq = (or_contrib *)realloc(seq, sizeof(or_contrib) * cap);
                if (alt_slot) {
                    s2 = (or_contrib *)realloc(s2, sizeof(or_contrib) * (cap + 1));
                    s3 = (or_contrib *)realloc(s3, sizeof(or_contrib) * (cap + 1));
                }
                dt = (double *)realloc(dt, sizeof(double) * 4 * cap);
                zi = (int64_t *)realloc(zi, sizeof(int64_t) * cap);
                ridx = (int64_t *)realloc(ridx, sizeof(int64_t) * cap);
            }
            /* O9: tile depth = depth of maximum response on the tile-centre
             * line; with the sub-tile level, one depth per 8x8 sub-tile on
             * the line through its centre (dt[q * m + j], q = 2 qy + qx) */
            for (int q = 0; q < (st->subtile_sort ? 4 : 1); ++q) {
                const double cx = st->subtile_sort ? tx * OR_TILE + (q & 1) * 8 + 4.0 : tx * OR_TILE + 0.5 * OR_TILE;
                const double cy = st->subtile_sort ? ty * OR_TILE + (q >> 1) * 8 + 4.0 : ty * OR_TILE + 0.5 * OR_TILE;
                for (int64_t j = 0; j < m; ++j) {
                    double r2, z;
                    or_response(&gs[lists[b + j]], cam, cx, cy, &r2, &z);
                    dt[q * m + j] = z;
                }
            }
            for (int py = ty * OR_TILE; py < ty * OR_TILE + OR_TILE && py < H; ++py)
                for (int px = tx * OR_TILE; px < tx * OR_TILE + OR_TILE && px < W; ++px) {
                    or_pixel_state ps = pixel_state_init(-1);
                    int nnear = 0, nties = 0;
                    /* this pixel's row of ordering depths: its sub-tile's, or the tile's */
                    const double *dq = st->subtile_sort
                                           ? dt + (int64_t)(2 * ((py - ty * OR_TILE) >= 8) + ((px - tx * OR_TILE) >= 8)) * m
                                           : dt;
                    int64_t ns = 0;
                    double x = px + 0.5, y = py + 0.5; /* pixel centre */
                    for (int64_t j = 0; j < m; ++j) {
                        const or_gauss *g = &gs[lists[b + j]];
                        double r2, z;
                        or_response(g, cam, x, y, &r2, &z);
                        double a = g->alpha_t * exp(-0.5 * r2);
                        if (a > st->alpha_max) a = st->alpha_max;
                        int near_a = fabs(a - st->alpha_min) <= st->band_alpha * st->alpha_min;
                        int near_z = fabs(z - cam->znear) <= st->band_z * fabs(cam->znear);
                        int contrib = a >= st->alpha_min && z >= cam->znear;
                        int near_member = 0;
                        if ((near_a && z >= cam->znear * (1 - st->band_z)) ||
                            (near_z && a >= st->alpha_min * (1 - st->band_alpha))) {
                            ps.flag |= 1;
                            near_member = 1;
                        }
                        if (g->status != OR_VISIBLE) {
                            /* ambiguous camera-inside Gaussian */
                            if (a >= st->alpha_min * (1 - st->band_alpha) && z >= cam->znear * (1 - st->band_z)) {
                                ps.flag |= 8;
                                near_member = 1;
                            }
                        }
                        if (near_member && alt_slot && nnear < OR_MAX_ALT) {
                            or_contrib *q = &nr[nnear].e;
                            q->dtile = dq[j];
                            q->id = lists[b + j];
                            q->z = z;
                            q->a = a;
                            q->c = g->color;
                            q->tat = -1.0;
                            q->r2 = r2;
                            q->clamped = g->alpha_t * exp(-0.5 * r2) > st->alpha_max;
                            nr[nnear].in_seq = contrib && g->status == OR_VISIBLE;
                            nnear++;
                        }
                        if (g->status != OR_VISIBLE) continue;
                        if (contrib) {
                            seq[ns].dtile = dq[j];
                            seq[ns].id = lists[b + j];
                            seq[ns].z = z;
                            seq[ns].a = a;
                            seq[ns].c = g->color;
                            seq[ns].tat = -1.0;
                            seq[ns].r2 = r2;
                            seq[ns].clamped = g->alpha_t * exp(-0.5 * r2) > st->alpha_max;
                            ns++;
                        }
                    }
                    /* O10: order by (tile depth, id), or (sub-tile depth, id) */
                    qsort(seq, ns, sizeof(or_contrib), cmp_tile_order);
                    window_blend(seq, ns, K, &ps, st, win);
                    /* Near-ties in either ordering key whose swap would move the
                     * pixel by more than three quarters of the image tolerance
                     * (1.5e-4 of 2e-4). */
                    if (ns > 1) {
                        const double imp = 1.5e-4;
                        if (K == 0 || ns > K) {
                            for (int64_t j = 1; j < ns; ++j) {
                                double d0 = seq[j - 1].dtile, d1 = seq[j].dtile;
                                double sc = fabs(d0) > fabs(d1) ? fabs(d0) : fabs(d1);
                                if (fabs(d1 - d0) <= st->band_tie * sc && swap_impact(&seq[j - 1], &seq[j]) > imp) {
                                    ps.flag |= 2;
                                    if (nties < OR_MAX_ALT) ties[nties++] = (or_tie){0, j - 1, j};
                                }
                            }
                        }
                        if (K > 0) {
                            for (int64_t j = 0; j < ns; ++j) zi[j] = j;
                            sort_idx_by_key(zi, ns, seq);
                            for (int64_t j = 1; j < ns; ++j) {
                                const or_contrib *p0 = &seq[zi[j - 1]], *p1 = &seq[zi[j]];
                                double sc = fabs(p0->z) > fabs(p1->z) ? fabs(p0->z) : fabs(p1->z);
                                if (fabs(p1->z - p0->z) <= st->band_tie * sc && swap_impact(p0, p1) > imp) {
                                    ps.flag |= 2;
                                    if (nties < OR_MAX_ALT) ties[nties++] = (or_tie){1, zi[j - 1], zi[j]};
                                }
                            }
                        }
                    }
                    int64_t pix = (int64_t)py * W + px;
                    if (alt_slot && alt_slot[pix] >= 0) {
                        int32_t sl = alt_slot[pix];
                        alt_n[sl] = pixel_alternatives(seq, ns, nr, nnear, ties, nties, &ps, K, st, cam, s2, s3, win,
                                                       alt_out + (int64_t)sl * OR_MAX_ALT * 4);
                    }
                    if (dL_drgb) {
                        double gC[3] = {dL_drgb[pix], dL_drgb[(int64_t)H * W + pix], dL_drgb[2 * (int64_t)H * W + pix]};
                        pixel_reverse(seq, ns, ridx, gs, cam, gC, x, y, gi);
                    }
                    for (int k = 0; k < 3; ++k) out_rgb[(int64_t)k * H * W + pix] = ps.C[k] + ps.T * cam->bg[k];
                    out_T[pix] = ps.T;
                    if (out_flags) out_flags[pix] = (uint8_t)ps.flag;
                    if (out_ncontrib) out_ncontrib[pix] = (int32_t)ns;
                    tot_contrib += ns;
                    tot_blend += ps.nblend;
                    tot_flag += ps.flag != 0;
                }
        }
        free(seq);
        free(s2);
        free(s3);
        free(win);
        free(dt);
        free(zi);
        free(ridx);
    }
    if (stats) {
        stats->n_visible = nvis;
        stats->n_candidates_total = total;
        stats->n_contrib_total = tot_contrib;
        stats->n_blended_total = tot_blend;
        stats->n_flagged = tot_flag;
    }
    free(gs);
    free(rects);
    free(use);
    free(cnt);
    free(fill);
    free(lists);
    return 0;
}

int or_render(const or_scene *sc, const or_camera *cam, const or_settings *st, const uint8_t *tile_sel,
              double *out_rgb, double *out_T, uint8_t *out_flags, int32_t *out_ncontrib, or_stats *stats)
{
    return render_impl(sc, cam, st, tile_sel, out_rgb, out_T, out_flags, out_ncontrib, stats, NULL, NULL, NULL, NULL,
                       NULL);
}

/* Alternative outcomes (see pixel_alternatives) of the pixels with
 * alt_slot[pix] >= 0 ([H][W], -1 elsewhere): alt_out [slots][OR_MAX_ALT][4]
 * (rgb + T * bg, T) and their number alt_n [slots].  Only tiles in tile_sel
 * (NULL = all) are rendered. */
int or_render_alternatives(const or_scene *sc, const or_camera *cam, const or_settings *st, const uint8_t *tile_sel,
                           const int32_t *alt_slot, double *alt_out, int32_t *alt_n)
{
    int64_t np = (int64_t)cam->width * cam->height;
    double *rgb = (double *)malloc(sizeof(double) * 3 * (np > 0 ? np : 1));
    double *T = (double *)malloc(sizeof(double) * (np > 0 ? np : 1));
    int rc = render_impl(sc, cam, st, tile_sel, rgb, T, NULL, NULL, NULL, NULL, NULL, alt_slot, alt_out, alt_n);
    free(rgb);
    free(T);
    return rc;
}

int or_max_alternatives(void) { return OR_MAX_ALT; }

/* ------------------------------------------------------------------------ */
/* Per-Gaussian outputs for stage checks: status, alpha~, tau, filtered scales,
 * colour, view mean, |o_g|^2.  out arrays are [n] (or [3][n]).              */
int or_preprocess(const or_scene *sc, const or_camera *cam, const or_settings *st, int32_t *status, int32_t *ambiguous,
                  double *alpha_t, double *tau, double *s_t /*[3][n]*/, double *color /*[3][n]*/, double *mu_v /*[3][n]*/,
                  double *og2)
{
    const int64_t n = sc->n;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        or_gauss g;
        or_prepare(sc, cam, st, i, &g);
        status[i] = g.status;
        if (ambiguous) ambiguous[i] = g.ambiguous;
        alpha_t[i] = g.alpha_t;
        tau[i] = g.tau;
        for (int k = 0; k < 3; ++k) {
            s_t[k * n + i] = g.s_t[k];
            color[k * n + i] = g.color[k];
            mu_v[k * n + i] = g.mu_v[k];
        }
        og2[i] = dot3(g.o_g, g.o_g);
    }
    return 0;
}

/* rho^2 and depth of maximum response for query (gaussian, x, y) triples,
 * ignoring the Gaussian's cull status (status is reported separately). */
int or_eval_points(const or_scene *sc, const or_camera *cam, const or_settings *st, int64_t nq, const int64_t *ids,
                   const double *xs, const double *ys, double *rho2, double *zstar, double *alpha)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t q = 0; q < nq; ++q) {
        or_gauss g;
        or_prepare(sc, cam, st, ids[q], &g);
        if (g.status == OR_INVALID) {
            rho2[q] = NAN; zstar[q] = NAN; alpha[q] = NAN;
            continue;
        }
        double r2, z;
        or_response(&g, cam, xs[q], ys[q], &r2, &z);
        rho2[q] = r2;
        zstar[q] = z;
        double a = g.alpha_t * exp(-0.5 * r2);
        alpha[q] = a > st->alpha_max ? st->alpha_max : a;
    }
    return 0;
}

/* Exact cone minimum for query (gaussian, rectangle) pairs; returns also tau. */
int or_cone_min_query(const or_scene *sc, const or_camera *cam, const or_settings *st, int64_t nq, const int64_t *ids,
                      const double *rects /*[nq][4] x0 x1 y0 y1*/, double *out_min, double *out_tau)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t q = 0; q < nq; ++q) {
        or_gauss g;
        or_prepare(sc, cam, st, ids[q], &g);
        out_tau[q] = g.tau;
        if (g.status == OR_INVALID || g.status == OR_LOW_OPACITY) {
            out_min[q] = NAN;
            continue;
        }
        out_min[q] = or_cone_min_rho2(&g, cam, rects[4 * q], rects[4 * q + 1], rects[4 * q + 2], rects[4 * q + 3]);
    }
    return 0;
}

/*
 * Pair classification for one tile (O13): for each queried Gaussian,
 *   need    = some pixel of the tile (inside the image) has alpha >= alpha_min
 *             and z* >= znear,
 *   near    = some pixel decision lies within the bands (exempt),
 *   allowed = exact pyramid minimum of rho^2 < tau + (1e-3 tau + 1e-4).
 * out_class: 0 not allowed, 1 allowed not needed, 2 needed, 3 exempt.
 * Gaussians whose status is not VISIBLE get class 0 (or 3 if ambiguous).
 */
int or_classify_pairs(const or_scene *sc, const or_camera *cam, const or_settings *st, int32_t tile, int64_t nq,
                      const int64_t *ids, int32_t *out_class)
{
    const int W = cam->width, H = cam->height;
    const int tiles_x = (W + OR_TILE - 1) / OR_TILE;
    int tx = tile % tiles_x, ty = tile / tiles_x;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < nq; ++q) {
        or_gauss g;
        or_prepare(sc, cam, st, ids[q], &g);
        if (g.status != OR_VISIBLE) {
            out_class[q] = (g.status == OR_CAM_INSIDE && g.ambiguous) ? 3 : 0;
            continue;
        }
        int need = 0, near = 0;
        for (int py = ty * OR_TILE; py < ty * OR_TILE + OR_TILE && py < H; ++py)
            for (int px = tx * OR_TILE; px < tx * OR_TILE + OR_TILE && px < W; ++px) {
                double r2, z;
                or_response(&g, cam, px + 0.5, py + 0.5, &r2, &z);
                double a = g.alpha_t * exp(-0.5 * r2);
                if (a > st->alpha_max) a = st->alpha_max;
                if (a >= st->alpha_min && z >= cam->znear) need = 1;
                if (fabs(a - st->alpha_min) <= st->band_alpha * st->alpha_min && z >= cam->znear * (1 - st->band_z)) near = 1;
                if (fabs(z - cam->znear) <= st->band_z * fabs(cam->znear) && a >= st->alpha_min * (1 - st->band_alpha)) near = 1;
            }
        double m = or_cone_min_rho2(&g, cam, tx * OR_TILE, tx * OR_TILE + OR_TILE, ty * OR_TILE, ty * OR_TILE + OR_TILE);
        int allowed = m < g.tau + (1e-3 * g.tau + 1e-4);
        if (need) out_class[q] = 2;
        else if (near) out_class[q] = 3;
        else out_class[q] = allowed ? 1 : 0;
    }
    return 0;
}

/*
 * Reference screen bounds (O14): the x and y screen range covered by the
 * level-tau ellipsoid's surface points with view depth > 0, from a dense
 * (nt x np) sampling of the surface.  out[4] = xmin, xmax, ymin, ymax (may be
 * +-inf when the surface reaches depth 0 with a nonzero lateral offset).
 * Returns the Gaussian's status.
 */
int or_sampled_bounds(const or_scene *sc, const or_camera *cam, const or_settings *st, int64_t i, int nt, int np,
                      double *out)
{
    or_gauss g;
    or_prepare(sc, cam, st, i, &g);
    out[0] = INFINITY; out[1] = -INFINITY; out[2] = INFINITY; out[3] = -INFINITY;
    if (g.status == OR_INVALID || g.status == OR_LOW_OPACITY) return g.status;
    double r = sqrt(g.tau);
    for (int a = 0; a <= nt; ++a) {
        double th = M_PI * a / nt;
        for (int b = 0; b < np; ++b) {
            double ph = 2 * M_PI * b / np;
            double p[3] = {r * sin(th) * cos(ph), r * sin(th) * sin(ph), r * cos(th)}, X[3];
            matvec3(g.M, p, X);
            for (int k = 0; k < 3; ++k) X[k] += g.mu_v[k];
            if (!(X[2] > 0)) continue;
            double xs = cam->cx + cam->fx * X[0] / X[2];
            double ys = cam->cy + cam->fy * X[1] / X[2];
            if (xs < out[0]) out[0] = xs;
            if (xs > out[1]) out[1] = xs;
            if (ys < out[2]) out[2] = ys;
            if (ys > out[3]) out[3] = ys;
        }
    }
    return g.status;
}

/* or_sampled_bounds for each of n_ids Gaussians: out[4 * q ..] and
 * status[q] for ids[q] (in parallel over the queries). */
int or_sampled_bounds_many(const or_scene *sc, const or_camera *cam, const or_settings *st, int64_t n_ids,
                           const int64_t *ids, int nt, int np, double *out, int32_t *status)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < n_ids; ++q) status[q] = or_sampled_bounds(sc, cam, st, ids[q], nt, np, out + 4 * q);
    return 0;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Gradients (reverse mode with every discrete decision held fixed).
 *
 * The pixel part is the plain reverse recursion of the blend (pixel_reverse),
 * giving per-Gaussian gradients of o_g, A, alpha~ and the colour.  The
 * per-Gaussian chain from the parameters to those quantities is
 * differentiated by the complex step: the same formulas as or_prepare are
 * evaluated in complex arithmetic with one parameter perturbed by i*h, and
 * Im(output)/h is the exact derivative (no subtraction, so no cancellation).
 * Decisions (max(z, znear), min(v_train, v), the colour clamp) are taken on
 * real parts, as in the forward pass.                                      */
#include <complex.h>

typedef double complex cx;

static cx cdot3(const cx *a, const cx *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Real spherical harmonics in polynomial form: for a unit direction,
 * sin^m(theta) cos(m phi) and sin^m(theta) sin(m phi) are the real and
 * imaginary parts of (x + i y)^m (expanded with real recurrences), and
 * P_l^m(cos theta) = sin^m(theta) Q_l^m(z) with Q_m^m = (-1)^m (2m-1)!!,
 * Q_{m+1}^m = (2m+1) z Q_m^m, (l-m) Q_l^m = (2l-1) z Q_{l-1}^m - (l+m-1) Q_{l-2}^m. */
static void sh_poly_cx(int degree, const cx *d, cx *Y)
{
    cx x = d[0], y = d[1], z = d[2];
    cx Am[4], Bm[4];
    Am[0] = 1.0;
    Bm[0] = 0.0;
    for (int m = 1; m <= 3; ++m) {
        Am[m] = x * Am[m - 1] - y * Bm[m - 1];
        Bm[m] = x * Bm[m - 1] + y * Am[m - 1];
    }
    for (int m = 0; m <= degree; ++m) {
        cx Q[4];
        double dfact = 1.0;
        for (int k = 1; k <= 2 * m - 1; k += 2) dfact *= k;
        Q[m] = ((m % 2) ? -1.0 : 1.0) * dfact;
        if (m + 1 <= degree) Q[m + 1] = (2.0 * m + 1.0) * z * Q[m];
        for (int l = m + 2; l <= degree; ++l) Q[l] = ((2.0 * l - 1.0) * z * Q[l - 1] - (l + m - 1.0) * Q[l - 2]) / (l - m);
        for (int l = m; l <= degree; ++l) {
            double N = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * fact(l - m) / fact(l + m));
            if (m == 0) {
                Y[l * l + l] = N * Q[l];
            } else {
                Y[l * l + l + m] = sqrt(2.0) * N * Q[l] * Am[m];
                Y[l * l + l - m] = sqrt(2.0) * N * Q[l] * Bm[m];
            }
        }
    }
}

void or_sh_basis_poly(int degree, const double *dir, double *Y)
{
    double n = sqrt(dot3(dir, dir));
    cx d[3] = {dir[0] / n, dir[1] / n, dir[2] / n}, Yc[16];
    sh_poly_cx(degree, d, Yc);
    for (int b = 0; b < (degree + 1) * (degree + 1); ++b) Y[b] = creal(Yc[b]);
}

/* Parameter vector of one Gaussian: mu (3), log s (3), q (4), logit (1),
 * sh [(deg+1)^2][3] (coefficient-major).  Outputs: o_g (3), A (9), alpha~,
 * colour (3) -- the same quantities as or_prepare. */
#define OR_NPAR_MAX (11 + 48)
static void cont_cx(const cx *par, int deg, double v_train, const or_camera *cam, const or_settings *st, cx *out)
{
    double RV[9], tV[3], o[3];
    camera_parts(cam, RV, tV, o);
    const cx *mu = par, *ls = par + 3, *q = par + 6;
    cx logit = par[10];
    const cx *sh = par + 11;
    cx s[3], s2[3], shat[3], st_[3];
    for (int k = 0; k < 3; ++k) s[k] = cexp(ls[k]);
    cx alpha = 1.0 / (1.0 + cexp(-logit));
    cx qn = csqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    cx w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
    cx R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
               2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
               2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    cx muv[3];
    for (int r = 0; r < 3; ++r) muv[r] = RV[3 * r] * mu[0] + RV[3 * r + 1] * mu[1] + RV[3 * r + 2] * mu[2] + tV[r];
    cx dz = creal(muv[2]) > cam->znear ? muv[2] : (cx)cam->znear;
    cx v = cam->fx / dz;
    if (v_train > 0 && v_train < creal(v)) v = v_train;
    cx a = st->filter_mode == 1 ? (cx)0.0 : st->filter_k / (v * v);
    for (int k = 0; k < 3; ++k) {
        s2[k] = s[k] * s[k];
        shat[k] = s2[k] + a;
        st_[k] = csqrt(shat[k]);
    }
    cx d[3] = {mu[0] - o[0], mu[1] - o[1], mu[2] - o[2]};
    cx dn = csqrt(cdot3(d, d));
    for (int k = 0; k < 3; ++k) d[k] /= dn;
    cx alpha_t;
    if (st->filter_mode == 1) {
        alpha_t = alpha;
    } else if (st->filter_mode == 2) {
        alpha_t = alpha * csqrt((s2[0] * s2[1] * s2[2]) / (shat[0] * shat[1] * shat[2]));
    } else {
        cx dp[3];
        for (int k = 0; k < 3; ++k) dp[k] = R[k] * d[0] + R[3 + k] * d[1] + R[6 + k] * d[2];
        cx num = dp[0] * dp[0] * s2[1] * s2[2] + dp[1] * dp[1] * s2[0] * s2[2] + dp[2] * dp[2] * s2[0] * s2[1];
        cx den = dp[0] * dp[0] * shat[1] * shat[2] + dp[1] * dp[1] * shat[0] * shat[2] + dp[2] * dp[2] * shat[0] * shat[1];
        alpha_t = alpha * csqrt(num / den);
    }
    /* o_g = S~^-1 R^T (o - mu);  A = S~^-1 R^T R_V^T */
    cx om[3] = {o[0] - mu[0], o[1] - mu[1], o[2] - mu[2]};
    for (int r = 0; r < 3; ++r) {
        out[r] = (R[r] * om[0] + R[3 + r] * om[1] + R[6 + r] * om[2]) / st_[r];
        for (int c = 0; c < 3; ++c)
            out[3 + 3 * r + c] = (R[r] * RV[3 * c] + R[3 + r] * RV[3 * c + 1] + R[6 + r] * RV[3 * c + 2]) / st_[r];
    }
    out[12] = alpha_t;
    cx Y[16];
    sh_poly_cx(deg, d, Y);
    int nb = (deg + 1) * (deg + 1);
    for (int ch = 0; ch < 3; ++ch) {
        cx acc = 0.5;
        for (int b = 0; b < nb; ++b) acc += Y[b] * sh[3 * b + ch];
        out[13 + ch] = creal(acc) > 0 ? acc : (cx)0.0;
    }
}

/* Values of the continuous chain (real parts), for consistency checks against or_prepare. */
int or_cont_values(const or_scene *sc, const or_camera *cam, const or_settings *st, int64_t i, double *out16)
{
    const int64_t n = sc->n;
    int nb = (sc->sh_degree + 1) * (sc->sh_degree + 1);
    cx par[OR_NPAR_MAX], out[16];
    for (int k = 0; k < 3; ++k) { par[k] = sc->means[k * n + i]; par[3 + k] = sc->log_scales[k * n + i]; }
    for (int k = 0; k < 4; ++k) par[6 + k] = sc->quats[k * n + i];
    par[10] = sc->opacity_logits[i];
    for (int b = 0; b < nb; ++b)
        for (int ch = 0; ch < 3; ++ch) par[11 + 3 * b + ch] = sc->sh[((int64_t)b * 3 + ch) * n + i];
    cont_cx(par, sc->sh_degree, sc->v_train ? sc->v_train[i] : -1.0, cam, st, out);
    for (int k = 0; k < 16; ++k) out16[k] = creal(out[k]);
    return 0;
}

/*
 * Gradient of L = sum(dL_drgb * rgb) with respect to the scene parameters,
 * written (not accumulated) into g_means [3][n], g_log_scales [3][n],
 * g_quats [4][n], g_logits [n], g_sh [(deg+1)^2][3][n].  Also returns the
 * forward image and flags (rgb, T, flags as in or_render).
 */
int or_render_backward(const or_scene *sc, const or_camera *cam, const or_settings *st, const double *dL_drgb,
                       double *out_rgb, double *out_T, uint8_t *out_flags, double *g_means, double *g_log_scales,
                       double *g_quats, double *g_logits, double *g_sh)
{
    const int64_t n = sc->n;
    double *gi = (double *)calloc((size_t)(n > 0 ? n : 1) * OR_GI, sizeof(double));
    if (!gi) return 1;
    or_stats stt;
    int rc = render_impl(sc, cam, st, NULL, out_rgb, out_T, out_flags, NULL, &stt, dL_drgb, gi, NULL, NULL, NULL);
    if (rc) { free(gi); return rc; }
    const int deg = sc->sh_degree, nb = (deg + 1) * (deg + 1);
    const int npar = 11 + 3 * nb;
    const double h = 1e-20;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        const double *G = gi + OR_GI * i;
        double gpar[OR_NPAR_MAX];
        for (int p = 0; p < npar; ++p) gpar[p] = 0.0;
        int any = 0;
        for (int k = 0; k < OR_GI; ++k) any |= G[k] != 0.0;
        if (any) {
            cx par[OR_NPAR_MAX], out[16];
            for (int k = 0; k < 3; ++k) { par[k] = sc->means[k * n + i]; par[3 + k] = sc->log_scales[k * n + i]; }
            for (int k = 0; k < 4; ++k) par[6 + k] = sc->quats[k * n + i];
            par[10] = sc->opacity_logits[i];
            for (int b = 0; b < nb; ++b)
                for (int ch = 0; ch < 3; ++ch) par[11 + 3 * b + ch] = sc->sh[((int64_t)b * 3 + ch) * n + i];
            double vt = sc->v_train ? sc->v_train[i] : -1.0;
            for (int p = 0; p < npar; ++p) {
                cx keep = par[p];
                par[p] = creal(keep) + I * h;
                cont_cx(par, deg, vt, cam, st, out);
                par[p] = keep;
                double acc = 0.0;
                for (int k = 0; k < 16; ++k) acc += G[k] * cimag(out[k]) / h;
                gpar[p] = acc;
            }
        }
        for (int k = 0; k < 3; ++k) { g_means[k * n + i] = gpar[k]; g_log_scales[k * n + i] = gpar[3 + k]; }
        for (int k = 0; k < 4; ++k) g_quats[k * n + i] = gpar[6 + k];
        g_logits[i] = gpar[10];
        for (int b = 0; b < nb; ++b)
            for (int ch = 0; ch < 3; ++ch) g_sh[((int64_t)b * 3 + ch) * n + i] = gpar[11 + 3 * b + ch];
    }
    free(gi);
    return 0;
}

/* The same 16 quantities from the real-arithmetic preparation. */
int or_prepare_values(const or_scene *sc, const or_camera *cam, const or_settings *st, int64_t i, double *out16)
{
    or_gauss g;
    or_prepare(sc, cam, st, i, &g);
    for (int k = 0; k < 3; ++k) out16[k] = g.o_g[k];
    for (int k = 0; k < 9; ++k) out16[3 + k] = g.A[k];
    out16[12] = g.alpha_t;
    for (int k = 0; k < 3; ++k) out16[13 + k] = g.color[k];
    return g.status;
}

/* ------------------------------------------------------------------------ */
/* Training sampling frequency (Sec. 3.2): the filter's stored per-Gaussian
 * maximum of f / d over the N_c training cameras, f the focal length in
 * pixels, d the view-space depth of the mean; Eq.(13) clamps the render-time
 * frequency to it.  Reading: a camera counts when the mean lies in front of
 * its near plane and projects inside the image (border included); when no
 * camera sees the mean, every camera with depth > znear counts; with none of
 * those either the value is +inf (no clamp).  f = fx.
 * Arithmetic order (fixed; the oracle is built without fused multiply-add):
 * X = ((R0 mu0 + R1 mu1) + R2 mu2) + t per row, x = cx + (fx X0) / z,
 * y = cy + (fy X1) / z, v = fx / z.
 * flags[i] = 1 when a frustum decision of some camera lies within 1e-9
 * (relative to the image size or znear) of its boundary. */
void or_training_frequency(const double *means, int64_t n, int ncam, const or_camera *cams, double *out,
                           uint8_t *flags)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double mu[3] = {means[i], means[n + i], means[2 * n + i]};
        double best_in = 0.0, best_any = 0.0;
        int near_edge = 0;
        for (int c = 0; c < ncam; ++c) {
            const double *V = cams[c].viewmat;
            double X[3];
            for (int r = 0; r < 3; ++r) X[r] = ((V[4 * r] * mu[0] + V[4 * r + 1] * mu[1]) + V[4 * r + 2] * mu[2]) + V[4 * r + 3];
            const double z = X[2], zn = cams[c].znear;
            if (fabs(z - zn) <= 1e-9 * fmax(1.0, zn)) near_edge = 1;
            if (!(z > zn)) continue;
            const double x = cams[c].cx + (cams[c].fx * X[0]) / z, y = cams[c].cy + (cams[c].fy * X[1]) / z;
            const double v = cams[c].fx / z;
            const double W = cams[c].width, H = cams[c].height;
            if (fabs(x) <= 1e-9 * W || fabs(x - W) <= 1e-9 * W || fabs(y) <= 1e-9 * H || fabs(y - H) <= 1e-9 * H)
                near_edge = 1;
            if (v > best_any) best_any = v;
            if (x >= 0.0 && x <= W && y >= 0.0 && y <= H && v > best_in) best_in = v;
        }
        out[i] = best_in > 0.0 ? best_in : (best_any > 0.0 ? best_any : INFINITY);
        if (flags) flags[i] = (uint8_t)near_edge;
    }
}
