// K1: per-Gaussian preprocessing, one thread per Gaussian.
//
// Reads the structure-of-arrays scene (coalesced) and writes, per Gaussian,
// a status word, a tile rectangle, a 128-byte blend record and a 128-byte
// culling record.  Geometry is computed in double precision (the pass is
// bound by HBM traffic, and double precision keeps the bounds quadratic and
// the anchored record free of cancellation); the records are stored as float.
#include "aaa_internal.h"
#include "gauss_setup.h"

namespace aaa {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kBoundEps = 1e-3;  // clamp margin of the angular bounds (rad)
constexpr double kBoundTan = 999.9996666666443;  // 1 / tan(kBoundEps): the tangent at pi/2 - kBoundEps

// Bounds of the level-tau ellipsoid seen from the camera in one view plane
// (Sec. 3.3, Eq. 14-17), as the tangents lo < hi of the two bounding angles
// (lateral over depth: screen offsets over focal length).  Rows a (lateral:
// view x or y) and c (depth) of M = R_V R S~ and the matching mean
// coordinates.  Returns false when the visible wedge is empty; sets full =
// true when the lateral axis line meets the ellipsoid (negative
// discriminant: the whole screen range).  Angles are clamped to
// (-pi/2, pi/2) by kBoundEps.
__device__ bool view_bounds(const double *Ma, const double *Mc, double ma, double mc, double tau, double &lo,
                            double &hi, bool &full)
{
    full = false;
    // s_ij = tau (M_i . M_j) - mu_i mu_j; discriminant s_ac^2 - s_aa s_cc,
    // expanded so that the mu^4 terms cancel exactly:
    //   D = tau |mc Ma - ma Mc|^2 - tau^2 |Ma x Mc|^2
    double e[3], x[3];
    for (int k = 0; k < 3; ++k) e[k] = mc * Ma[k] - ma * Mc[k];
    cross3d(Ma, Mc, x);
    double D = tau * dot3(e, e) - tau * tau * dot3(x, x);
    if (D < 0.0) {
        full = true;
        return true;
    }
    double sac = tau * dot3(Ma, Mc) - ma * mc;
    double scc = tau * dot3(Mc, Mc) - mc * mc;
    double sq = sqrt(D);
    if (mc > 0.0 && scc < 0.0) {
        // The ellipsoid lies in front of the camera (its depth extent
        // sqrt(tau |M_c|^2) is below the mean's depth): both bounding angles
        // are in (-pi/2, pi/2), where the tangent is monotonic, and the
        // tangent of each angle atan2(s_ac +- sqrt(D), s_cc) is the quotient
        // itself.
        double r1 = (sac + sq) / scc, r2 = (sac - sq) / scc;
        lo = fmax(fmin(r1, r2), -kBoundTan);
        hi = fmin(fmax(r1, r2), kBoundTan);
        return lo < hi;
    }
    double ra = atan2(sac + sq, scc);
    double rb = atan2(sac - sq, scc);
    double tm = atan2(ma, mc);
    // representative of a root (mod pi) in [tm - pi, tm)
    auto below = [&](double r) {
        double t = r - tm;
        t -= kPi * floor(t / kPi);
        return tm - kPi + t;
    };
    double a1 = below(ra), a2 = below(rb) + kPi;
    double b1 = below(rb), b2 = below(ra) + kPi;
    double t1, t2;
    if (a2 - a1 <= b2 - b1) { t1 = a1; t2 = a2; } else { t1 = b1; t2 = b2; }
    // bring the wedge to the representation that can meet (-pi/2, pi/2)
    if (t1 > 0.5 * kPi) { t1 -= 2.0 * kPi; t2 -= 2.0 * kPi; }
    if (t2 < -0.5 * kPi) { t1 += 2.0 * kPi; t2 += 2.0 * kPi; }
    t1 = fmax(t1, -0.5 * kPi + kBoundEps);
    t2 = fmin(t2, 0.5 * kPi - kBoundEps);
    if (!(t1 < t2)) return false;
    lo = tan(t1);
    hi = tan(t2);
    return true;
}

// Anchored line record and culling geometry of a visible item whose tile
// rectangle is [x0, x1) x [y0, y1) (the anchor: the pixel centre nearest the
// projected mean, kept inside the rectangle's pixels; the rectangle's centre
// when the mean is not in front).
__device__ void build_geom(const Setup &S, const CamDev &cam, int x0, int x1, int y0, int y1, TileGeom<double> &g)
{
    const double *muv = S.muv, *M = S.M, *A = S.A, *og = S.og;
    int pxl = x0 * kTile, pxh = min(x1 * kTile, cam.width) - 1;
    int pyl = y0 * kTile, pyh = min(y1 * kTile, cam.height) - 1;
    double xa, ya;
    if (muv[2] > 0.0) {
        double xm = cam.cx + cam.fx * muv[0] / muv[2];
        double ym = cam.cy + cam.fy * muv[1] / muv[2];
        xa = fmin(fmax(floor(xm), (double)pxl), (double)pxh) + 0.5;
        ya = fmin(fmax(floor(ym), (double)pyl), (double)pyh) + 0.5;
    } else {
        xa = floor(0.5 * (pxl + pxh)) + 0.5;
        ya = floor(0.5 * (pyl + pyh)) + 0.5;
    }
    // anchored line coefficients (Eq. 4-5 written as o_g x r_g and -o_g . r_g)
    double ua = (xa - cam.cx) / cam.fx, va = (ya - cam.cy) / cam.fy;
    g.xa = xa;
    g.ya = ya;
    for (int r = 0; r < 3; ++r) {
        g.c0[r] = A[3 * r] * ua + A[3 * r + 1] * va + A[3 * r + 2];
        g.c1[r] = A[3 * r] / cam.fx;
        g.c2[r] = A[3 * r + 1] / cam.fy;
    }
    // scale so that |c0| = 1 (rho^2 and depth are invariant)
    double lam = 1.0 / sqrt(dot3(g.c0, g.c0));
    for (int r = 0; r < 3; ++r) { g.c0[r] *= lam; g.c1[r] *= lam; g.c2[r] *= lam; }
    cross3d(og, g.c0, g.w0);
    cross3d(og, g.c1, g.w1);
    cross3d(og, g.c2, g.w2);
    // c carries one factor lambda already; l needs lambda^2
    g.l[0] = -lam * dot3(og, g.c0);
    g.l[1] = -lam * dot3(og, g.c1);
    g.l[2] = -lam * dot3(og, g.c2);
    g.og2 = S.og2;
    // culling geometry of the screen planes relative to the anchor
    double G[9];  // Sigma~ in view space = M M^T
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) G[3 * r + c] = dot3(&M[3 * r], &M[3 * c]);
    g.dx0 = muv[0] - ua * muv[2];
    g.dx1 = muv[2] / cam.fx;
    g.dy0 = muv[1] - va * muv[2];
    g.dy1 = muv[2] / cam.fy;
    for (int k = 0; k < 3; ++k) {
        g.nx0[k] = M[k] - ua * M[6 + k];
        g.nx1[k] = M[6 + k] / cam.fx;
        g.ny0[k] = M[3 + k] - va * M[6 + k];
        g.ny1[k] = M[6 + k] / cam.fy;
        g.qx0[k] = G[3 * k] - ua * G[3 * k + 2];
        g.qx1[k] = G[3 * k + 2] / cam.fx;
        g.qy0[k] = G[3 * k + 1] - va * G[3 * k + 2];
        g.qy1[k] = G[3 * k + 2] / cam.fy;
        g.muv[k] = muv[k];
    }
}

// Whether the mean lies inside the pyramid of the whole view (then the
// minimum of Eq. 18 over the view is 0 and the item is not culled there).
__device__ __forceinline__ bool mean_in_view(const TileGeom<double> &g, const CamDev &cam)
{
    const double sL = g.dx0 - (0.0 - g.xa) * g.dx1, sR = g.dx0 - ((double)cam.width - g.xa) * g.dx1;
    const double sT = g.dy0 - (0.0 - g.ya) * g.dy1, sB = g.dy0 - ((double)cam.height - g.ya) * g.dy1;
    return !(sL < 0.0 || sR > 0.0 || sT < 0.0 || sB > 0.0);
}

// One item (Gaussian i, view v), item = i * nviews + v: the threads of a
// Gaussian's views are adjacent, so its parameters are fetched from HBM once
// per batch.  Returns true when the item is visible so far but its mean
// lies outside the view pyramid: the cull of Sec. 3.4 against the whole view
// is then left to k_view_cull (its double-precision pyramid minimum needs
// more registers than the rest of this pass).  The SH degree is a template
// parameter, so that the colour's coefficient loads unroll and are all in
// flight together.
template <int DEG>
__device__ bool preprocess_item(const PreArgs &a, int64_t item)
{
    const int64_t i = item / a.nviews;
    const int v = (int)(item - i * a.nviews);
    const ViewDev &vw = a.views[v];
    const int64_t n = a.n;
    a.rect[item] = make_int4(0, 0, 0, 0);
    a.area[item] = 0u;
    Setup S;
    const int st0 = setup_gaussian(a, i, vw, S);
    if (st0 != kVisible) {
        a.status[item] = st0;
        return false;
    }
    const double *muv = S.muv, *M = S.M, *d = S.d;
    const double alpha_t = S.alpha_t, tau = S.tau, og2 = S.og2;
    if (og2 < tau) {  // Sec. 3.3: camera inside the ellipsoid
        a.status[item] = kCamInside;
        return false;
    }
    // Sec. 3.3 bounds in the x-z and y-z view planes
    const CamDev &cam = vw.cam;
    double tx_lo, tx_hi, ty_lo, ty_hi;
    bool fullx, fully;
    bool okx = view_bounds(&M[0], &M[6], muv[0], muv[2], tau, tx_lo, tx_hi, fullx);
    bool oky = view_bounds(&M[3], &M[6], muv[1], muv[2], tau, ty_lo, ty_hi, fully);
    if (!okx || !oky) {
        a.status[item] = kOutside;
        return false;
    }
    int x0 = 0, x1 = cam.tiles_x, y0 = 0, y1 = cam.tiles_y;
    float4 box = make_float4(-INFINITY, INFINITY, -INFINITY, INFINITY);
    if (!fullx) {
        double px_lo = cam.cx + cam.fx * tx_lo - 1e-3, px_hi = cam.cx + cam.fx * tx_hi + 1e-3;
        x0 = (int)fmax(0.0, fmin((double)cam.tiles_x, floor(px_lo / kTile)));
        x1 = (int)fmax(0.0, fmin((double)cam.tiles_x, floor(px_hi / kTile) + 1.0));
        box.x = (float)px_lo;
        box.y = (float)px_hi;
    }
    if (!fully) {
        double py_lo = cam.cy + cam.fy * ty_lo - 1e-3, py_hi = cam.cy + cam.fy * ty_hi + 1e-3;
        y0 = (int)fmax(0.0, fmin((double)cam.tiles_y, floor(py_lo / kTile)));
        y1 = (int)fmax(0.0, fmin((double)cam.tiles_y, floor(py_hi / kTile) + 1.0));
        box.z = (float)py_lo;
        box.w = (float)py_hi;
    }
    if (x0 >= x1 || y0 >= y1) {
        a.status[item] = kOutside;
        return false;
    }
    TileGeom<double> g;
    build_geom(S, cam, x0, x1, y0, y1, g);
    const bool pending = !mean_in_view(g, cam);
    float4 *rec = a.rec + (size_t)item * kRecQuads;
    rec[0] = make_float4(g.c0[0], g.c0[1], g.c0[2], g.c1[0]);
    rec[1] = make_float4(g.c1[1], g.c1[2], g.c2[0], g.c2[1]);
    rec[2] = make_float4(g.c2[2], g.w0[0], g.w0[1], g.w0[2]);
    rec[3] = make_float4(g.w1[0], g.w1[1], g.w1[2], g.w2[0]);
    rec[4] = make_float4(g.w2[1], g.w2[2], g.l[0], g.l[1]);
    rec[5] = make_float4(g.l[2], g.xa, g.ya, alpha_t);
    // prefilter level slightly above tau so that it never rejects an
    // evaluation the exact alpha test would accept
    rec[6] = make_float4((float)(tau * (1.0 + 1e-4) + 1e-6), (float)tau, (float)og2, 0.f);
    float4 *cu = a.cull + (size_t)item * kCullQuads;
    cu[0] = make_float4(g.dx0, g.dx1, g.dy0, g.dy1);
    cu[1] = make_float4(g.nx0[0], g.nx0[1], g.nx0[2], g.nx1[0]);
    cu[2] = make_float4(g.nx1[1], g.nx1[2], g.ny0[0], g.ny0[1]);
    cu[3] = make_float4(g.ny0[2], g.ny1[0], g.ny1[1], g.ny1[2]);
    cu[4] = make_float4(g.qx0[0], g.qx0[1], g.qx0[2], g.qx1[0]);
    cu[5] = make_float4(g.qx1[1], g.qx1[2], g.qy0[0], g.qy0[1]);
    cu[6] = make_float4(g.qy0[2], g.qy1[0], g.qy1[1], g.qy1[2]);
    cu[7] = make_float4(muv[0], muv[1], muv[2], 0.f);
    a.rect[item] = make_int4(x0, x1, y0, y1);
    a.bbox[item] = box;
    a.area[item] = (uint32_t)((x1 - x0) * (y1 - y0));
    a.status[item] = kVisible;
    // colour from real SH along the camera->mean direction (after the
    // geometry is stored, so that its registers are free for the loads)
    constexpr int nb = (DEG + 1) * (DEG + 1);
    float c[3 * nb];
#pragma unroll
    for (int k = 0; k < 3 * nb; ++k) c[k] = a.sh[(int64_t)k * n + i];  // coefficient b, channel ch at k = 3 b + ch
    double Y[16];
    sh_eval(DEG, d[0], d[1], d[2], Y);
    float col[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.5;
#pragma unroll
        for (int b = 0; b < nb; ++b) acc += Y[b] * (double)c[3 * b + ch];
        col[ch] = (float)fmax(acc, 0.0);
    }
    rec[7] = make_float4(col[0], col[1], col[2], 0.f);
    return pending;
}

// Items with their mean outside the view pyramid are listed per workgroup
// (pending[256 b + k], k < pending_n[b]) for k_view_cull.  Three waves per
// SIMD: the pass then holds its 154 VGPRs without spilling (at four, about
// 20 spilled registers per lane moved more scratch traffic than the
// parameters themselves).
template <int DEG>
__global__ __launch_bounds__(256, 3) void k_preprocess(PreArgs a)
{
    __shared__ uint32_t n_pend;
    if (threadIdx.x == 0) n_pend = 0;
    __syncthreads();
    const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool pend = item < a.n * a.nviews && preprocess_item<DEG>(a, item);
    const uint64_t m = __ballot(pend);
    uint32_t base = 0;
    if (__lane_id() == 0 && m) base = atomicAdd(&n_pend, (uint32_t)__popcll(m));
    base = (uint32_t)__shfl((int)base, 0);
    if (pend) {
        const uint64_t below = __lane_id() == 0 ? 0ull : (~0ull >> (64 - __lane_id()));
        a.pending[(size_t)blockIdx.x * 256 + base + (uint32_t)__popcll(m & below)] = (uint32_t)item;
    }
    __syncthreads();
    if (threadIdx.x == 0) a.pending_n[blockIdx.x] = n_pend;
}

// Sec. 3.4: cull the listed items against the pyramid of the whole view
// (double-precision minimum of Eq. 18, same geometry as the records).  One
// workgroup gathers the lists of kViewCullGroup preprocess workgroups, so
// that its waves run full (each list holds only the few items of its 256
// whose mean lies outside the view).
constexpr int kViewCullGroup = 8;

__global__ __launch_bounds__(256) void k_view_cull(PreArgs a, int64_t nlists)
{
    __shared__ uint32_t pre[kViewCullGroup + 1];
    const int64_t l0 = (int64_t)blockIdx.x * kViewCullGroup;
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int k = 0; k < kViewCullGroup; ++k) {
            pre[k] = acc;
            acc += l0 + k < nlists ? a.pending_n[l0 + k] : 0u;
        }
        pre[kViewCullGroup] = acc;
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < pre[kViewCullGroup]; j += blockDim.x) {
        int k = 0;
        while (j >= pre[k + 1]) ++k;  // the list holding the j-th gathered item
        const int64_t item = a.pending[(size_t)(l0 + k) * 256 + (j - pre[k])];
        const int64_t i = item / a.nviews;
        const int v = (int)(item - i * a.nviews);
        const ViewDev &vw = a.views[v];
        const CamDev &cam = vw.cam;
        Setup S;
        setup_gaussian(a, i, vw, S);
        const int4 r = a.rect[item];
        TileGeom<double> g;
        build_geom(S, cam, r.x, r.y, r.z, r.w, g);
        const double mview = tile_min_rho2<double>(g, 0.0, (double)cam.width, 0.0, (double)cam.height, cam);
        if (!(mview < S.tau)) {
            a.status[item] = kOutside;
            a.rect[item] = make_int4(0, 0, 0, 0);
            a.area[item] = 0u;
        }
    }
}

}  // namespace

hipError_t launch_preprocess(const PreArgs &a, hipStream_t s)
{
    if (a.n <= 0 || a.nviews <= 0) return hipSuccess;
    int64_t blocks = (a.n * a.nviews + 255) / 256;
    switch (a.sh_degree) {
    case 0: hipLaunchKernelGGL(k_preprocess<0>, dim3((unsigned)blocks), dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL(k_preprocess<1>, dim3((unsigned)blocks), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_preprocess<2>, dim3((unsigned)blocks), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(k_preprocess<3>, dim3((unsigned)blocks), dim3(256), 0, s, a); break;
    }
    hipLaunchKernelGGL(k_view_cull, dim3((unsigned)((blocks + kViewCullGroup - 1) / kViewCullGroup)), dim3(256), 0, s,
                       a, blocks);
    return hipGetLastError();
}

}  // namespace aaa
