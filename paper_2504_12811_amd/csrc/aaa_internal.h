// Internal definitions shared by the HIP kernels and the host library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aaa {

constexpr int kTile = 16;          // tile edge in pixels
constexpr int kRecQuads = 8;       // float4 per blend record (128 B)
constexpr int kCullQuads = 8;      // float4 per culling record (128 B)
constexpr float kLog2eHalf = 0.72134752044448170368f;  // log2(e) / 2
constexpr int kGradStride = 24;    // floats per Gaussian in the record-gradient buffer:
                                   // c0 c1 c2 w0 w1 w2 (18), alpha~ (1), colour (3), pad

enum Status : int32_t { kVisible = 0, kInvalid = 1, kLowOpacity = 2, kCamInside = 3, kOutside = 4 };

// Blend record of one Gaussian for one view (128 B, float4 granularity):
//   r_g(dx,dy) = c0 + dx c1 + dy c2   line direction in normalised Gaussian space
//   w(dx,dy)   = w0 + dx w1 + dy w2   o_g x r_g
//   l(dx,dy)   = l0 + dx l1 + dy l2   -o_g . r_g
// with (dx, dy) the pixel-centre offset from the anchor (xa, ya), itself a
// pixel centre, so offsets are exact in float.  rho^2 = |w|^2 / |r_g|^2 and
// the depth of the maximum is l / |r_g|^2 (c, w scaled by lambda, l by lambda^2).
//   q0 = c0x c0y c0z c1x     q4 = w2y w2z l0 l1
//   q1 = c1y c1z c2x c2y     q5 = l2 xa ya alpha~
//   q2 = c2z w0x w0y w0z     q6 = tau_pre tau og2 -
//   q3 = w1x w1y w1z w2x     q7 = r g b -
// Culling record (screen-plane geometry relative to the anchor, view space):
//   plane x = xa + D: normal in Gaussian space nx0 - D nx1, offset dx0 - D dx1,
//   Sigma~_view (1,0,-u) = qx0 - D qx1; same for y.
//   p0 = dx0 dx1 dy0 dy1      p4 = qx0 qx1.x
//   p1 = nx0 nx1.x            p5 = qx1.yz qy0.xy
//   p2 = nx1.yz ny0.xy        p6 = qy0.z qy1
//   p3 = ny0.z ny1            p7 = mu_view -
struct Rec {
    float c0[3], c1[3], c2[3], w0[3], w1[3], w2[3], l[3];
    float xa, ya, alpha, tau_pre, tau, og2;
};

template <typename T>
struct TileGeom {
    T xa, ya;
    T c0[3], c1[3], c2[3], w0[3], w1[3], w2[3], l[3];
    T og2;
    T dx0, dx1, dy0, dy1;
    T nx0[3], nx1[3], ny0[3], ny1[3];
    T qx0[3], qx1[3], qy0[3], qy1[3];
    T muv[3];
};

struct CamDev {
    double fx, fy, cx, cy;
    int32_t width, height, tiles_x, tiles_y;
    double znear;
};

// One view of a batch (device memory).  Items of the per-Gaussian stages are
// indexed i * nviews + v; tiles of view v are tile_base + ty * tiles_x + tx in
// the global tile numbering shared by the sort and the ranges.
struct ViewDev {
    double RV[9], tV[3], o[3];  // world->view rotation, translation, camera centre
    CamDev cam;
    int32_t tile_base;
    int32_t _pad;
    int64_t pix_base;            // offset of the view's pixels in the per-pixel scratch
    float bg[3];
    float *out_rgb, *out_T;      // [3][H][W], [H][W]
    const float *dL_drgb;        // backward only
};

template <typename T>
__device__ __forceinline__ T dot3(const T *a, const T *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Minimum of rho^2 over the pyramid of the screen rectangle [x0,x1]x[y0,y1]
// (Eq. 18).  The pyramid is four half-spaces through the camera centre; the
// minimum of the convex rho^2 lies on a face whose half-space the mean
// violates (or is 0 when the mean is inside).  For each such face: the plane
// minimum if it lies inside the face (checked with a small slack so that the
// result never exceeds the exact minimum by more than rounding), and the
// minima on the face's two edge rays (the apex when the edge minimum is
// behind the camera).  Rectangle corners are given relative to the anchor.
template <typename T>
__device__ __forceinline__ T edge_min(const TileGeom<T> &g, T dX, T dY)
{
    T r[3], w[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r[k] = g.c0[k] + dX * g.c1[k] + dY * g.c2[k];
        w[k] = g.w0[k] + dX * g.w1[k] + dY * g.w2[k];
    }
    T l = g.l[0] + dX * g.l[1] + dY * g.l[2];
    T v = dot3(w, w) / dot3(r, r);
    return l > T(0) ? v : g.og2;
}

// plane x = xa + dX (vert=true) or y = ya + dY (vert=false); s = signed plane
// offset; [lo, hi] = the other axis' range as view slopes.
template <typename T>
__device__ __forceinline__ T plane_min(const TileGeom<T> &g, bool vert, T D, T s, T lo, T hi)
{
    const T *n0 = vert ? g.nx0 : g.ny0;
    const T *n1 = vert ? g.nx1 : g.ny1;
    const T *q0 = vert ? g.qx0 : g.qy0;
    const T *q1 = vert ? g.qx1 : g.qy1;
    T n[3], q[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        n[k] = n0[k] - D * n1[k];
        q[k] = q0[k] - D * q1[k];
    }
    T nn = dot3(n, n);
    T val = s * s / nn;
    T f = s / nn;
    T X[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) X[k] = g.muv[k] - f * q[k];
    T o = vert ? X[1] : X[0];  // the coordinate bounded by [lo, hi] * z
    T a = o - lo * X[2];
    T b = hi * X[2] - o;
    T scale = (o < T(0) ? -o : o) + (X[2] < T(0) ? -X[2] : X[2]) * ((lo < T(0) ? -lo : lo) + (hi < T(0) ? -hi : hi));
    T tol = (sizeof(T) == 4 ? T(1e-4) : T(1e-9)) * scale;
    bool feas = a >= -tol && b >= -tol;
    return feas ? val : T(INFINITY);
}

template <typename T>
__device__ __forceinline__ T tile_min_rho2(const TileGeom<T> &g, T x0, T x1, T y0, T y1, const CamDev &cam)
{
    T dX0 = x0 - g.xa, dX1 = x1 - g.xa, dY0 = y0 - g.ya, dY1 = y1 - g.ya;
    T sL = g.dx0 - dX0 * g.dx1;
    T sR = g.dx0 - dX1 * g.dx1;
    T sT = g.dy0 - dY0 * g.dy1;
    T sB = g.dy0 - dY1 * g.dy1;
    bool vL = sL < T(0), vR = sR > T(0), vT = sT < T(0), vB = sB > T(0);
    if (!(vL || vR || vT || vB)) return T(0);
    T best = g.og2;
    T u0 = (x0 - T(cam.cx)) / T(cam.fx), u1 = (x1 - T(cam.cx)) / T(cam.fx);
    T v0 = (y0 - T(cam.cy)) / T(cam.fy), v1 = (y1 - T(cam.cy)) / T(cam.fy);
    if (vL || vT) best = fmin(best, edge_min(g, dX0, dY0));
    if (vL || vB) best = fmin(best, edge_min(g, dX0, dY1));
    if (vR || vT) best = fmin(best, edge_min(g, dX1, dY0));
    if (vR || vB) best = fmin(best, edge_min(g, dX1, dY1));
    if (vL) best = fmin(best, plane_min(g, true, dX0, sL, v0, v1));
    if (vR) best = fmin(best, plane_min(g, true, dX1, sR, v0, v1));
    if (vT) best = fmin(best, plane_min(g, false, dY0, sT, u0, u1));
    if (vB) best = fmin(best, plane_min(g, false, dY1, sB, u0, u1));
    return best;
}

__device__ __forceinline__ void load_tile_geom(const float4 *__restrict__ rec, const float4 *__restrict__ cull, TileGeom<float> &g)
{
    float4 q0 = rec[0], q1 = rec[1], q2 = rec[2], q3 = rec[3], q4 = rec[4], q5 = rec[5], q6 = rec[6];
    g.c0[0] = q0.x; g.c0[1] = q0.y; g.c0[2] = q0.z;
    g.c1[0] = q0.w; g.c1[1] = q1.x; g.c1[2] = q1.y;
    g.c2[0] = q1.z; g.c2[1] = q1.w; g.c2[2] = q2.x;
    g.w0[0] = q2.y; g.w0[1] = q2.z; g.w0[2] = q2.w;
    g.w1[0] = q3.x; g.w1[1] = q3.y; g.w1[2] = q3.z;
    g.w2[0] = q3.w; g.w2[1] = q4.x; g.w2[2] = q4.y;
    g.l[0] = q4.z; g.l[1] = q4.w; g.l[2] = q5.x;
    g.xa = q5.y; g.ya = q5.z;
    g.og2 = q6.z;
    float4 p0 = cull[0], p1 = cull[1], p2 = cull[2], p3 = cull[3], p4 = cull[4], p5 = cull[5], p6 = cull[6], p7 = cull[7];
    g.dx0 = p0.x; g.dx1 = p0.y; g.dy0 = p0.z; g.dy1 = p0.w;
    g.nx0[0] = p1.x; g.nx0[1] = p1.y; g.nx0[2] = p1.z;
    g.nx1[0] = p1.w; g.nx1[1] = p2.x; g.nx1[2] = p2.y;
    g.ny0[0] = p2.z; g.ny0[1] = p2.w; g.ny0[2] = p3.x;
    g.ny1[0] = p3.y; g.ny1[1] = p3.z; g.ny1[2] = p3.w;
    g.qx0[0] = p4.x; g.qx0[1] = p4.y; g.qx0[2] = p4.z;
    g.qx1[0] = p4.w; g.qx1[1] = p5.x; g.qx1[2] = p5.y;
    g.qy0[0] = p5.z; g.qy0[1] = p5.w; g.qy0[2] = p6.x;
    g.qy1[0] = p6.y; g.qy1[1] = p6.z; g.qy1[2] = p6.w;
    g.muv[0] = p7.x; g.muv[1] = p7.y; g.muv[2] = p7.z;
}

// The record part of load_tile_geom (lines, depth numerator, anchor).
__device__ __forceinline__ void load_line_geom(const float4 *__restrict__ rec, TileGeom<float> &g)
{
    float4 q0 = rec[0], q1 = rec[1], q2 = rec[2], q3 = rec[3], q4 = rec[4], q5 = rec[5];
    g.c0[0] = q0.x; g.c0[1] = q0.y; g.c0[2] = q0.z;
    g.c1[0] = q0.w; g.c1[1] = q1.x; g.c1[2] = q1.y;
    g.c2[0] = q1.z; g.c2[1] = q1.w; g.c2[2] = q2.x;
    g.w0[0] = q2.y; g.w0[1] = q2.z; g.w0[2] = q2.w;
    g.w1[0] = q3.x; g.w1[1] = q3.y; g.w1[2] = q3.z;
    g.w2[0] = q3.w; g.w2[1] = q4.x; g.w2[2] = q4.y;
    g.l[0] = q4.z; g.l[1] = q4.w; g.l[2] = q5.x;
    g.xa = q5.y; g.ya = q5.z;
}

// Wave-wide scans and reductions on DPP lane moves (VALU, a few cycles each)
// instead of LDS permutes: an inclusive sum shifts within rows of 16 lanes
// (row_shr 1, 2, 4, 8), then adds lane 15's sum into rows 1 and 3 and lane
// 31's into rows 2 and 3 (row_bcast); lanes whose source lies outside the
// row, or whose row is masked off, add the 0 passed as the old value.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x)
{
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15, rows 1 and 3
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31, rows 2 and 3
    return x;
}

__device__ __forceinline__ uint64_t wave_incl_sum64(uint64_t x)
{
#define AAA_DPP64_STEP(ctrl, rows)                                                                              \
    {                                                                                                           \
        const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, ctrl, rows, 0xF, false);  \
        const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), ctrl, rows, 0xF, \
                                                                  false);                                       \
        x += ((uint64_t)hi << 32) | lo;                                                                         \
    }
    AAA_DPP64_STEP(0x111, 0xF)
    AAA_DPP64_STEP(0x112, 0xF)
    AAA_DPP64_STEP(0x114, 0xF)
    AAA_DPP64_STEP(0x118, 0xF)
    AAA_DPP64_STEP(0x142, 0xA)
    AAA_DPP64_STEP(0x143, 0xC)
#undef AAA_DPP64_STEP
    return x;
}

// Minimum and maximum over the wave, returned to every lane (wave-uniform):
// quad swaps and the half-row and row mirrors leave each row's result in all
// of its lanes, then the four row results are read out.
__device__ __forceinline__ void wave_minmax(uint32_t &mn, uint32_t &mx)
{
#define AAA_DPP_MINMAX(ctrl)                                                                  \
    mn = min(mn, (uint32_t)__builtin_amdgcn_update_dpp((int)mn, (int)mn, ctrl, 0xF, 0xF, false)); \
    mx = max(mx, (uint32_t)__builtin_amdgcn_update_dpp((int)mx, (int)mx, ctrl, 0xF, 0xF, false));
    AAA_DPP_MINMAX(0xB1)   // quad_perm 1,0,3,2
    AAA_DPP_MINMAX(0x4E)   // quad_perm 2,3,0,1
    AAA_DPP_MINMAX(0x141)  // row_half_mirror
    AAA_DPP_MINMAX(0x140)  // row_mirror
#undef AAA_DPP_MINMAX
    mn = min(min((uint32_t)__builtin_amdgcn_readlane((int)mn, 0), (uint32_t)__builtin_amdgcn_readlane((int)mn, 16)),
             min((uint32_t)__builtin_amdgcn_readlane((int)mn, 32), (uint32_t)__builtin_amdgcn_readlane((int)mn, 48)));
    mx = max(max((uint32_t)__builtin_amdgcn_readlane((int)mx, 0), (uint32_t)__builtin_amdgcn_readlane((int)mx, 16)),
             max((uint32_t)__builtin_amdgcn_readlane((int)mx, 32), (uint32_t)__builtin_amdgcn_readlane((int)mx, 48)));
}

__device__ __forceinline__ uint32_t wave_max(uint32_t x)
{
    uint32_t mn = 0u;
    wave_minmax(mn, x);
    return x;
}

// Order-preserving map of a float to uint32 (-0 -> +0; NaN never occurs).
__device__ __forceinline__ uint32_t order_key(float f)
{
    uint32_t b = __float_as_uint(f);
    if (b == 0x80000000u) b = 0u;
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Tile-pair keep test of the pair counter: pyramid minimum below this
// limit, tau with a relative slack of 2e-4 (+1e-5) for float rounding.
__device__ __forceinline__ float keep_limit(float tau) { return tau * (1.0f + 2e-4f) + 1e-5f; }

}  // namespace aaa

// Host-side launchers (defined in the .hip files).
namespace aaa {
struct PreArgs {
    const float *means, *log_scales, *quats, *logits, *sh, *v_train;
    int64_t n;
    int sh_degree;
    const ViewDev *views;
    int nviews;
    double filter_k, alpha_min, alpha_max;
    int filter_mode;  // 0 adaptive, 1 off, 2 volume
    int32_t *status;  // per item
    int4 *rect;
    uint32_t *area;   // tiles in the rectangle (0 unless visible)
    float4 *rec;
    float4 *cull;
    float4 *bbox;     // screen bounding box of the rho^2 <= tau region: x_lo, x_hi, y_lo, y_hi (pixels)
    uint32_t *pending;    // per item: items left to the whole-view cull, listed per workgroup of 256
    uint32_t *pending_n;  // per workgroup of 256 items: its number of listed items
};
hipError_t launch_preprocess(const PreArgs &a, hipStream_t s);

// Sorted pair values: the Gaussian index, and, when the scene has fewer than
// 2^28 Gaussians, the 8x8 quadrants of the pair's tile that the Gaussian's
// screen bounding box reaches in bits 28..31 (bit 28 + 2 qy + qx, the blend
// wave of that quadrant).  A wave skips the entries whose bit is clear: no
// pixel centre of its quadrant lies within half a pixel of the box.
constexpr int kQuadShift = 28;
constexpr uint32_t kQuadIdMask = (1u << kQuadShift) - 1u;
constexpr int64_t kQuadMaxGaussians = (int64_t)1 << kQuadShift;

// One training camera of K7: world->view rows (3x4, row-major), intrinsics,
// image size, near plane.
struct TrainCam {
    double V[12];
    double fx, fy, cx, cy, w, h, znear;
};
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, double lr, double b1, double b2,
                       double eps, double c1, double c2, hipStream_t s);
hipError_t launch_train_freq(const float *means, int64_t n, const TrainCam *cams, int ncam, float *out,
                             hipStream_t s);

// Pair emission over the batch's candidate tests, numbered by area_off (the
// exclusive scan of the rectangle areas, items + 1 entries; at most keep_cap of them,
// a multiple of 64; with more, the three kernels do nothing and the caller
// must ask for a larger pair buffer).  chunk_item (keep_cap / 64 words) holds
// the item of every 64th test (written by the scan of the areas, see
// launch_exclusive_scan); the counter stores, per chunk of 64 tests,
// the keep bits (keep_bits, keep_cap / 64 words) and their number
// (chunk_cnt); after an exclusive scan of the batch's chunks of chunk_cnt
// into kept_before (launch_exclusive_scan with count_of = &area_off[items]),
// the writer emits every kept test's pair at index
// kept_before[chunk] + (kept tests before it in the chunk).  Items must
// number below 2^32.
// subtile: count one pair per 8x8 sub-tile a kept test's box reaches (bbox)
hipError_t launch_count_pairs(const int4 *rect, const float4 *rec, const float4 *cull, const uint64_t *area_off,
                              int64_t items, const ViewDev *views, int nviews, bool tile_cull,
                              unsigned long long *tests, uint64_t *keep_bits, uint32_t *chunk_cnt,
                              const uint32_t *chunk_item, uint64_t keep_cap, const float4 *bbox, bool subtile,
                              hipStream_t s);
// quads: pack the quadrant bits of each pair (from bbox) into its value;
// subtile: write one pair per reached sub-tile, keyed by sub-tile number and
// sub-tile-centre depth (values carry no quadrant bits)
hipError_t launch_write_pairs(const int4 *rect, const float4 *rec, const float4 *cull, const uint64_t *area_off,
                              int64_t items, const ViewDev *views, int nviews, const uint64_t *keep_bits,
                              const uint32_t *chunk_item, const uint64_t *kept_before, uint64_t keep_cap,
                              uint64_t max_pairs, uint64_t *keys, uint32_t *vals, const float4 *bbox, bool quads,
                              bool tile_cull, bool subtile, hipStream_t s);
// host[0] = *a, host[1] = *b, host[3] = *note (then *note = 0; none when
// note is null), then host[2] = seq (system scope, in that order; host:
// coherent pinned memory).  One thread.
__device__ __forceinline__ void publish_words(const uint64_t *a, const uint64_t *b, uint64_t *host, uint64_t seq,
                                              uint32_t *note)
{
    host[0] = *a;
    host[1] = *b;
    if (note) host[3] = atomicExch(note, 0u);
    __threadfence_system();
    __hip_atomic_store(&host[2], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
// publish_words in a one-thread launch (instead of small copies)
hipError_t launch_publish2(const uint64_t *a, const uint64_t *b, uint64_t *host, uint64_t seq, uint32_t *note,
                           hipStream_t s);
// p[i] &= mask for i < n
hipError_t launch_and_u32(uint32_t *p, uint64_t n, uint32_t mask, hipStream_t s);
size_t scan_tmp_bytes(int64_t n);
// Exclusive scan of n counts into n + 1 offsets (the last: the total).  With
// count_of (device), only the first min(n, ceil(*count_of / 64)) counts are
// scanned (entries past them are never read) and the total is also stored
// at out[n].  With chunk_item: chunk_item[c] = the index i whose range
// [out[i], out[i + 1]) holds position 64 c, for c < cap_chunks.
hipError_t launch_exclusive_scan(const uint32_t *in, uint64_t *out /*n+1*/, int64_t n, void *tmp, hipStream_t s,
                                 const uint64_t *count_of = nullptr, uint32_t *chunk_item = nullptr,
                                 uint64_t cap_chunks = 0);

size_t sort_tmp_bytes(uint64_t n);
// Stable LSD sort by bits [begin_bit, end_bit); clear[0 .. nclear) is
// zeroed on the way (by the first pass).
hipError_t radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt, uint64_t n,
                            int begin_bit, int end_bit, void *tmp, hipStream_t s, bool *result_in_alt,
                            uint32_t *clear = nullptr, uint64_t nclear = 0);
// Phase 2 of the pair sort: the lists [ranges[2 l], ranges[2 l + 1]) of
// keys/vals sorted in place by the low word of their keys (stable).  First
// kernel: the lists of up to 512 entries; the longer ones are queued
// (queues holds 2 nlists entries, n_queued[0..2], *note and *done zero at
// entry) and noted in *note (kNoteSortMid / Large / Huge); lists longer
// than kLongList / kSortNoteList set the bits kNoteLongRoute /
// kNoteSortWide, and those longer than kSortNoteList are left to global
// passes over the whole key (the caller's).  Once every list is filed the
// kernel publishes (publish_words) pub_a, pub_b and the note with sequence
// number seq.  Then: the queued lists of the tiers whose bits `which` has
// (rest; the other buffers are scratch for lists longer than 8192 entries).
struct SortPublish {
    const uint64_t *a, *b;
    uint64_t *host;
    uint64_t seq;
};
// Tile ranking by list length class for the blend's order (lists are
// tiles): tile_key [nlists] receives rank | class << kOrderRankBits,
// class_count [kOrderClasses] (zero at entry) the class sizes, class_start
// [kOrderClasses] their starts, longest class first.  tile_key null: none.
// Classes: four per octave of length + 1 (the octave and the two bits
// below its leading one), capped.
constexpr int kOrderClasses = 64;
constexpr int kOrderRankBits = 26;
struct TileOrderScratch {
    uint32_t *tile_key, *class_count, *class_start;
};
hipError_t launch_segment_sort_first(uint64_t *keys, uint32_t *vals, uint64_t n, const uint32_t *ranges,
                                     int64_t nlists, uint32_t *queues, uint32_t *n_queued, uint32_t *note,
                                     uint32_t *done, SortPublish pub, TileOrderScratch order, hipStream_t s);
hipError_t launch_segment_sort_rest(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt,
                                    uint64_t n, const uint32_t *ranges, int64_t nlists, const uint32_t *queues,
                                    const uint32_t *n_queued, uint32_t which, hipStream_t s);
// order[0 .. ntiles): the tiles by decreasing list length class (see
// TileOrderScratch; any order within a class), so that the blend's longest
// lists are dispatched first.
hipError_t launch_tile_order(const uint32_t *tile_key, const uint32_t *class_start, int ntiles, uint32_t *order,
                             hipStream_t s);
// ranges [ntiles][2] of the sorted keys (cleared first unless `cleared`)
hipError_t launch_tile_ranges(const uint64_t *keys, uint64_t n, uint32_t *ranges, int ntiles, hipStream_t s,
                              bool cleared = false);

struct BlendArgs {
    const float4 *rec;             // per item (i * nviews + v)
    const uint32_t *vals;
    uint32_t id_mask;              // Gaussian index bits of a value (kQuadIdMask when values carry quadrant bits)
    uint32_t quad_on;              // bits forced on before the quadrant test (~kQuadIdMask when they carry none)
    const uint32_t *ranges;        // per global tile, or per 8x8 sub-tile (4 tile + quadrant) with quad_lists
    bool quad_lists;               // every quadrant wave walks its own sub-tile's list
    const ViewDev *views;
    int nviews;
    int total_tiles;
    float alpha_min, alpha_max, t_min;
    uint32_t *n_done;              // per pixel (view pix_base + y * W + x): list entries consumed
    uint32_t *n_ins;               // per pixel: contributors inserted (forward output)
    unsigned long long *counters;  // [0] evaluations, [1] contributors, [2] prefilter passes
    // backward only
    float *grad_rec;               // per item, kGradStride floats
    // slots: per (tile quadrant, contributor rank, lane) dL/dalpha and T alpha;
    // quadrant q = 4 * tile + wave owns 64 * (wave_off[q + 1] - wave_off[q])
    // slots from 64 * wave_off[q], rank-major, so a wave's 64 lanes store and
    // load one contiguous row per rank
    const uint64_t *wave_off;
    float2 *slots;
    bool rank16;                   // pass 1: every contributor rank fits 16 bits
    // forward only: tiles with longer lists are left to k_blend_long when
    // *n_long (written by k_find_long) is at most kMaxLongTiles
    uint32_t long_list;
    const uint32_t *n_long;
    // workgroup slot -> tile, tiles with longer lists first (null: slot =
    // tile); k_blend and k_grad
    const uint32_t *tile_order;
};
hipError_t launch_blend(const BlendArgs &a, int K, bool stats, bool pass1, hipStream_t s);
hipError_t launch_grad(const BlendArgs &a, hipStream_t s);
// caps[4 * tile + wave] = the largest n_ins over the quadrant's pixels;
// *max_big (zeroed beforehand) = the largest of those above 65535, if any
hipError_t launch_wave_caps(const ViewDev *views, int nviews, int total_tiles, const uint32_t *n_ins, uint32_t *caps,
                            uint32_t *max_big, hipStream_t s);
// Long tile lists: k_find_long collects tiles with more than a.long_list
// entries (n_long must be zero beforehand); launch_blend_long computes the
// per-pixel entry masks (pixmask: (pairs / 64 + tiles + 2) * 256 words;
// summary: summary_words >= ((pairs / 64 + tiles + 2) / 64 + 1) * 256, zeroed
// here) and renders those tiles with one walk per pixel (K <= 16).  grid: an
// upper bound of the number of long tiles.
hipError_t launch_find_long(const BlendArgs &a, uint32_t *long_tiles, uint32_t *n_long, hipStream_t s);
hipError_t launch_blend_long(const BlendArgs &a, int K, bool stats, const uint32_t *long_tiles, const uint32_t *n_long,
                             unsigned grid, uint64_t *pixmask, uint64_t *summary, uint64_t summary_words,
                             hipStream_t s);
// Lists longer than this are left out of the per-list phase of the pair
// sort (one workgroup each would run far below the chip's bandwidth); when
// one occurs, global passes over the whole key sort the pairs.
constexpr uint32_t kSortNoteList = 32768;
constexpr uint32_t kLongList = 4096;      // entries above which a forward tile is rendered by k_blend_long
constexpr uint32_t kMaxLongTiles = 1024;  // ... when at most this many tiles are that long
// Bits of the note the per-list sort publishes to the host.
constexpr uint32_t kNoteSortWide = 1u;    // a list longer than kSortNoteList
constexpr uint32_t kNoteLongRoute = 2u;   // a list longer than kLongList
constexpr uint32_t kNoteSortMid = 4u;     // lists queued for each of the three longer per-list sorts
constexpr uint32_t kNoteSortLarge = 8u;
constexpr uint32_t kNoteSortHuge = 16u;

struct GradOut {
    float *means, *log_scales, *quats, *logits, *sh;
};
// K6b over the Gaussians with a visible item (list: n entries, count: one
// uint32 zeroed beforehand; both caller workspace).
hipError_t launch_preprocess_bwd(const PreArgs &a, const float *grad_rec, GradOut g, uint32_t *list, uint32_t *count,
                                 hipStream_t s);
}  // namespace aaa
