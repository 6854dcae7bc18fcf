// K2: tile-pair emission.  For every visible Gaussian, every tile of its
// bounding rectangle is tested in 3D (Sec. 3.4, Eq. 18); the counter keeps
// the results, a scan numbers the survivors, and the writer emits
// (tile << 32 | order key of the tile depth, Gaussian index) at each
// survivor's number.
//
// Work split: the candidate (item, rectangle tile) tests are numbered through
// an exclusive scan of the rectangle areas, and every lane takes one test
// (grid-stride), so lanes stay busy whatever the mix of rectangle sizes.  The
// last kernel of that scan also records the item of every 64th test; a
// wave's 64 tests then lie between two recorded items and each lane searches
// that bracket, held across the lanes.
//
// Pairs are written in test order (item, then tile within the rectangle):
// items occupy increasing ranges, so the stable sort breaks key ties by item,
// i.e. by Gaussian index within a view.
#include <algorithm>
#include <atomic>

#include "aaa_internal.h"

namespace aaa {

namespace {

constexpr int kEmitBlocks = 2048;  // grid of the balanced emitter (grid-stride), at most

// The candidates of tile_min_rho2 (Eq. 18) tested against thr without
// divisions: each is a ratio with a positive denominator (|r|^2 on an edge
// ray, |n|^2 on a face), compared as numerator < thr * denominator, and a
// face minimum's feasibility is taken on its point scaled by |n|^2 (the
// tolerance scales with it).
__device__ __forceinline__ bool edge_below(const TileGeom<float> &g, float dX, float dY, float thr)
{
    float r[3], w[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r[k] = g.c0[k] + dX * g.c1[k] + dY * g.c2[k];
        w[k] = g.w0[k] + dX * g.w1[k] + dY * g.w2[k];
    }
    const float l = g.l[0] + dX * g.l[1] + dY * g.l[2];
    return l > 0.0f && dot3(w, w) < thr * dot3(r, r);  // behind the camera: the apex, tested apart
}

__device__ __forceinline__ bool face_below(const TileGeom<float> &g, bool vert, float D, float s, float lo, float hi,
                                           float thr)
{
    const float *n0 = vert ? g.nx0 : g.ny0;
    const float *n1 = vert ? g.nx1 : g.ny1;
    const float *q0 = vert ? g.qx0 : g.qy0;
    const float *q1 = vert ? g.qx1 : g.qy1;
    float n[3], q[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        n[k] = n0[k] - D * n1[k];
        q[k] = q0[k] - D * q1[k];
    }
    const float nn = dot3(n, n);
    float X[3];  // |n|^2 times the face minimum in view space
#pragma unroll
    for (int k = 0; k < 3; ++k) X[k] = nn * g.muv[k] - s * q[k];
    const float o = vert ? X[1] : X[0];
    const float a = o - lo * X[2], b = hi * X[2] - o;
    const float scale = fabsf(o) + fabsf(X[2]) * (fabsf(lo) + fabsf(hi));
    const float tol = 1e-4f * scale;
    return s * s < thr * nn && a >= -tol && b >= -tol;
}

// Whether the minimum of rho^2 over the pyramid of tile (tx, ty) lies below
// tau with the keep test's slack (keep_limit).  The record parts are loaded
// as the tests need them (side offsets, then the lines for the edge rays,
// then the face geometry), so that fewer registers are live at once.
__device__ __forceinline__ bool tile_keep(const float4 *__restrict__ rec, const float4 *__restrict__ cull, int tx,
                                          int ty, const CamDev &cam)
{
    TileGeom<float> g;
    const float4 q6 = rec[6], p0 = cull[0];
    const float thr = keep_limit(q6.y);
    g.og2 = q6.z;
    g.dx0 = p0.x; g.dx1 = p0.y; g.dy0 = p0.z; g.dy1 = p0.w;
    load_line_geom(rec, g);
    const float x0 = (float)(tx * kTile), x1 = x0 + kTile, y0 = (float)(ty * kTile), y1 = y0 + kTile;
    const float dX0 = x0 - g.xa, dX1 = x1 - g.xa, dY0 = y0 - g.ya, dY1 = y1 - g.ya;
    const float sL = g.dx0 - dX0 * g.dx1, sR = g.dx0 - dX1 * g.dx1;
    const float sT = g.dy0 - dY0 * g.dy1, sB = g.dy0 - dY1 * g.dy1;
    const bool vL = sL < 0.0f, vR = sR > 0.0f, vT = sT < 0.0f, vB = sB > 0.0f;
    if (!(vL || vR || vT || vB) || g.og2 < thr) return true;  // mean inside the pyramid, or the apex
    bool below = false;
    if (vL || vT) below = edge_below(g, dX0, dY0, thr);
    if (!below && (vL || vB)) below = edge_below(g, dX0, dY1, thr);
    if (!below && (vR || vT)) below = edge_below(g, dX1, dY0, thr);
    if (!below && (vR || vB)) below = edge_below(g, dX1, dY1, thr);
    if (below) return true;
    {
        const float4 p1 = cull[1], p2 = cull[2], p3 = cull[3], p4 = cull[4], p5 = cull[5], p6 = cull[6], p7 = cull[7];
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
    // view slopes of the rectangle (one reciprocal per axis; the face test's
    // tolerance covers its rounding)
    const float ifx = __builtin_amdgcn_rcpf((float)cam.fx), ify = __builtin_amdgcn_rcpf((float)cam.fy);
    const float cx = (float)cam.cx, cy = (float)cam.cy;
    const float u0 = (x0 - cx) * ifx, u1 = (x1 - cx) * ifx, v0 = (y0 - cy) * ify, v1 = (y1 - cy) * ify;
    if (vL) below = face_below(g, true, dX0, sL, v0, v1, thr);
    if (!below && vR) below = face_below(g, true, dX1, sR, v0, v1, thr);
    if (!below && vT) below = face_below(g, false, dY0, sT, u0, u1, thr);
    if (!below && vB) below = face_below(g, false, dY1, sB, u0, u1, thr);
    return below;
}

// depth of the maximum on the line through the tile centre
__device__ __forceinline__ float tile_depth(const TileGeom<float> &g, int tx, int ty)
{
    float dX = (float)(tx * kTile + kTile / 2) - g.xa;
    float dY = (float)(ty * kTile + kTile / 2) - g.ya;
    float r[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) r[k] = g.c0[k] + dX * g.c1[k] + dY * g.c2[k];
    float l = g.l[0] + dX * g.l[1] + dY * g.l[2];
    return l / dot3(r, r);
}

// depth of the maximum on the line through the centre of 8x8 sub-tile q
// (bit 2 qy + qx) of tile (tx, ty)
__device__ __forceinline__ float subtile_depth(const TileGeom<float> &g, int tx, int ty, int q)
{
    float dX = (float)(tx * kTile + (q & 1) * 8 + 4) - g.xa;
    float dY = (float)(ty * kTile + (q >> 1) * 8 + 4) - g.ya;
    float r[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) r[k] = g.c0[k] + dX * g.c1[k] + dY * g.c2[k];
    float l = g.l[0] + dX * g.l[1] + dY * g.l[2];
    return l / dot3(r, r);
}

// Quadrants (bit 2 qy + qx) of tile (tx, ty) whose 8x8 pixel square meets
// the bounding box; pixel centres lie half a pixel inside the square.
__device__ __forceinline__ uint32_t quad_bits(float4 box, int tx, int ty)
{
    uint32_t m = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float x0 = (float)(tx * kTile + (q & 1) * 8), y0 = (float)(ty * kTile + (q >> 1) * 8);
        const bool meets = box.x <= x0 + 8.0f && box.y >= x0 && box.z <= y0 + 8.0f && box.w >= y0;
        m |= meets ? 1u << q : 0u;
    }
    return m;
}

__device__ __forceinline__ uint64_t bits_below(int lane) { return lane == 0 ? 0ull : (~0ull >> (64 - lane)); }

// exclusive prefix sum over the lanes of the wave
__device__ __forceinline__ uint32_t wave_exclusive_sum(uint32_t v) { return wave_incl_sum(v) - v; }

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src)
{
    const int lo = __shfl((int)(uint32_t)v, src), hi = __shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}


// Pass 1 (count) and pass 2 (write) share one body.  Items are (Gaussian,
// view) pairs, item = i * nviews + v.  The candidate tests come in chunks of
// 64, one chunk per wave step; chunk_item holds the item of each chunk's
// first test, so a lane finds its item in a bracket held across the wave.
// The counter stores each chunk's 64 results (keep_bits) and their number
// (chunk_cnt); an exclusive scan of the numbers (kept_before) gives every
// kept test its pair slot: the number of kept tests before it.  Slots thus
// follow test order (item, then tile within the rectangle), with no atomics.
// Both passes do nothing when the batch has more than keep_cap tests (the
// host reports that as a pair overflow, asking for a larger pair buffer).
//
// With `subtile` (the middle level of the hierarchical sort) a kept test
// emits one pair per 8x8 sub-tile of its tile that the item's bounding box
// reaches (all four in the ablation without tile culling), keyed by the
// sub-tile number 4 tile + q and the depth on the sub-tile-centre line, so
// that the global sort leaves every sub-tile an exact depth-ordered list of
// its own; the counts and slots then count pairs, not tests.
// (The writer is compiled for eight waves per SIMD: its code then keeps
// fewer scalar registers and runs 29% faster on the 3M view; the counter
// needs its 76 registers.)
template <bool WRITE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WRITE ? 8 : 1))) void k_pairs(const int4 *__restrict__ rects, const float4 *__restrict__ recs,
                                               const float4 *__restrict__ culls, const uint64_t *__restrict__ area_off,
                                               int64_t nitems, const ViewDev *__restrict__ views, int nviews,
                                               bool tile_cull, unsigned long long *__restrict__ tests,
                                               uint64_t *__restrict__ keep_bits, uint32_t *__restrict__ chunk_cnt,
                                               const uint32_t *__restrict__ chunk_item,
                                               const uint64_t *__restrict__ kept_before, uint64_t keep_cap,
                                               uint64_t max_pairs, uint64_t *__restrict__ keys,
                                               uint32_t *__restrict__ vals, const float4 *__restrict__ bbox, bool quads,
                                               bool subtile)
{
    const uint64_t C = area_off[nitems];  // candidate tests of the whole batch
    if (C > keep_cap) return;
    const int lane = (int)__lane_id();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long n_first = 0, n_tests = 0;
    for (uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); t0 < C; t0 += stride) {
        const uint64_t c = t0 >> 6;
        uint64_t kall = 0;
        if (WRITE) {
            kall = keep_bits[c];
            if (kall == 0) continue;  // uniform: no test of this chunk was kept
        }
        const uint64_t t = t0 + (uint64_t)lane;
        const bool valid = t < C;
        const uint64_t tq = valid ? t : C - 1;
        // this lane's item: the largest g with area_off[g] <= tq (its area is
        // then > 0), between the first items of this chunk and the next
        const int64_t g_lo = (int64_t)chunk_item[c];
        const int64_t g_hi = t0 + 64 < C ? (int64_t)chunk_item[c + 1] : nitems - 1;
        int64_t g;
        if (g_hi - g_lo < 64) {
            // bracket held across the lanes: lane k has area_off[g_lo + k]
            const int64_t span = g_hi - g_lo + 1;
            const uint64_t mine = lane < span ? area_off[g_lo + lane] : ~0ull;
            int k = 0;
            for (int half = 32; half >= 1; half >>= 1) {
                const int q = k + half < 64 ? k + half : 63;
                const uint64_t x = shfl_u64(mine, q);
                if (k + half < span && x <= tq) k += half;
            }
            g = g_lo + k;
        } else {
            // many empty items in between: binary search of the bracket
            int64_t lo = g_lo, hi = g_hi;
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo + 1) / 2;
                if (area_off[mid] <= tq)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            g = lo;
        }
        const uint64_t g0 = area_off[g];
        const int j = (int)(tq - g0);
        const int4 r = rects[g];
        const int w = r.y - r.x;
        const int tx = r.x + j % w, ty = r.z + j / w;
        const ViewDev &vw = views[g % nviews];
        TileGeom<float> geo;
        if (!WRITE) {
            const bool keep = valid && (!tile_cull || tile_keep(recs + (size_t)g * kRecQuads,
                                                                culls + (size_t)g * kCullQuads, tx, ty, vw.cam));
            kall = __ballot(keep);
            uint32_t cnt = (uint32_t)__popcll(kall);
            if (subtile) {
                const uint32_t qb = keep ? (tile_cull ? quad_bits(bbox[g], tx, ty) : 15u) : 0u;
                cnt = __popc(qb) + wave_exclusive_sum(__popc(qb));
                cnt = (uint32_t)__shfl((int)cnt, 63);  // the wave's total
            }
            if (lane == 0) {
                keep_bits[c] = kall;
                chunk_cnt[c] = cnt;
            }
            n_tests += valid ? 1 : 0;
            n_first += (valid && j == 0) ? 1 : 0;
        } else if (subtile) {
            const bool kept = valid && ((kall >> lane) & 1ull);
            const uint32_t qb = kept ? (tile_cull ? quad_bits(bbox[g], tx, ty) : 15u) : 0u;
            uint64_t slot = kept_before[c] + wave_exclusive_sum(__popc(qb));
            if (kept) {
                load_line_geom(recs + (size_t)g * kRecQuads, geo);
                const uint32_t tile = (uint32_t)(vw.tile_base + ty * vw.cam.tiles_x + tx);
                for (int q = 0; q < 4; ++q) {
                    if (!((qb >> q) & 1u)) continue;
                    if (slot < max_pairs) {
                        keys[slot] = ((uint64_t)(4 * tile + q) << 32) | order_key(subtile_depth(geo, tx, ty, q));
                        vals[slot] = (uint32_t)(g / nviews);
                    }
                    ++slot;
                }
            }
        } else {
            if (valid && ((kall >> lane) & 1ull)) {
                const uint64_t slot = kept_before[c] + (uint64_t)__popcll(kall & bits_below(lane));
                if (slot < max_pairs) {
                    load_line_geom(recs + (size_t)g * kRecQuads, geo);
                    const uint32_t tile = (uint32_t)(vw.tile_base + ty * vw.cam.tiles_x + tx);
                    keys[slot] = ((uint64_t)tile << 32) | order_key(tile_depth(geo, tx, ty));
                    uint32_t val = (uint32_t)(g / nviews);
                    if (quads) val |= quad_bits(bbox[g], tx, ty) << kQuadShift;
                    vals[slot] = val;
                }
            }
        }
    }
    if (!WRITE && tests) {
        // one atomic per wave: tests[0] += visible items, tests[1] += tile tests
        for (int off = 32; off > 0; off >>= 1) {
            n_tests += __shfl_down(n_tests, off);
            n_first += __shfl_down(n_first, off);
        }
        if (lane == 0) {
            if (n_first) atomicAdd(&tests[0], n_first);
            if (n_tests) atomicAdd(&tests[1], n_tests);
        }
    }
}

// ---------------------------------------------------------------- scan
// Exclusive scan of uint32 counts into uint64 offsets (n + 1 entries; the
// last one is the total).  Three passes: block sums, scan of the block sums
// in one block, block-local scans plus the block prefix.
constexpr int kScanBlock = 1024;  // elements per block (256 threads x 4)

__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t *smem, uint64_t &total)
{
    // smem: 256 entries
    const int t = threadIdx.x;
    const int lane = __lane_id(), wave = t >> 6;
    const uint64_t x = wave_incl_sum64(v);
    if (lane == 63) smem[wave] = x;
    __syncthreads();
    uint64_t wpre = 0;
    for (int w = 0; w < wave; ++w) wpre += smem[w];
    total = smem[0] + smem[1] + smem[2] + smem[3];
    __syncthreads();
    return wpre + x - v;
}

// The element count n is the host's, or, when count_of is given, taken on
// the device as min(n, ceil(*count_of / 64)): a scan over the 64-test chunks
// of a batch whose test count only the device knows.  The total goes to
// out[n] and, for the device-side count, also to out[n_host].
__device__ __forceinline__ int64_t scan_len(int64_t n, const uint64_t *count_of)
{
    if (!count_of) return n;
    const int64_t m = (int64_t)((*count_of + 63) >> 6);
    return m < n ? m : n;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t *__restrict__ in, int64_t n_host,
                                                     const uint64_t *__restrict__ count_of, uint64_t *__restrict__ sums)
{
    __shared__ uint64_t sm[4];
    const int64_t n = scan_len(n_host, count_of);
    const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
    if (b0 >= n) return;  // uniform per block
    uint64_t acc = 0;
    for (int k = 0; k < 4; ++k) {
        int64_t idx = b0 + threadIdx.x * 4 + k;
        if (idx < n) acc += in[idx];
    }
    uint64_t tot;
    block_exclusive_scan(acc, sm, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_sums(uint64_t *__restrict__ sums, int64_t n_host,
                                                   const uint64_t *__restrict__ count_of)
{
    __shared__ uint64_t sm[4];
    __shared__ uint64_t carry;
    const int64_t nb = (scan_len(n_host, count_of) + kScanBlock - 1) / kScanBlock;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += 256) {
        int64_t idx = c0 + threadIdx.x;
        uint64_t v = idx < nb ? sums[idx] : 0;
        uint64_t tot;
        uint64_t ex = block_exclusive_scan(v, sm, tot);
        uint64_t cr = carry;
        if (idx < nb) sums[idx] = cr + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry = cr + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

// With chunk_item: chunk_item[c] = the element whose range [out[i],
// out[i + 1]) holds position 64 c, for the chunks below cap_chunks (every
// element writes the chunks that start inside its range).
__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t *__restrict__ in, int64_t n_host,
                                                    const uint64_t *__restrict__ count_of,
                                                    const uint64_t *__restrict__ sums, uint64_t *__restrict__ out,
                                                    uint32_t *__restrict__ chunk_item, uint64_t cap_chunks)
{
    __shared__ uint64_t sm[4];
    const int64_t n = scan_len(n_host, count_of);
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        out[n] = sums[nb];
        out[n_host] = sums[nb];
    }
    const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
    if (b0 >= n) return;  // uniform per block
    uint32_t v[4];
    uint64_t acc = 0;
    for (int k = 0; k < 4; ++k) {
        int64_t idx = b0 + threadIdx.x * 4 + k;
        v[k] = idx < n ? in[idx] : 0u;
        acc += v[k];
    }
    uint64_t tot;
    uint64_t ex = block_exclusive_scan(acc, sm, tot) + sums[blockIdx.x];
    for (int k = 0; k < 4; ++k) {
        int64_t idx = b0 + threadIdx.x * 4 + k;
        if (idx < n) {
            out[idx] = ex;
            if (chunk_item && v[k]) {
                const uint64_t c1 = (ex + v[k] - 1) >> 6;
                for (uint64_t c = (ex + 63) >> 6; c <= c1 && c < cap_chunks; ++c) chunk_item[c] = (uint32_t)idx;
            }
        }
        ex += v[k];
    }
}

}  // namespace

// Grid of a grid-stride emitter kernel: the workgroups the device holds at
// once (no second, late round of workgroups), at most kEmitBlocks.
template <typename K>
static unsigned resident_blocks(K kernel)
{
    static std::atomic<unsigned> cached[16];  // per device (0: not yet known)
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= 16) return kEmitBlocks;
    unsigned nb = cached[d].load(std::memory_order_relaxed);
    if (nb == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess || per_cu <= 0 ||
            cus <= 0)
            return kEmitBlocks;
        nb = (unsigned)std::min<int64_t>((int64_t)per_cu * cus, kEmitBlocks);
        cached[d].store(nb, std::memory_order_relaxed);
    }
    return nb;
}

hipError_t launch_count_pairs(const int4 *rect, const float4 *rec, const float4 *cull, const uint64_t *area_off,
                              int64_t items, const ViewDev *views, int nviews, bool tile_cull,
                              unsigned long long *tests, uint64_t *keep_bits, uint32_t *chunk_cnt,
                              const uint32_t *chunk_item, uint64_t keep_cap, const float4 *bbox, bool subtile,
                              hipStream_t s)
{
    if (items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pairs<false>, dim3(resident_blocks(k_pairs<false>)), dim3(256), 0, s, rect, rec, cull,
                       area_off, items, views,
                       nviews, tile_cull, tests, keep_bits, chunk_cnt, chunk_item, (const uint64_t *)nullptr, keep_cap,
                       (uint64_t)0, (uint64_t *)nullptr, (uint32_t *)nullptr, bbox, false, subtile);
    return hipGetLastError();
}

hipError_t launch_write_pairs(const int4 *rect, const float4 *rec, const float4 *cull, const uint64_t *area_off,
                              int64_t items, const ViewDev *views, int nviews, const uint64_t *keep_bits,
                              const uint32_t *chunk_item, const uint64_t *kept_before, uint64_t keep_cap,
                              uint64_t max_pairs, uint64_t *keys, uint32_t *vals, const float4 *bbox, bool quads,
                              bool tile_cull, bool subtile, hipStream_t s)
{
    if (items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pairs<true>, dim3(kEmitBlocks), dim3(256), 0, s, rect, rec, cull, area_off, items, views,
                       nviews, tile_cull, (unsigned long long *)nullptr, const_cast<uint64_t *>(keep_bits),
                       (uint32_t *)nullptr, chunk_item, kept_before, keep_cap, max_pairs, keys, vals, bbox, quads,
                       subtile);
    return hipGetLastError();
}

__global__ void k_publish2(const uint64_t *__restrict__ a, const uint64_t *__restrict__ b, uint64_t *host, uint64_t seq,
                           uint32_t *note)
{
    if (threadIdx.x == 0) publish_words(a, b, host, seq, note);
}

hipError_t launch_publish2(const uint64_t *a, const uint64_t *b, uint64_t *host, uint64_t seq, uint32_t *note,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_publish2, dim3(1), dim3(64), 0, s, a, b, host, seq, note);
    return hipGetLastError();
}

__global__ void k_and_u32(uint32_t *__restrict__ p, uint64_t n, uint32_t mask)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] &= mask;
}

hipError_t launch_and_u32(uint32_t *p, uint64_t n, uint32_t mask, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_and_u32, dim3((unsigned)std::min<uint64_t>((n + 255) / 256, 4096)), dim3(256), 0, s, p, n,
                       mask);
    return hipGetLastError();
}

size_t scan_tmp_bytes(int64_t n)
{
    int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    return (size_t)(nb + 1) * sizeof(uint64_t);
}

hipError_t launch_exclusive_scan(const uint32_t *in, uint64_t *out, int64_t n, void *tmp, hipStream_t s,
                                 const uint64_t *count_of, uint32_t *chunk_item, uint64_t cap_chunks)
{
    int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    uint64_t *sums = (uint64_t *)tmp;
    if (n <= 0) {
        return hipMemsetAsync(out, 0, sizeof(uint64_t), s);
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(256), 0, s, in, n, count_of, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, sums, n, count_of);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, s, in, n, count_of, (const uint64_t *)sums,
                       out, chunk_item, cap_chunks);
    return hipGetLastError();
}

}  // namespace aaa
