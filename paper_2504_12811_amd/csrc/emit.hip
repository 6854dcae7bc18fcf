// K2: tile-pair emission.  For every visible Gaussian, every tile of its
// bounding rectangle is tested in 3D (Sec. 3.4, Eq. 18); the pair counter
// counts survivors, an exclusive scan turns counts into offsets, and the
// writer emits (tile << 32 | order key of the tile depth, Gaussian index) in
// Gaussian order, so that a stable sort breaks key ties by index.
//
// Work split: one lane per Gaussian for small rectangles; rectangles with
// more than kWaveRect tiles are handed to a whole wavefront, whose lanes
// stride over the tiles (ballot + popcount give the wave's count and each
// lane's write slot, preserving the row-major tile order).
#include "aaa_internal.h"

namespace aaa {

namespace {

constexpr int kWaveRect = 64;

__device__ __forceinline__ bool tile_keep(const TileGeom<float> &g, int tx, int ty, float tau, const CamDev &cam)
{
    float x0 = (float)(tx * kTile), y0 = (float)(ty * kTile);
    float m = tile_min_rho2<float>(g, x0, x0 + kTile, y0, y0 + kTile, cam);
    return keep_threshold(m, tau);
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

__device__ __forceinline__ uint64_t lane_mask_lt()
{
    unsigned lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Pass 1 (count) and pass 2 (write) share one body.
// Items are (Gaussian, view) pairs, item = i * nviews + v; pairs are emitted
// in item order, so within a view they come in Gaussian order.
template <bool WRITE>
__global__ __launch_bounds__(256) void k_pairs(const int32_t *__restrict__ status, const int4 *__restrict__ rects,
                                               const float4 *__restrict__ recs, const float4 *__restrict__ culls,
                                               int64_t nitems, const ViewDev *__restrict__ views, int nviews,
                                               bool tile_cull, uint32_t *__restrict__ counts,
                                               unsigned long long *__restrict__ tests, const uint64_t *__restrict__ offsets,
                                               uint64_t max_pairs, uint64_t *__restrict__ keys,
                                               uint32_t *__restrict__ vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = nitems;
    const bool live = i < n && status[i] == kVisible;
    int4 rc = live ? rects[i] : make_int4(0, 0, 0, 0);
    const int rw = rc.y - rc.x, rh = rc.w - rc.z;
    const int area = rw * rh;
    const bool big = live && area > kWaveRect;
    uint32_t my_count = 0;
    uint64_t base = 0;
    if (WRITE && live) base = offsets[i];
    unsigned long long ntests = 0;
    // small rectangles: one lane each
    if (live && !big) {
        const ViewDev &vw = views[i % nviews];
        const CamDev &cam = vw.cam;
        TileGeom<float> g;
        load_tile_geom(recs + (size_t)i * kRecQuads, culls + (size_t)i * kCullQuads, g);
        const float tau = recs[(size_t)i * kRecQuads + 6].y;
        for (int ty = rc.z; ty < rc.w; ++ty)
            for (int tx = rc.x; tx < rc.y; ++tx) {
                ++ntests;
                if (!tile_cull || tile_keep(g, tx, ty, tau, cam)) {
                    if (WRITE) {
                        uint64_t slot = base + my_count;
                        if (slot < max_pairs) {
                            uint32_t tile = (uint32_t)(vw.tile_base + ty * cam.tiles_x + tx);
                            keys[slot] = ((uint64_t)tile << 32) | order_key(tile_depth(g, tx, ty));
                            vals[slot] = (uint32_t)(i / nviews);
                        }
                    }
                    ++my_count;
                }
            }
        if (!WRITE) counts[i] = my_count;
    }
    // big rectangles: the whole wave walks each one in turn
    uint64_t bigmask = __ballot(big);
    while (bigmask) {
        const int src = __ffsll((unsigned long long)bigmask) - 1;
        bigmask &= bigmask - 1;
        const int64_t j = __shfl(i, src);
        const int4 r = make_int4(__shfl(rc.x, src), __shfl(rc.y, src), __shfl(rc.z, src), __shfl(rc.w, src));
        const uint64_t jbase = WRITE ? (uint64_t)__shfl((long long)base, src) : 0ull;
        const ViewDev &vw = views[j % nviews];
        const CamDev &cam = vw.cam;
        TileGeom<float> g;
        load_tile_geom(recs + (size_t)j * kRecQuads, culls + (size_t)j * kCullQuads, g);
        const float tau = recs[(size_t)j * kRecQuads + 6].y;
        const int w = r.y - r.x;
        const int tot = w * (r.w - r.z);
        uint32_t running = 0;
        for (int t0 = 0; t0 < tot; t0 += 64) {
            const int t = t0 + (int)__lane_id();
            bool keep = false;
            int tx = 0, ty = 0;
            if (t < tot) {
                tx = r.x + t % w;
                ty = r.z + t / w;
                ++ntests;
                keep = !tile_cull || tile_keep(g, tx, ty, tau, cam);
            }
            uint64_t m = __ballot(keep);
            if (WRITE && keep) {
                uint64_t slot = jbase + running + __popcll(m & lane_mask_lt());
                if (slot < max_pairs) {
                    uint32_t tile = (uint32_t)(vw.tile_base + ty * cam.tiles_x + tx);
                    keys[slot] = ((uint64_t)tile << 32) | order_key(tile_depth(g, tx, ty));
                    vals[slot] = (uint32_t)(j / nviews);
                }
            }
            running += (uint32_t)__popcll(m);
        }
        if (!WRITE && (int)__lane_id() == src) counts[j] = running;
    }
    if (!WRITE && i < n && !live) counts[i] = 0;
    if (!WRITE && tests) {
        // one atomic per wave: tests[0] += visible Gaussians, tests[1] += tile tests
        unsigned long long v = ntests, c = live ? 1ull : 0ull;
        for (int off = 32; off > 0; off >>= 1) {
            v += __shfl_down(v, off);
            c += __shfl_down(c, off);
        }
        if (__lane_id() == 0) {
            if (c) atomicAdd(&tests[0], c);
            if (v) atomicAdd(&tests[1], v);
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
    uint64_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        uint64_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) smem[wave] = x;
    __syncthreads();
    uint64_t wpre = 0;
    for (int w = 0; w < wave; ++w) wpre += smem[w];
    total = smem[0] + smem[1] + smem[2] + smem[3];
    __syncthreads();
    return wpre + x - v;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t *__restrict__ in, int64_t n, uint64_t *__restrict__ sums)
{
    __shared__ uint64_t sm[4];
    const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
    uint64_t acc = 0;
    for (int k = 0; k < 4; ++k) {
        int64_t idx = b0 + threadIdx.x * 4 + k;
        if (idx < n) acc += in[idx];
    }
    uint64_t tot;
    block_exclusive_scan(acc, sm, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_sums(uint64_t *__restrict__ sums, int64_t nb)
{
    __shared__ uint64_t sm[4];
    __shared__ uint64_t carry;
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

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t *__restrict__ in, int64_t n,
                                                    const uint64_t *__restrict__ sums, int64_t nb,
                                                    uint64_t *__restrict__ out)
{
    __shared__ uint64_t sm[4];
    const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
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
        if (idx < n) out[idx] = ex;
        ex += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums[nb];
}

}  // namespace

hipError_t launch_count_pairs(const int32_t *status, const int4 *rect, const float4 *rec, const float4 *cull, int64_t n,
                              const ViewDev *views, int nviews, bool tile_cull, uint32_t *counts,
                              unsigned long long *tests, hipStream_t s)
{
    const int64_t items = n * nviews;
    if (items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pairs<false>, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s, status, rect, rec, cull,
                       items, views, nviews, tile_cull, counts, tests, (const uint64_t *)nullptr, (uint64_t)0,
                       (uint64_t *)nullptr, (uint32_t *)nullptr);
    return hipGetLastError();
}

hipError_t launch_write_pairs(const int32_t *status, const int4 *rect, const float4 *rec, const float4 *cull, int64_t n,
                              const ViewDev *views, int nviews, bool tile_cull, const uint64_t *offsets,
                              uint64_t max_pairs, uint64_t *keys, uint32_t *vals, hipStream_t s)
{
    const int64_t items = n * nviews;
    if (items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pairs<true>, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s, status, rect, rec, cull,
                       items, views, nviews, tile_cull, (uint32_t *)nullptr, (unsigned long long *)nullptr, offsets,
                       max_pairs, keys, vals);
    return hipGetLastError();
}

size_t scan_tmp_bytes(int64_t n)
{
    int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    return (size_t)(nb + 1) * sizeof(uint64_t);
}

hipError_t launch_exclusive_scan(const uint32_t *in, uint64_t *out, int64_t n, void *tmp, hipStream_t s)
{
    int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    uint64_t *sums = (uint64_t *)tmp;
    if (n <= 0) {
        return hipMemsetAsync(out, 0, sizeof(uint64_t), s);
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(256), 0, s, in, n, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, sums, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, s, in, n, (const uint64_t *)sums, nb, out);
    return hipGetLastError();
}

}  // namespace aaa
