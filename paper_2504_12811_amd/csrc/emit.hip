// K2: tile-pair emission.  For every visible Gaussian, every tile of its
// bounding rectangle is tested in 3D (Sec. 3.4, Eq. 18); the pair counter
// counts survivors, an exclusive scan turns counts into offsets, and the
// writer emits (tile << 32 | order key of the tile depth, Gaussian index).
//
// Work split: the candidate (item, rectangle tile) tests are numbered through
// an exclusive scan of the rectangle areas, and every lane takes one test
// (grid-stride), so lanes stay busy whatever the mix of rectangle sizes.  A
// lane finds its item in the area offsets: the wave brackets its 64
// candidates with two cooperative 64-way searches, then each lane searches
// the bracket held across the lanes.  The lanes of
// one item inside a wave form a contiguous segment; its first lane adds the
// segment's survivors to the item's count with one atomic.
//
// The writer places an item's pairs in the item's slot range [offset,
// offset + count) in whatever order its segments arrive (each segment's
// leader takes a block of slots by an atomic on the item's count, which
// runs down to 0).  Items occupy increasing ranges, so the stable sort still
// breaks key ties by item, i.e. by Gaussian index within a view; within one
// item all keys differ (one pair per tile), so the order inside its range
// does not change the sorted result.
#include <algorithm>

#include "aaa_internal.h"

namespace aaa {

namespace {

constexpr int kEmitBlocks = 2048;  // grid of the balanced emitter (grid-stride)

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

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src)
{
    const int lo = __shfl((int)(uint32_t)v, src), hi = __shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Largest g in [lo, hi] with off[g] <= target, for a wave-uniform target and
// non-decreasing off with off[lo] <= target: each round every lane probes one
// of 64 evenly spaced points and a ballot keeps the stretch between the last
// probe at or below the target and the next probe (4 rounds for 10^6 items).
__device__ __forceinline__ int64_t wave_search(const uint64_t *__restrict__ off, int64_t lo, int64_t hi,
                                               uint64_t target, int lane)
{
    while (hi > lo) {
        const int64_t step = (hi - lo + 64) / 64;
        const int64_t p = lo + (int64_t)lane * step;
        const bool le = p <= hi && off[p] <= target;
        const uint64_t b = __ballot(le);  // lanes 0..k, lane 0 probes lo
        const int k = 63 - __builtin_clzll(b);
        lo = lo + (int64_t)k * step;
        hi = lo + step - 1 < hi ? lo + step - 1 : hi;
        if (step == 1) break;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_zero_u32(uint32_t *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Pass 1 (count) and pass 2 (write) share one body.  Items are (Gaussian,
// view) pairs, item = i * nviews + v.
template <bool WRITE>
__global__ __launch_bounds__(256) void k_pairs(const int4 *__restrict__ rects, const float4 *__restrict__ recs,
                                               const float4 *__restrict__ culls, const uint64_t *__restrict__ area_off,
                                               int64_t nitems, const ViewDev *__restrict__ views, int nviews,
                                               bool tile_cull, uint32_t *__restrict__ counts,
                                               unsigned long long *__restrict__ tests,
                                               const uint64_t *__restrict__ offsets, uint64_t max_pairs,
                                               uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                               const float4 *__restrict__ bbox, bool quads,
                                               uint64_t *__restrict__ keep_bits, const uint32_t *__restrict__ chunk_item,
                                               uint64_t keep_cap)
{
    const uint64_t C = area_off[nitems];  // candidate tests of the whole batch
    // When the batch has at most keep_cap tests, chunk_item gives the item of
    // each wave's first test (no search), and the counter leaves each wave's
    // 64 test results in keep_bits for the writer (no second test).
    const bool bits = keep_bits != nullptr && C <= keep_cap;
    const int lane = (int)__lane_id();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long n_first = 0, n_tests = 0;
    for (uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); t0 < C; t0 += stride) {
        const uint64_t t = t0 + (uint64_t)lane;
        const bool valid = t < C;
        const uint64_t tq = valid ? t : C - 1;
        // this lane's item: the largest g with area_off[g] <= tq (its area is
        // then > 0).  The wave first brackets its 64 candidates with two
        // 64-way searches, then each lane searches the bracket.
        const uint64_t t_last = t0 + 63 < C ? t0 + 63 : C - 1;
        int64_t g_lo, g_hi;
        if (bits) {
            // the next chunk's first item bounds this chunk's last one
            g_lo = (int64_t)chunk_item[t0 >> 6];
            g_hi = t0 + 64 < C ? (int64_t)chunk_item[(t0 >> 6) + 1] : nitems - 1;
        } else {
            g_lo = wave_search(area_off, 0, nitems - 1, t0, lane);
            g_hi = wave_search(area_off, g_lo, nitems - 1, t_last, lane);
        }
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
        const uint64_t g0 = area_off[g], g1 = area_off[g + 1];
        const int j = (int)(tq - g0);
        const int4 r = rects[g];
        const int w = r.y - r.x;
        const int tx = r.x + j % w, ty = r.z + j / w;
        const ViewDev &vw = views[g % nviews];
        TileGeom<float> geo;
        bool keep;
        if (WRITE && bits) {
            keep = valid && ((keep_bits[t0 >> 6] >> lane) & 1ull);
            if (keep) load_line_geom(recs + (size_t)g * kRecQuads, geo);
        } else {
            load_tile_geom(recs + (size_t)g * kRecQuads, culls + (size_t)g * kCullQuads, geo);
            const float tau = recs[(size_t)g * kRecQuads + 6].y;
            keep = valid && (!tile_cull || tile_keep(geo, tx, ty, tau, vw.cam));
        }
        // this item's lanes in the wave: [s0, s1)
        const int s0 = g0 > t0 ? (int)(g0 - t0) : 0;
        const int s1 = g1 - t0 < 64 ? (int)(g1 - t0) : 64;
        const uint64_t seg = (s1 >= 64 ? ~0ull : ((1ull << s1) - 1ull)) & ~bits_below(s0);
        const uint64_t kall = __ballot(keep);
        const uint64_t km = kall & seg;
        const uint32_t nk = (uint32_t)__popcll(km);
        if (!WRITE) {
            if (bits && lane == 0) keep_bits[t0 >> 6] = kall;
            if (valid && lane == s0 && nk) atomicAdd(&counts[g], nk);
            n_tests += valid ? 1 : 0;
            n_first += (valid && j == 0) ? 1 : 0;
        } else {
            uint32_t base = 0;
            if (valid && lane == s0 && nk) base = atomicSub(&counts[g], nk) - nk;
            base = (uint32_t)__shfl((int)base, s0);
            if (keep) {
                const uint64_t slot = offsets[g] + base + (uint64_t)__popcll(km & bits_below(lane));
                if (slot < max_pairs) {
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

// chunk_item[c] = the item holding candidate test 64 c, for the chunks below
// cap_chunks: every item with tests writes the chunks that start inside its
// range [area_off[g], area_off[g + 1]).
__global__ __launch_bounds__(256) void k_chunk_items(const uint64_t *__restrict__ area_off, int64_t nitems,
                                                     uint64_t cap_chunks, uint32_t *__restrict__ chunk_item)
{
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < nitems;
         g += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t g0 = area_off[g], g1 = area_off[g + 1];
        if (g1 <= g0) continue;
        const uint64_t c1 = (g1 - 1) >> 6;
        for (uint64_t c = (g0 + 63) >> 6; c <= c1 && c < cap_chunks; ++c) chunk_item[c] = (uint32_t)g;
    }
}

}  // namespace

hipError_t launch_chunk_items(const uint64_t *area_off, int64_t items, uint64_t keep_cap, uint32_t *chunk_item,
                              hipStream_t s)
{
    if (items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_chunk_items, dim3((unsigned)std::min<int64_t>((items + 255) / 256, 4096)), dim3(256), 0, s,
                       area_off, items, keep_cap / 64, chunk_item);
    return hipGetLastError();
}

hipError_t launch_count_pairs(const int4 *rect, const float4 *rec, const float4 *cull, const uint64_t *area_off,
                              int64_t items, const ViewDev *views, int nviews, bool tile_cull, uint32_t *counts,
                              unsigned long long *tests, uint64_t *keep_bits, const uint32_t *chunk_item, uint64_t keep_cap, hipStream_t s)
{
    if (items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)std::min<int64_t>((items + 255) / 256, 1024)), dim3(256), 0, s,
                       counts, items);
    hipLaunchKernelGGL(k_pairs<false>, dim3(kEmitBlocks), dim3(256), 0, s, rect, rec, cull, area_off, items, views,
                       nviews, tile_cull, counts, tests, (const uint64_t *)nullptr, (uint64_t)0, (uint64_t *)nullptr,
                       (uint32_t *)nullptr, (const float4 *)nullptr, false, keep_bits, chunk_item, keep_cap);
    return hipGetLastError();
}

hipError_t launch_write_pairs(const int4 *rect, const float4 *rec, const float4 *cull, const uint64_t *area_off,
                              int64_t items, const ViewDev *views, int nviews, bool tile_cull, uint32_t *counts,
                              const uint64_t *offsets, uint64_t max_pairs, uint64_t *keys, uint32_t *vals,
                              const float4 *bbox, bool quads, uint64_t *keep_bits, const uint32_t *chunk_item, uint64_t keep_cap,
                              hipStream_t s)
{
    if (items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pairs<true>, dim3(kEmitBlocks), dim3(256), 0, s, rect, rec, cull, area_off, items, views,
                       nviews, tile_cull, counts, (unsigned long long *)nullptr, offsets, max_pairs, keys, vals, bbox,
                       quads, keep_bits, chunk_item, keep_cap);
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
