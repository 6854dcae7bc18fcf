// K3: stable LSD radix sort of (uint64 key, uint32 value) pairs, 8-bit
// digits, and K4: tile ranges of the sorted keys.
//
// Each pass: (1) per-block digit histograms into a digit-major [digit][block]
// table, (2) one workgroup per digit scans its row in place (the block's
// offset within the digit) and records the digit's total, (3) a stable
// scatter, whose workgroups add the prefix of the digit totals themselves.
// A block owns 2048 consecutive keys (24 KB of LDS staging: six workgroups
// per CU; 4096 or 8192 keys per block measured slower, the longer runs per
// digit not making up for the lower occupancy); each of its four wavefronts
// ranks a contiguous quarter in
// rounds of 64 with a ballot-based match on the digit bits (lanes with equal
// digits see each other through eight ballots), so the rank of a key is the
// number of equal digits before it in its wave's segment.  The block then
// stages its pairs in LDS in digit order (wave order, then rank: stable) and
// writes each digit's run to consecutive global positions from the digit's
// global prefix, so stores coalesce.
#include "aaa_internal.h"

namespace aaa {

namespace {

constexpr int kBits = 8;
constexpr int kBins = 1 << kBits;
constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kPerBlock = kThreads * kItems;   // 2048
constexpr int kPerWave = kPerBlock / 4;        // 512

__device__ __forceinline__ uint64_t lanemask_lt()
{
    unsigned lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__global__ __launch_bounds__(kThreads) void k_hist(const uint64_t *__restrict__ keys, uint64_t n, int shift,
                                                   uint32_t *__restrict__ hist, uint32_t nblocks)
{
    __shared__ uint32_t h[4][kBins];
    const int t = threadIdx.x, wave = t >> 6;
    for (int k = t; k < 4 * kBins; k += kThreads) (&h[0][0])[k] = 0;
    __syncthreads();
    const uint64_t b0 = (uint64_t)blockIdx.x * kPerBlock;
#pragma unroll 4
    for (int k = 0; k < kItems; ++k) {
        uint64_t idx = b0 + (uint64_t)k * kThreads + t;
        if (idx < n) {
            uint32_t d = (uint32_t)(keys[idx] >> shift) & (kBins - 1);
            atomicAdd(&h[wave][d], 1u);
        }
    }
    __syncthreads();
    uint32_t s = h[0][t] + h[1][t] + h[2][t] + h[3][t];
    hist[(uint64_t)t * nblocks + blockIdx.x] = s;
}

// Row d of the [digit][block] table: exclusive prefix over the blocks, in
// place, and the row total in totals[d].  Each thread takes 8 consecutive
// entries per round (2048 per round: long rows take few rounds).
constexpr int kScanPer = 8;

__global__ __launch_bounds__(kThreads) void k_digit_scan(uint32_t *__restrict__ hist, uint32_t nblocks,
                                                         uint32_t *__restrict__ totals)
{
    __shared__ uint32_t wsum[4];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    uint32_t *row = hist + (uint64_t)blockIdx.x * nblocks;
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < nblocks; c0 += kThreads * kScanPer) {
        const uint32_t i0 = c0 + (uint32_t)t * kScanPer;
        uint32_t v[kScanPer], sum = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            v[k] = i0 + k < nblocks ? row[i0 + k] : 0u;
            sum += v[k];
        }
        uint32_t x = sum;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        uint32_t wpre = 0;
        for (int w = 0; w < wave; ++w) wpre += wsum[w];
        const uint32_t chunk = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        uint32_t run = carry + wpre + x - sum;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            if (i0 + k < nblocks) row[i0 + k] = run;
            run += v[k];
        }
        carry += chunk;
        __syncthreads();
    }
    if (t == 0) totals[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kThreads) void k_scatter(const uint64_t *__restrict__ keys_in,
                                                      const uint32_t *__restrict__ vals_in, uint64_t n, int shift,
                                                      const uint32_t *__restrict__ offsets,
                                                      const uint32_t *__restrict__ totals, uint32_t nblocks,
                                                      uint64_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out)
{
    __shared__ uint32_t cnt[4][kBins];   // per-wave digit counts, then per-wave prefixes
    __shared__ uint32_t lbase[kBins];    // block-local start of each digit
    __shared__ uint32_t wsum[4];
    __shared__ uint64_t gsum[4];
    __shared__ uint64_t gbase[kBins];    // global start of each digit for this block
    __shared__ uint64_t skey[kPerBlock];
    __shared__ uint32_t sval[kPerBlock];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    for (int k = t; k < 4 * kBins; k += kThreads) (&cnt[0][0])[k] = 0;
    __syncthreads();
    const uint64_t b0 = (uint64_t)blockIdx.x * kPerBlock;
    const uint64_t seg = b0 + (uint64_t)wave * kPerWave;
    const uint64_t lt = lanemask_lt();
    uint64_t key[kItems];
    uint32_t val[kItems], rank[kItems], dig[kItems];
    bool valid[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        uint64_t idx = seg + (uint64_t)r * 64 + lane;
        valid[r] = idx < n;
        key[r] = valid[r] ? keys_in[idx] : 0ull;
        val[r] = valid[r] ? vals_in[idx] : 0u;
        uint32_t d = (uint32_t)(key[r] >> shift) & (kBins - 1);
        dig[r] = d;
        uint64_t m = __ballot(valid[r]);
#pragma unroll
        for (int b = 0; b < kBits; ++b) {
            uint64_t bb = __ballot((d >> b) & 1u);
            m &= ((d >> b) & 1u) ? bb : ~bb;
        }
        uint32_t before = (uint32_t)__popcll(m & lt);
        uint32_t base = 0;
        if (valid[r]) base = cnt[wave][d];
        rank[r] = base + before;
        __builtin_amdgcn_wave_barrier();
        if (valid[r] && before == 0) cnt[wave][d] = base + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // digit t: prefixes over the waves, block total, global start
    uint32_t tot = 0;
    for (int w = 0; w < 4; ++w) {
        const uint32_t c = cnt[w][t];
        cnt[w][t] = tot;
        tot += c;
    }
    // exclusive scans over the 256 digits of the block totals (block-local
    // starts) and of the global digit totals (global starts)
    const uint64_t dt = totals[t];
    uint32_t x = tot;
    uint64_t gx = dt;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        const uint64_t gy = __shfl_up(gx, off);
        if (lane >= off) {
            x += y;
            gx += gy;
        }
    }
    if (lane == 63) {
        wsum[wave] = x;
        gsum[wave] = gx;
    }
    __syncthreads();
    uint32_t wpre = 0;
    uint64_t gpre = 0;
    for (int w = 0; w < wave; ++w) {
        wpre += wsum[w];
        gpre += gsum[w];
    }
    lbase[t] = wpre + x - tot;
    gbase[t] = gpre + gx - dt + offsets[(uint64_t)t * nblocks + blockIdx.x];
    __syncthreads();
    // stage the block's pairs in digit order (stable: wave order, then rank)
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        if (valid[r]) {
            const uint32_t lp = lbase[dig[r]] + cnt[wave][dig[r]] + rank[r];
            skey[lp] = key[r];
            sval[lp] = val[r];
        }
    }
    __syncthreads();
    // write runs of equal digits to consecutive global positions
    const uint32_t nloc = (uint32_t)(n - b0 < (uint64_t)kPerBlock ? n - b0 : (uint64_t)kPerBlock);
    for (uint32_t i = t; i < nloc; i += kThreads) {
        const uint64_t k = skey[i];
        const uint32_t d = (uint32_t)(k >> shift) & (kBins - 1);
        const uint64_t pos = gbase[d] + (i - lbase[d]);
        keys_out[pos] = k;
        vals_out[pos] = sval[i];
    }
}

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_ranges(const uint64_t *__restrict__ keys, uint64_t n, uint32_t *__restrict__ ranges)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t tile = (uint32_t)(keys[i] >> 32);
    if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != tile) ranges[2 * (uint64_t)tile] = (uint32_t)i;
    if (i == n - 1 || (uint32_t)(keys[i + 1] >> 32) != tile) ranges[2 * (uint64_t)tile + 1] = (uint32_t)(i + 1);
}

}  // namespace

static uint32_t sort_blocks(uint64_t n) { return (uint32_t)((n + kPerBlock - 1) / kPerBlock); }

size_t sort_tmp_bytes(uint64_t n)
{
    uint64_t nb = sort_blocks(n > 0 ? n : 1);
    uint64_t cells = nb * kBins;
    size_t b = cells * sizeof(uint32_t);
    b = (b + 255) & ~(size_t)255;
    return b + kBins * sizeof(uint32_t) + 256;
}

hipError_t radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt, uint64_t n,
                            int begin_bit, int end_bit, void *tmp, hipStream_t s, bool *result_in_alt)
{
    *result_in_alt = false;
    if (n <= 1 || end_bit <= begin_bit) return hipSuccess;
    uint32_t nb = sort_blocks(n);
    uint64_t cells = (uint64_t)nb * kBins;
    char *p = (char *)tmp;
    uint32_t *hist = (uint32_t *)p;
    uint32_t *totals = (uint32_t *)(p + ((cells * sizeof(uint32_t) + 255) & ~(size_t)255));
    uint64_t *ki = keys, *ko = keys_alt;
    uint32_t *vi = vals, *vo = vals_alt;
    for (int shift = begin_bit; shift < end_bit; shift += kBits) {
        hipLaunchKernelGGL(k_hist, dim3(nb), dim3(kThreads), 0, s, (const uint64_t *)ki, n, shift, hist, nb);
        hipLaunchKernelGGL(k_digit_scan, dim3(kBins), dim3(kThreads), 0, s, hist, nb, totals);
        hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kThreads), 0, s, (const uint64_t *)ki, (const uint32_t *)vi, n,
                           shift, (const uint32_t *)hist, (const uint32_t *)totals, nb, ko, vo);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t *tk = ki; ki = ko; ko = tk;
        uint32_t *tv = vi; vi = vo; vo = tv;
        *result_in_alt = !*result_in_alt;
    }
    return hipSuccess;
}

hipError_t launch_tile_ranges(const uint64_t *keys, uint64_t n, uint32_t *ranges, int ntiles, hipStream_t s)
{
    uint64_t m = 2ull * (uint64_t)ntiles;
    if (m) hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, ranges, m, 0u);
    if (n) hipLaunchKernelGGL(k_ranges, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, keys, n, ranges);
    return hipGetLastError();
}

}  // namespace aaa
