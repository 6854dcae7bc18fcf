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
#include <algorithm>

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

// The lanes of the wave whose digit d (nbits <= MAXB bits, the higher ones
// zero) equals this lane's, among the lanes with `valid` set.  One ballot per
// digit bit; each lane ORs into its mask of disagreeing lanes the bit's
// ballot XOR its own bit spread over a word (0 or ~0), one three-input bit
// operation per mask half.
template <int MAXB = kBits>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid, int nbits = MAXB)
{
    const uint64_t v = __ballot(valid);
    uint32_t lo = ~(uint32_t)v, hi = ~(uint32_t)(v >> 32);
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        if (b < nbits) {  // uniform
            uint32_t own;  // bit b of d spread over the word (written as one v_bfe_i32)
            asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(own) : "v"(d), "i"(b));
            const uint64_t bb = __ballot(own != 0u);
            lo = __builtin_amdgcn_bitop3_b32(lo, (uint32_t)bb, own, 0xF6);  // lo | (bb ^ own)
            hi = __builtin_amdgcn_bitop3_b32(hi, (uint32_t)(bb >> 32), own, 0xF6);
        }
    }
    return ~(((uint64_t)hi << 32) | lo);
}

__global__ __launch_bounds__(kThreads) void k_hist(const uint64_t *__restrict__ keys, uint64_t n, int shift,
                                                   int nbits, uint32_t *__restrict__ hist, uint32_t nblocks,
                                                   uint32_t *__restrict__ clear, uint64_t nclear)
{
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < nclear; i += (uint64_t)gridDim.x * kThreads)
        clear[i] = 0u;
    __shared__ uint32_t h[4][kBins];
    const int t = threadIdx.x, wave = t >> 6;
    for (int k = t; k < 4 * kBins; k += kThreads) (&h[0][0])[k] = 0;
    __syncthreads();
    const uint64_t b0 = (uint64_t)blockIdx.x * kPerBlock;
#pragma unroll 4
    for (int k = 0; k < kItems; ++k) {
        uint64_t idx = b0 + (uint64_t)k * kThreads + t;
        if (idx < n) {
            uint32_t d = (uint32_t)(keys[idx] >> shift) & ((1u << nbits) - 1u);
            atomicAdd(&h[wave][d], 1u);
        }
    }
    __syncthreads();
    uint32_t s = h[0][t] + h[1][t] + h[2][t] + h[3][t];
    if (t < (1 << nbits)) hist[(uint64_t)t * nblocks + blockIdx.x] = s;
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
        const uint32_t x = wave_incl_sum(sum);
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
                                                      int nbits, const uint32_t *__restrict__ offsets,
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
        uint32_t d = (uint32_t)(key[r] >> shift) & ((1u << nbits) - 1u);
        dig[r] = d;
        const uint64_t m = match_digit(d, valid[r], nbits);
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
    const bool live = t < (1 << nbits);  // digits past 2^nbits are empty
    const uint64_t dt = live ? totals[t] : 0u;
    const uint32_t x = wave_incl_sum(tot);
    const uint64_t gx = wave_incl_sum64(dt);
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
    gbase[t] = gpre + gx - dt + (live ? offsets[(uint64_t)t * nblocks + blockIdx.x] : 0u);
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
        const uint32_t d = (uint32_t)(k >> shift) & ((1u << nbits) - 1u);
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


// --------------------------------------------------------- segment sort
//
// Second phase of the pair sort.  The LSD passes over the high word of the
// keys (the list number) leave every list a contiguous run in pair-writing
// order; each run is then sorted by the low word (the depth key), stably,
// which gives the order of a full LSD sort of the 64-bit keys.  One
// workgroup per list:
//  - k_seg_first (1 wave): runs of 2..kSegWave entries, in registers and
//    LDS; longer runs are queued for
//  - k_seg_mid (4 waves): runs up to kSegSmall entries the same way,
//  - k_seg_large (16 waves): runs up to kSegLarge entries the same way, or
//  - k_seg_huge (16 waves): longer runs by 8-bit LSD passes over the run in
//    global memory (the other pair buffer holds the intermediate order), in
//    chunks of kSegLarge.
// Entries sit in registers, kSegItems per thread: wave w holds entries
// w S + 64 r + lane (r < S / 64) of the run or chunk, so that wave order,
// then round, then lane is entry order.  A pass ranks each entry among the
// equal digits of its wave (ballot match, as in k_scatter), scans the
// per-wave digit counts in (digit, wave) order and moves the entries
// through LDS to their new places.  The depth words are sorted as offsets
// from the run's minimum, so only the passes that the span of the run's
// words needs are made; a pass whose digit is the same for every entry of
// the run moves nothing.

constexpr int kSegItems = 8;
constexpr int kSegWave = 64 * kSegItems;         // 512
constexpr int kSegSmall = 4 * 64 * kSegItems;    // 2048
constexpr int kSegLarge = 16 * 64 * kSegItems;   // 8192

// Counts and digit starts fit 16 bits (at most 512 entries per wave and
// 16 * 512 per run or chunk), which keeps the 16-wave form at two
// workgroups per CU.  Digits of up to kB bits (9-bit digits for one and four
// waves, a 25-27-bit span in three passes instead of four, measured slower).
// With one wave these words are not needed (ballots instead), which keeps
// the one-wave form at 5 KB (eight workgroups per SIMD).
template <int W>
struct SegExtra {
    uint32_t skip[4];         // per pass: one digit holds the whole run (set once, never reset)
    uint32_t red[2][W];       // per-wave minimum and maximum of the depth words
};
template <>
struct SegExtra<1> {};

template <int W>
struct SegShared : SegExtra<W> {
    static constexpr int kB = 8;
    static constexpr int kNB = 1 << kB;
    alignas(16) uint16_t cnt[W][kNB];   // per-wave digit counts, then per-wave prefixes
    alignas(16) uint16_t lbase[kNB];    // start of each digit in the run or chunk
    uint32_t key[W * 64 * kSegItems];
    uint32_t val[W * 64 * kSegItems];
};

// Width of pass `pass` of `passes` over `bits` bits: (nearly) equal digits.
__device__ __forceinline__ int digit_bits(int bits, int passes, int pass)
{
    const int done = (bits * pass) / passes;
    return (bits * (pass + 1)) / passes - done;
}

// Rank the wave's valid entries (e < m) by their digit of nbits bits at
// `shift`; per-wave counts in sh.cnt[wave].  Returns digit | rank << 16 in
// dr[] (ranks below 2^13).
template <int W>
__device__ __forceinline__ void seg_rank(SegShared<W> &sh, const uint32_t (&k)[kSegItems], uint32_t e0, uint32_t m,
                                         int shift, int nbits, int rounds, uint32_t (&dr)[kSegItems])
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t lt = lanemask_lt();
    const uint32_t mask = (1u << nbits) - 1u;
#pragma unroll
    for (int r = 0; r < kSegItems; ++r) {
        if (r < rounds) {
            const bool valid = e0 + (uint32_t)(r * 64 + lane) < m;
            const uint32_t dg = (k[r] >> shift) & mask;
            const uint64_t mm = match_digit<SegShared<W>::kB>(dg, valid, nbits);
            const uint32_t before = (uint32_t)__popcll(mm & lt);
            uint32_t base = 0;
            if (valid) base = sh.cnt[wave][dg];
            dr[r] = dg | ((base + before) << 16);
            __builtin_amdgcn_wave_barrier();
            if (valid && before == 0) sh.cnt[wave][dg] = (uint16_t)(base + (uint32_t)__popcll(mm));
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// Lane l of the first wave owns digits P l .. P l + P - 1 (P = bins / 64):
// per-wave prefixes in sh.cnt, exclusive digit starts in sh.lbase (a
// lane-local prefix, then one scan over the wave).  Whether one digit holds
// all m entries: *flag set (if given) before the closing barrier, and, on the
// first wave, returned for the lane's digits.
template <int W>
__device__ __forceinline__ bool seg_scan(SegShared<W> &sh, uint32_t m, uint32_t *flag)
{
    bool one = false;
    constexpr int P = SegShared<W>::kNB / 64, WORDS = P / 2;
    const int t = threadIdx.x;
    if (t < 64) {
        uint32_t tot[P];
#pragma unroll
        for (int j = 0; j < P; ++j) tot[j] = 0u;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            uint32_t c[WORDS], o[WORDS];
            uint32_t *row = (uint32_t *)&sh.cnt[w][P * t];
#pragma unroll
            for (int j = 0; j < WORDS; ++j) o[j] = tot[2 * j] | (tot[2 * j + 1] << 16);
            if constexpr (WORDS == 2) {
                const uint2 x = *(uint2 *)row;
                *(uint2 *)row = make_uint2(o[0], o[1]);
                c[0] = x.x; c[1] = x.y;
            } else {
                const uint4 x = *(uint4 *)row;
                *(uint4 *)row = make_uint4(o[0], o[1], o[2], o[3]);
                c[0] = x.x; c[1] = x.y; c[2] = x.z; c[3] = x.w;
            }
#pragma unroll
            for (int j = 0; j < WORDS; ++j) {
                tot[2 * j] += c[j] & 0xffffu;
                tot[2 * j + 1] += c[j] >> 16;
            }
        }
        uint32_t mine = 0u;
#pragma unroll
        for (int j = 0; j < P; ++j) {
            one = one || tot[j] == m;
            mine += tot[j];
        }
        if (flag && one) *flag = 1u;
        const uint32_t x = wave_incl_sum(mine);
        uint32_t run = x - mine, lb[WORDS];
#pragma unroll
        for (int j = 0; j < WORDS; ++j) {
            lb[j] = run | ((run + tot[2 * j]) << 16);
            run += tot[2 * j] + tot[2 * j + 1];
        }
        uint32_t *lrow = (uint32_t *)&sh.lbase[P * t];
        if constexpr (WORDS == 2)
            *(uint2 *)lrow = make_uint2(lb[0], lb[1]);
        else
            *(uint4 *)lrow = make_uint4(lb[0], lb[1], lb[2], lb[3]);
    }
    __syncthreads();
    return one;
}

// One in-LDS pass (number `pass`) over m <= W * 512 register-resident
// entries, by their digit of nbits bits at `shift`.
template <int W>
__device__ __forceinline__ void seg_pass(SegShared<W> &sh, uint32_t (&k)[kSegItems], uint32_t (&v)[kSegItems],
                                         uint32_t m, int shift, int nbits, int pass, uint32_t S)
{
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int rounds = (int)(S / 64);
    const uint32_t e0 = (uint32_t)wave * S;
    for (int i = t; i < W * SegShared<W>::kNB / 2; i += W * 64) ((uint32_t *)&sh.cnt[0][0])[i] = 0u;
    __syncthreads();
    uint32_t dr[kSegItems];
#pragma unroll
    for (int r = 0; r < kSegItems; ++r) asm("" : "=v"(dr[r]));  // rounds past `rounds` keep whatever is there
    seg_rank<W>(sh, k, e0, m, shift, nbits, rounds, dr);
    __syncthreads();
    // a pass whose digit is the same for every entry moves nothing
    if constexpr (W == 1) {
        if (__ballot(seg_scan<W>(sh, m, nullptr)) != 0ull) return;
    } else {
        (void)seg_scan<W>(sh, m, &sh.skip[pass]);
        if (sh.skip[pass]) return;  // uniform
    }
#pragma unroll
    for (int r = 0; r < kSegItems; ++r) {
        if (r < rounds && e0 + (uint32_t)(r * 64 + lane) < m) {
            const uint32_t dg = dr[r] & 0xffffu;
            const uint32_t pos = sh.lbase[dg] + sh.cnt[wave][dg] + (dr[r] >> 16);
            sh.key[pos] = k[r];
            sh.val[pos] = v[r];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSegItems; ++r) {
        const uint32_t e = e0 + (uint32_t)(r * 64 + lane);
        if (r < rounds && e < m) {
            k[r] = sh.key[e];
            v[r] = sh.val[e];
        }
    }
    __syncthreads();
}

// Minimum and maximum of the workgroup's mn / mx (uniform results; one
// barrier when W > 1).
template <int W>
__device__ __forceinline__ void seg_minmax(SegShared<W> &sh, uint32_t &mn, uint32_t &mx)
{
    wave_minmax(mn, mx);
    if constexpr (W > 1) {
        const int wave = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            sh.red[0][wave] = mn;
            sh.red[1][wave] = mx;
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < W; ++w) {
            mn = min(mn, sh.red[0][w]);
            mx = max(mx, sh.red[1][w]);
        }
    }
}

// Sort a run of m <= W * 512 entries at keys/vals + start in place.  The
// depth words are sorted as offsets from the run's minimum, over the bits
// their span needs (a run whose words are all equal is already in order).
template <int W>
__device__ __forceinline__ void seg_sort_lds(SegShared<W> &sh, uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                             uint64_t start, uint32_t m, uint64_t hi)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // per-wave segment: a multiple of 64, at most 512
    const uint32_t S = ((m + W * 64 - 1) / (W * 64)) * 64;
    const uint32_t e0 = (uint32_t)wave * S;
    if constexpr (W > 1) {
        if (threadIdx.x < 4) sh.skip[threadIdx.x] = 0u;  // ordered by the first pass's barrier
    }
    uint32_t k[kSegItems], v[kSegItems];
    uint32_t mn = ~0u, mx = 0u;
#pragma unroll
    for (int r = 0; r < kSegItems; ++r) {
        const uint32_t e = e0 + (uint32_t)(r * 64 + lane);
        const bool ok = r * 64 < (int)S && e < m;
        k[r] = ok ? ((const uint32_t *)(keys + start + e))[0] : 0u;  // the low (depth) word
        v[r] = ok ? vals[start + e] : 0u;
        if (ok) {
            mn = min(mn, k[r]);
            mx = max(mx, k[r]);
        }
    }
    seg_minmax<W>(sh, mn, mx);
    const uint32_t span = mx - mn;
    if (span == 0u) return;
    const int bits = 32 - __clz((int)span);
#pragma unroll
    for (int r = 0; r < kSegItems; ++r) k[r] -= mn;
    const int passes = (bits + SegShared<W>::kB - 1) / SegShared<W>::kB;
    for (int pass = 0, shift = 0; pass < passes; ++pass) {
        const int nb = digit_bits(bits, passes, pass);
        seg_pass<W>(sh, k, v, m, shift, nb, pass, S);
        shift += nb;
    }
#pragma unroll
    for (int r = 0; r < kSegItems; ++r) {
        const uint32_t e = e0 + (uint32_t)(r * 64 + lane);
        if (r * 64 < (int)S && e < m) {
            keys[start + e] = hi | (k[r] + mn);
            vals[start + e] = v[r];
        }
    }
}

// Lists of 2 .. kSegWave entries, one wave each.  The first ceil(nlists /
// 64) workgroups (dispatched first) each file 64 lists that need more than
// one wave, workgroup g the lists 64 g .. 64 g + 63 (one atomic per queue for
// the 64 lists): queue_mid takes lists of
// kSegWave + 1 .. kSegSmall entries, queue_large from its front those of
// kSegSmall + 1 .. kSegLarge and from its back (queue_large[nlists - 1 - j])
// the longer ones up to kSortNoteList (the two together hold at most nlists
// lists); counts in n_queued[0..2], the bit of each tier that has lists in
// *note, with kNoteLongRoute / kNoteSortWide for lists longer than kLongList
// / kSortNoteList (the latter are left to global passes over the whole key).
// The last of these workgroups to finish publishes the note to the host.
// With `order` (lists are tiles), they also rank the tiles by length class
// (see launch_tile_order): a per-class count, then its prefix from the
// longest class down, computed by the last of them.
__global__ __launch_bounds__(64) void k_seg_first(uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                  const uint32_t *__restrict__ ranges, uint32_t nlists,
                                                  uint32_t *__restrict__ queue_mid, uint32_t *__restrict__ queue_large,
                                                  uint32_t *__restrict__ n_queued, uint32_t *note, uint32_t *done,
                                                  SortPublish pub, TileOrderScratch order)
{
    __shared__ SegShared<1> sh;
    const uint32_t list = blockIdx.x;
    if (list >= nlists) return;
    const int lane = (int)threadIdx.x;
    const uint32_t filers = (nlists + 63u) / 64u;
    if (list < filers) {
        const uint32_t l = 64u * list + (uint32_t)lane;
        uint32_t ml = 0u;
        if (l < nlists) {
            const uint32_t a = ranges[2 * l], b = ranges[2 * l + 1];
            ml = b > a ? b - a : 0u;
        }
        const uint64_t lt = lanemask_lt();
        if (order.tile_key) {
            // length class of each tile, ranked within the class
            const uint32_t v = ml + 1u, e = 31u - (uint32_t)__clz((int)v);
            const uint32_t sub = (e >= 2u ? v >> (e - 2u) : v << (2u - e)) & 3u;
            const uint32_t cl = min(4u * e + sub, (uint32_t)kOrderClasses - 1u);
            // the lanes of each class; its first lane adds the class's
            // count for all of them (one atomic instruction for every class)
            static_assert(kOrderClasses <= 64, "classes of 6 bits");
            const uint64_t m = match_digit<6>(cl, l < nlists);
            const uint32_t before = (uint32_t)__popcll(m & lt);
            uint32_t at = 0u;
            if (l < nlists && before == 0u) at = atomicAdd(&order.class_count[cl], (uint32_t)__popcll(m));
            at = (uint32_t)__shfl((int)at, l < nlists ? __ffsll((long long)m) - 1 : lane);
            if (l < nlists) order.tile_key[l] = (at + before) | (cl << kOrderRankBits);
        }
        const uint64_t huge = __ballot(ml > (uint32_t)kSegLarge && ml <= kSortNoteList);
        const uint64_t big = __ballot(ml > (uint32_t)kSegSmall && ml <= (uint32_t)kSegLarge);
        const uint64_t mid = __ballot(ml > (uint32_t)kSegWave && ml <= (uint32_t)kSegSmall);
        const uint64_t lng = __ballot(ml > kLongList);
        const uint64_t wide = __ballot(ml > kSortNoteList);
        uint32_t qh = 0u, qb = 0u, qm = 0u, last = 0u;
        if (lane == 0) {
            if (huge) qh = atomicAdd(&n_queued[2], (uint32_t)__popcll(huge));
            if (big) qb = atomicAdd(&n_queued[1], (uint32_t)__popcll(big));
            if (mid) qm = atomicAdd(&n_queued[0], (uint32_t)__popcll(mid));
            const uint32_t bits = (huge ? kNoteSortHuge : 0u) | (big ? kNoteSortLarge : 0u) |
                                  (mid ? kNoteSortMid : 0u) | (lng ? kNoteLongRoute : 0u) |
                                  (wide ? kNoteSortWide : 0u);
            if (bits) atomicOr(note, bits);
            __threadfence();
            last = atomicAdd(done, 1u) == filers - 1u;
        }
        // the last filing workgroup completes the tile order's class starts
        // (lane c: class kOrderClasses - 1 - c) and publishes the note
        if (__shfl((int)last, 0)) {
            __threadfence();
            if (order.tile_key) {
                const int c = kOrderClasses - 1 - lane;
                const uint32_t cnt = c >= 0 ? atomicAdd(&order.class_count[c], 0u) : 0u;
                const uint32_t incl = wave_incl_sum(cnt);
                if (c >= 0) order.class_start[c] = incl - cnt;
            }
            if (lane == 0) publish_words(pub.a, pub.b, pub.host, pub.seq, note);
        }
        qh = (uint32_t)__shfl((int)qh, 0);
        qb = (uint32_t)__shfl((int)qb, 0);
        qm = (uint32_t)__shfl((int)qm, 0);
        if ((huge >> lane) & 1ull) queue_large[nlists - 1u - (qh + (uint32_t)__popcll(huge & lt))] = l;
        if ((big >> lane) & 1ull) queue_large[qb + (uint32_t)__popcll(big & lt)] = l;
        if ((mid >> lane) & 1ull) queue_mid[qm + (uint32_t)__popcll(mid & lt)] = l;
    }
    const uint32_t start = ranges[2 * list], end = ranges[2 * list + 1];
    const uint32_t m = end > start ? end - start : 0u;
    if (m > (uint32_t)kSegWave || m < 2) return;
    seg_sort_lds<1>(sh, keys, vals, start, m, (uint64_t)list << 32);
}

__global__ __launch_bounds__(256) void k_seg_mid(uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                 const uint32_t *__restrict__ ranges, const uint32_t *__restrict__ queue,
                                                 const uint32_t *__restrict__ n_queued)
{
    __shared__ SegShared<4> sh;
    if (blockIdx.x >= *n_queued) return;
    const uint32_t list = queue[blockIdx.x];
    const uint32_t start = ranges[2 * list], end = ranges[2 * list + 1];
    seg_sort_lds<4>(sh, keys, vals, start, end - start, (uint64_t)list << 32);
}

// Runs longer than kSegLarge: LSD passes over the run in global memory,
// chunk after chunk (stable), ping-ponging with the other buffer; a copy
// brings the result back when an odd number of passes moved it.
__device__ void seg_sort_global(SegShared<16> &sh, uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                uint64_t *__restrict__ keys_alt, uint32_t *__restrict__ vals_alt, uint64_t start,
                                uint32_t m, uint64_t hi)
{
    constexpr int W = 16;
    __shared__ uint32_t hist[kBins], run[kBins];
    __shared__ uint32_t gbase[kBins];
    __shared__ uint32_t wsum[4];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int nthr = W * 64;
    uint64_t *ksrc = keys, *kdst = keys_alt;
    uint32_t *vsrc = vals, *vdst = vals_alt;
    int moved = 0;
    if (t < 4) sh.skip[t] = 0u;
    // depth words as offsets from the run's minimum, over the bits of their span
    // (sweeps over the run load eight entries per thread before using them)
    uint32_t mn = ~0u, mx = 0u;
    for (uint32_t e0 = t; e0 < m; e0 += 8 * nthr) {
        uint32_t kk[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t e = e0 + (uint32_t)(j * nthr);
            kk[j] = e < m ? (uint32_t)keys[start + e] : ~0u;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (e0 + (uint32_t)(j * nthr) < m) {
                mn = min(mn, kk[j]);
                mx = max(mx, kk[j]);
            }
        }
    }
    seg_minmax<W>(sh, mn, mx);
    const uint32_t span = mx - mn;
    const int bits = span ? 32 - __clz((int)span) : 0;
    const int passes = (bits + kBits - 1) / kBits;
    for (int pass = 0, shift = 0; pass < passes; shift += digit_bits(bits, passes, pass), ++pass) {
        const int nbits = digit_bits(bits, passes, pass);
        const uint32_t mask = (1u << nbits) - 1u;
        uint32_t *skip = &sh.skip[pass];
        // digit totals of the whole run
        if (t < kBins) hist[t] = 0u;
        __syncthreads();
        for (uint32_t e0 = t; e0 < m; e0 += 8 * nthr) {
            uint32_t kk[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const uint32_t e = e0 + (uint32_t)(j * nthr);
                kk[j] = e < m ? (uint32_t)ksrc[start + e] : 0u;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (e0 + (uint32_t)(j * nthr) < m) atomicAdd(&hist[((kk[j] - mn) >> shift) & mask], 1u);
        }
        __syncthreads();
        if (t < kBins) {
            const uint32_t c = hist[t];
            if (c == m) *skip = 1u;
            const uint32_t x = wave_incl_sum(c);
            if (lane == 63) wsum[t >> 6] = x;
            gbase[t] = x - c;
            run[t] = 0u;
        }
        __syncthreads();
        if (*skip) continue;  // uniform
        if (t < kBins) {
            uint32_t wpre = 0;
            for (int w = 0; w < (t >> 6); ++w) wpre += wsum[w];
            gbase[t] += wpre;
        }
        __syncthreads();
        for (uint32_t c0 = 0; c0 < m; c0 += (uint32_t)kSegLarge) {
            const uint32_t mc = m - c0 < (uint32_t)kSegLarge ? m - c0 : (uint32_t)kSegLarge;
            const uint32_t e0 = (uint32_t)wave * 512u;
            uint32_t k[kSegItems], v[kSegItems], dr[kSegItems];
#pragma unroll
            for (int r = 0; r < kSegItems; ++r) {
                const uint32_t e = e0 + (uint32_t)(r * 64 + lane);
                k[r] = e < mc ? (uint32_t)ksrc[start + c0 + e] - mn : 0u;
                v[r] = e < mc ? vsrc[start + c0 + e] : 0u;
            }
            for (int i = t; i < W * kBins / 2; i += nthr) ((uint32_t *)&sh.cnt[0][0])[i] = 0u;
            __syncthreads();
            seg_rank<W>(sh, k, e0, mc, shift, nbits, kSegItems, dr);
            __syncthreads();
            (void)seg_scan<W>(sh, mc, nullptr);
            // stage in digit order, then write each digit's run to its place
#pragma unroll
            for (int r = 0; r < kSegItems; ++r) {
                if (e0 + (uint32_t)(r * 64 + lane) < mc) {
                    const uint32_t dg = dr[r] & 0xffffu;
                    const uint32_t pos = sh.lbase[dg] + sh.cnt[wave][dg] + (dr[r] >> 16);
                    sh.key[pos] = k[r];
                    sh.val[pos] = v[r];
                }
            }
            __syncthreads();
            for (uint32_t i = t; i < mc; i += nthr) {
                const uint32_t kk = sh.key[i];
                const uint32_t dg = (kk >> shift) & mask;
                const uint64_t pos = start + gbase[dg] + run[dg] + (i - sh.lbase[dg]);
                kdst[pos] = hi | (kk + mn);
                vdst[pos] = sh.val[i];
            }
            __syncthreads();
            if (t < kBins) run[t] += (t + 1 < kBins ? (uint32_t)sh.lbase[t + 1] : mc) - sh.lbase[t];
            __syncthreads();
        }
        uint64_t *tk = ksrc; ksrc = kdst; kdst = tk;
        uint32_t *tv = vsrc; vsrc = vdst; vdst = tv;
        ++moved;
    }
    if (moved & 1) {
        for (uint32_t e = t; e < m; e += nthr) {
            keys[start + e] = keys_alt[start + e];
            vals[start + e] = vals_alt[start + e];
        }
    }
}

// Lists of kSegSmall + 1 .. kSegLarge entries: at most 64 registers, so that
// two workgroups share a CU (one sorts while the other loads or stores).
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_seg_large(
    uint64_t *__restrict__ keys, uint32_t *__restrict__ vals, const uint32_t *__restrict__ ranges,
    const uint32_t *__restrict__ queue, const uint32_t *__restrict__ n_queued)
{
    __shared__ SegShared<16> sh;
    if (blockIdx.x >= *n_queued) return;
    const uint32_t list = queue[blockIdx.x];
    const uint32_t start = ranges[2 * list], end = ranges[2 * list + 1];
    seg_sort_lds<16>(sh, keys, vals, start, end - start, (uint64_t)list << 32);
}

// Lists of kSegLarge + 1 .. kSortNoteList entries, queued from the back.
__global__ __launch_bounds__(1024) void k_seg_huge(uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                   uint64_t *__restrict__ keys_alt, uint32_t *__restrict__ vals_alt,
                                                   const uint32_t *__restrict__ ranges,
                                                   const uint32_t *__restrict__ queue_end,
                                                   const uint32_t *__restrict__ n_queued)
{
    __shared__ SegShared<16> sh;
    if (blockIdx.x >= *n_queued) return;
    const uint32_t list = queue_end[-1 - (int64_t)blockIdx.x];
    const uint32_t start = ranges[2 * list], end = ranges[2 * list + 1];
    seg_sort_global(sh, keys, vals, keys_alt, vals_alt, start, end - start, (uint64_t)list << 32);
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
                            int begin_bit, int end_bit, void *tmp, hipStream_t s, bool *result_in_alt,
                            uint32_t *clear, uint64_t nclear)
{
    *result_in_alt = false;
    if (n <= 1 || end_bit <= begin_bit) {
        if (nclear) hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((nclear + 255) / 256)), dim3(256), 0, s, clear,
                                       nclear, 0u);
        return hipGetLastError();
    }
    uint32_t nb = sort_blocks(n);
    uint64_t cells = (uint64_t)nb * kBins;
    char *p = (char *)tmp;
    uint32_t *hist = (uint32_t *)p;
    uint32_t *totals = (uint32_t *)(p + ((cells * sizeof(uint32_t) + 255) & ~(size_t)255));
    uint64_t *ki = keys, *ko = keys_alt;
    uint32_t *vi = vals, *vo = vals_alt;
    // ceil(bits / 8) passes with digits of (nearly) equal width: fewer bins
    // per pass where the bits allow (longer runs per digit in the scatter)
    const int bits = end_bit - begin_bit, passes = (bits + kBits - 1) / kBits;
    for (int pass = 0, shift = begin_bit; pass < passes; ++pass) {
        const int left = passes - pass, nbits = (bits - (shift - begin_bit) + left - 1) / left;
        hipLaunchKernelGGL(k_hist, dim3(nb), dim3(kThreads), 0, s, (const uint64_t *)ki, n, shift, nbits, hist, nb,
                           clear, pass == 0 ? nclear : 0);
        hipLaunchKernelGGL(k_digit_scan, dim3(1u << nbits), dim3(kThreads), 0, s, hist, nb, totals);
        hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kThreads), 0, s, (const uint64_t *)ki, (const uint32_t *)vi, n,
                           shift, nbits, (const uint32_t *)hist, (const uint32_t *)totals, nb, ko, vo);
        shift += nbits;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t *tk = ki; ki = ko; ko = tk;
        uint32_t *tv = vi; vi = vo; vo = tv;
        *result_in_alt = !*result_in_alt;
    }
    return hipSuccess;
}

hipError_t launch_segment_sort_first(uint64_t *keys, uint32_t *vals, uint64_t n, const uint32_t *ranges,
                                     int64_t nlists, uint32_t *queues, uint32_t *n_queued, uint32_t *note,
                                     uint32_t *done, SortPublish pub, TileOrderScratch order, hipStream_t s)
{
    if (nlists <= 0) return launch_publish2(pub.a, pub.b, pub.host, pub.seq, note, s);
    hipLaunchKernelGGL(k_seg_first, dim3((unsigned)nlists), dim3(64), 0, s, keys, vals, ranges, (uint32_t)nlists,
                       queues, queues + nlists, n_queued, note, done, pub, order);
    return hipGetLastError();
}

hipError_t launch_segment_sort_rest(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt,
                                    uint64_t n, const uint32_t *ranges, int64_t nlists, const uint32_t *queues,
                                    const uint32_t *n_queued, uint32_t which, hipStream_t s)
{
    if (n <= 1 || nlists <= 0) return hipSuccess;
    // at most n / (L + 1) runs are longer than L entries
    const uint64_t mid = (which & kNoteSortMid) ? std::min<uint64_t>((uint64_t)nlists, n / (kSegWave + 1)) : 0;
    if (mid)
        hipLaunchKernelGGL(k_seg_mid, dim3((unsigned)mid), dim3(256), 0, s, keys, vals, ranges, queues, n_queued);
    const uint64_t large = (which & kNoteSortLarge) ? std::min<uint64_t>((uint64_t)nlists, n / (kSegSmall + 1)) : 0;
    if (large)
        hipLaunchKernelGGL(k_seg_large, dim3((unsigned)large), dim3(1024), 0, s, keys, vals, ranges, queues + nlists,
                           n_queued + 1);
    const uint64_t huge = (which & kNoteSortHuge) ? std::min<uint64_t>((uint64_t)nlists, n / (kSegLarge + 1)) : 0;
    if (huge)
        hipLaunchKernelGGL(k_seg_huge, dim3((unsigned)huge), dim3(1024), 0, s, keys, vals, keys_alt, vals_alt, ranges,
                           queues + 2 * nlists, n_queued + 2);
    return hipGetLastError();
}

// order[class_start[class] + rank] = tile for every tile, from the keys
// (rank | class << 27) that the per-list sort's filing workgroups wrote.
__global__ void k_tile_scatter(const uint32_t *__restrict__ tile_key, const uint32_t *__restrict__ class_start,
                               int ntiles, uint32_t *__restrict__ order)
{
    const int tile = blockIdx.x * blockDim.x + threadIdx.x;
    if (tile >= ntiles) return;
    const uint32_t k = tile_key[tile];
    order[class_start[k >> kOrderRankBits] + (k & ((1u << kOrderRankBits) - 1u))] = (uint32_t)tile;
}

hipError_t launch_tile_order(const uint32_t *tile_key, const uint32_t *class_start, int ntiles, uint32_t *order,
                             hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_scatter, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, s, tile_key, class_start,
                       ntiles, order);
    return hipGetLastError();
}

hipError_t launch_tile_ranges(const uint64_t *keys, uint64_t n, uint32_t *ranges, int ntiles, hipStream_t s,
                              bool cleared)
{
    uint64_t m = cleared ? 0 : 2ull * (uint64_t)ntiles;
    if (m) hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, ranges, m, 0u);
    if (n) hipLaunchKernelGGL(k_ranges, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, keys, n, ranges);
    return hipGetLastError();
}

}  // namespace aaa
