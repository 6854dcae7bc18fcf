// K5: per-tile blending, and K6a: its adjoint in two passes.
//
// One workgroup per 16x16 tile; each wavefront owns an 8x8 quadrant and walks
// the tile's sorted list on its own (no barriers, per-wave early exit).  Every
// lane of a wave needs the same Gaussian at the same time, so the list entry
// and its record are fetched with scalar loads and reach the arithmetic as
// SGPR operands.
//
// Per pixel and list entry (Sec. 3.1, Eq. 4-5): rho^2 and the depth of the
// maximum along the pixel line from the anchored record; alpha =
// min(alpha_max, alpha~ exp(-rho^2/2)).  Contributors (alpha >= alpha_min,
// depth >= znear) enter a per-ray window of K entries kept sorted by depth in
// registers (the per-ray level of the hierarchical re-sort, Sec. 4); when it
// overflows its front is blended front to back; blending stops before the
// first entry that would take the transmittance below t_min.
//
// Adjoint.  Pass 1 replays the forward exactly (same code, explicit FMAs)
// and, at every blended entry k, evaluates the front-to-back derivative
//   dL/dalpha_k = T_k (c_k . g) - ((C_out - A_k) . g) / (1 - alpha_k),
//   A_k = sum_{j <= k} T_j alpha_j c_j,
// so no per-pixel list is kept from the forward: the state is recomputed per
// tile.  It stores (dL/dalpha_k, T_k alpha_k) in the pixel's slot for the
// entry's contributor rank (its position among the pixel's contributors in
// list order).  Pass 2 walks the list in list order again, so that all lanes
// look at the same Gaussian: each contributing lane turns its two scalars into
// the 22 record gradients (line coefficients, alpha~, colour), the wave sums
// them with DPP row reductions, and one instruction adds them atomically.
#include <algorithm>

#include "aaa_internal.h"

namespace aaa {

namespace {

// A wave-uniform read of a buffer that the kernel never writes, through the
// constant address space: the compiler then issues a scalar load even in a
// kernel that also stores to global memory (for a generic pointer it cannot
// rule out that those stores alias the buffer, and falls back to a vector
// load that waits behind every store in flight).
template <typename T>
__device__ __forceinline__ T uniform_read(const T *p)
{
    return *(const __attribute__((address_space(4))) T *)p;
}

struct PixelState {
    float T, C[3];
    bool done;
};

// Slots per run on one XCD: the q-th slot that XCD x takes (consecutive
// workgroups land on consecutive XCDs) is the (q % kXcdRun)-th of its
// (q / kXcdRun)-th run of kXcdRun consecutive slots, so that neighbouring
// slots (neighbouring tiles, which share records) share an L2 while the
// XCDs still take the slot order together.  Launches cover a multiple of
// 8 kXcdRun slots.
constexpr int kXcdRun = 4;
__device__ __forceinline__ int xcd_slot(int q, int x) { return ((q / kXcdRun) * 8 + x) * kXcdRun + q % kXcdRun; }
inline int slot_runs(int nslots) { return (nslots + 8 * kXcdRun - 1) / (8 * kXcdRun) * kXcdRun; }

struct Eval {
    float rx, ry, rz, wx, wy, wz, D, N;
};

// Line direction r and o_g x r at a pixel offset, with explicit FMAs so that
// the forward pass and its replays take identical decisions.
__device__ __forceinline__ Eval eval_line(float dx, float dy, float4 q0, float4 q1, float4 q2, float4 q3, float4 q4)
{
    Eval e;
    e.rx = __fmaf_rn(dy, q1.z, __fmaf_rn(dx, q0.w, q0.x));
    e.ry = __fmaf_rn(dy, q1.w, __fmaf_rn(dx, q1.x, q0.y));
    e.rz = __fmaf_rn(dy, q2.x, __fmaf_rn(dx, q1.y, q0.z));
    e.wx = __fmaf_rn(dy, q3.w, __fmaf_rn(dx, q3.x, q2.y));
    e.wy = __fmaf_rn(dy, q4.x, __fmaf_rn(dx, q3.y, q2.z));
    e.wz = __fmaf_rn(dy, q4.y, __fmaf_rn(dx, q3.z, q2.w));
    e.D = __fmaf_rn(e.rz, e.rz, __fmaf_rn(e.ry, e.ry, e.rx * e.rx));
    e.N = __fmaf_rn(e.wz, e.wz, __fmaf_rn(e.wy, e.wy, e.wx * e.wx));
    return e;
}

// What the evaluation of one list entry reads from its record (line
// coefficients, depth numerator, anchor, alpha~, prefilter threshold): 25
// scalars, fetched one list entry ahead.
struct Hot {
    float4 q0, q1, q2, q3;
    float w2y, w2z, l0, l1, l2, xa, ya, at, tp;
};

__device__ __forceinline__ Hot load_hot(const float4 *__restrict__ rec, uint32_t item)
{
    const float4 *r = rec + (size_t)item * kRecQuads;
    const float *f = (const float *)r;
    Hot h;
    h.q0 = r[0];
    h.q1 = r[1];
    h.q2 = r[2];
    h.q3 = r[3];
    h.w2y = f[16];
    h.w2z = f[17];
    h.l0 = f[18];
    h.l1 = f[19];
    h.l2 = f[20];
    h.xa = f[21];
    h.ya = f[22];
    h.at = f[23];
    h.tp = f[24];
    return h;
}

__device__ __forceinline__ Eval eval_line(float dx, float dy, const Hot &h)
{
    Eval e;
    e.rx = __fmaf_rn(dy, h.q1.z, __fmaf_rn(dx, h.q0.w, h.q0.x));
    e.ry = __fmaf_rn(dy, h.q1.w, __fmaf_rn(dx, h.q1.x, h.q0.y));
    e.rz = __fmaf_rn(dy, h.q2.x, __fmaf_rn(dx, h.q1.y, h.q0.z));
    e.wx = __fmaf_rn(dy, h.q3.w, __fmaf_rn(dx, h.q3.x, h.q2.y));
    e.wy = __fmaf_rn(dy, h.w2y, __fmaf_rn(dx, h.q3.y, h.q2.z));
    e.wz = __fmaf_rn(dy, h.w2z, __fmaf_rn(dx, h.q3.z, h.q2.w));
    e.D = __fmaf_rn(e.rz, e.rz, __fmaf_rn(e.ry, e.ry, e.rx * e.rx));
    e.N = __fmaf_rn(e.wz, e.wz, __fmaf_rn(e.wy, e.wy, e.wx * e.wx));
    return e;
}

struct BwdPixel {
    float A[3];     // front colour accumulated so far
    float Cout[3];  // forward output of the pixel
    float g[3];     // dL / d out_rgb
    float2 *slots;  // this lane's column of its quadrant's slot rows (row = contributor rank, stride 64)
};

__device__ __forceinline__ float3 float3_of(float4 q) { return make_float3(q.x, q.y, q.z); }

// Blend (forward) or replay (pass 1) one popped entry.  Pass 1 writes the
// slot of every contributor it pops: the two scalars when the entry is
// blended, zeros when the ray has terminated (at this entry or before), so
// every slot below the pixel's contributor count is written exactly once.
// The forward passes the entry's colour in `cf` (gathered ahead of use);
// pass 1 gathers it here, only for entries that blend.
template <bool PASS1>
__device__ __forceinline__ void blend_entry(PixelState &ps, const float4 *__restrict__ rec, uint32_t item, float3 cf,
                                            uint32_t rank, float a, float t_min, BwdPixel &bp, uint32_t cap)
{
    if (a > 0.0f) {  // window fillers and idle lanes carry alpha 0
        bool blends = false;
        if (!ps.done) {
            const float Tn = ps.T * (1.0f - a);
            if (Tn < t_min) {
                ps.done = true;
            } else {
                const float3 c = PASS1 ? float3_of(rec[(size_t)item * kRecQuads + 7]) : cf;
                const float W = ps.T * a;
                if (PASS1) {
                    bp.A[0] += W * c.x;
                    bp.A[1] += W * c.y;
                    bp.A[2] += W * c.z;
                    const float cg = c.x * bp.g[0] + c.y * bp.g[1] + c.z * bp.g[2];
                    const float Sg = (bp.Cout[0] - bp.A[0]) * bp.g[0] + (bp.Cout[1] - bp.A[1]) * bp.g[1] +
                                     (bp.Cout[2] - bp.A[2]) * bp.g[2];
                    // 1 - a >= 1 - alpha_max > 0
                    if (rank < cap)
                        bp.slots[(size_t)rank * 64] =
                            make_float2(ps.T * cg - Sg * __builtin_amdgcn_rcpf(1.0f - a), W);
                } else {
                    ps.C[0] += W * c.x;
                    ps.C[1] += W * c.y;
                    ps.C[2] += W * c.z;
                }
                ps.T = Tn;
                blends = true;
            }
        }
        if (PASS1 && !blends && rank < cap) bp.slots[(size_t)rank * 64] = make_float2(0.0f, 0.0f);
    }
}

// RankT: the LDS type of pass 1's contributor ranks (uint16_t when every
// rank of the frame fits, which leaves room for a fourth workgroup per CU).
// WPB: waves per workgroup, 4 (a tile) or 1 (a quadrant: a wave that
// finishes early frees its registers and LDS at once, which the forward
// gains from; the replay does better with whole tiles).
template <int K, bool STATS, bool PASS1, typename RankT = uint32_t, int WPB = 4>
__global__ __launch_bounds__(64 * WPB) void k_blend(const float4 *__restrict__ rec, const uint32_t *__restrict__ vals,
                                                    BlendArgs a)
{
    const int ntiles = a.total_tiles;
    // Consecutive workgroups land on consecutive XCDs; slots are dealt to the
    // XCDs in short runs (xcd_slot), so that each XCD gets an even share of
    // dense and sparse image regions (contiguous bands per XCD left the XCDs
    // with dense bands working long after the others); with one wave per
    // workgroup the four quadrants of a tile share an XCD.
    // Without a tile order slot s renders tile s; with one, slot s renders tile
    // tile_order[s] (longest lists first, so the last workgroups to start
    // are short ones).
    const int wq = (int)(blockIdx.x >> 3);
    const int slot = xcd_slot(WPB == 4 ? wq : wq >> 2, (int)(blockIdx.x & 7));
    if (slot >= ntiles) return;
    const int tile = a.tile_order ? (int)uniform_read(a.tile_order + slot) : slot;
    int v = 0;  // the view owning this tile (views are ordered by tile_base)
    while (v + 1 < a.nviews && a.views[v + 1].tile_base <= tile) ++v;
    const ViewDev &vw = a.views[v];
    const int nv = a.nviews;
    const int lt = tile - vw.tile_base;
    const int tx = lt % vw.cam.tiles_x, ty = lt / vw.cam.tiles_x;
    // wave-uniform (readfirstlane): the quadrant tests on list entries are
    // then scalar branches, and the list loads stay scalar loads
    const int wave = WPB == 4 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : (wq & 3);
    const int lane = threadIdx.x & 63;
    const int wl = WPB == 4 ? wave : 0;  // this wave's LDS rows
    const int px = tx * kTile + (wave & 1) * 8 + (lane & 7);
    const int py = ty * kTile + (wave >> 1) * 8 + (lane >> 3);
    const bool inside = px < vw.cam.width && py < vw.cam.height;
    const float fxp = (float)px + 0.5f, fyp = (float)py + 0.5f;
    // wave-uniform (readfirstlane): the list walk stays on scalar loads
    const int list = __builtin_amdgcn_readfirstlane(a.quad_lists ? 4 * tile + wave : tile);
    const uint32_t start = a.ranges[2 * list], end = a.ranges[2 * list + 1];
    // k_blend_long renders long lists when they are few (see k_find_long)
    if (!PASS1 && end - start > a.long_list && *a.n_long <= kMaxLongTiles) return;
    const size_t hw = (size_t)vw.cam.width * vw.cam.height;
    const size_t pix = inside ? (size_t)py * vw.cam.width + px : 0;
    const size_t gpix = vw.pix_base + pix;

    // Per-ray window, kept sorted by depth in registers; each entry's payload
    // (item, alpha and, in pass 1, the contributor rank) sits in LDS at
    // [wave][slot][lane] and never moves: a popped entry's slot takes the
    // entry inserted in its place.
    //  - K <= 16: one 32-bit key per entry, the depth's offset above znear in
    //    float ulps (order-preserving for positive floats; contributors have
    //    depth >= znear) in the high 28 bits and the slot in the low 4, so
    //    the whole insertion is one v_med3_u32 per position.  Depths are
    //    ordered exactly up to 2^32 znear; farther ones compare equal (and
    //    then order by slot, as exactly equal depths do).
    //  - K = 32: depths and slot numbers in two registers per position.
    constexpr int KS = K > 0 ? K : 1;
    constexpr bool kKeyed = K > 0 && K <= 16;
    __shared__ uint2 pay[K > 0 ? WPB : 1][KS][64];
    __shared__ RankT pay_rank[PASS1 && K > 0 ? WPB : 1][PASS1 ? KS : 1][64];
    float wz[KS];
    uint32_t ws[KS];
    uint32_t wk[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        wz[k] = -INFINITY;  // fillers: popped first, with alpha 0
        ws[k] = (uint32_t)k;
        wk[k] = (uint32_t)k;  // filler keys: depth offset 0, slot k
        if constexpr (K > 0) pay[wl][k][lane] = make_uint2(0u, 0u);
    }
    PixelState ps;
    ps.T = 1.0f;
    ps.C[0] = ps.C[1] = ps.C[2] = 0.0f;
    ps.done = !inside;
    BwdPixel bp;
    bp.slots = nullptr;
    for (int c = 0; c < 3; ++c) {
        bp.A[c] = 0.0f;
        bp.Cout[c] = (PASS1 && inside) ? vw.out_rgb[c * hw + pix] : 0.0f;
        bp.g[c] = (PASS1 && inside) ? vw.dL_drgb[c * hw + pix] : 0.0f;
    }
    uint32_t cap = 0;  // pass 1: slots of this pixel (its contributor count in the forward)
    if (PASS1 && inside) {
        bp.slots = a.slots + a.wave_off[4 * tile + wave] * 64 + lane;
        cap = a.n_ins[gpix];
    }
    // pass 1 of a quadrant without contributors has no slot to write.  (The
    // test also waits for `cap` here, once: the loop's uses of it would
    // otherwise each wait for every slot store in flight.)
    if (PASS1 && __builtin_amdgcn_ballot_w64(cap != 0u) == 0ull) return;
    uint32_t consumed = 0, rank = 0;
    uint32_t n_eval = 0, n_near = 0;
    uint32_t w_steps = 0, w_near = 0, w_contrib = 0;  // wave-uniform
    const float amin = a.alpha_min, amax = a.alpha_max, tmin = a.t_min, znear = (float)vw.cam.znear;
    const uint32_t zbits = __float_as_uint(znear);

    for (uint32_t i = start; i < end; ++i) {
        if (__builtin_amdgcn_ballot_w64(!ps.done) == 0ull) break;
        const uint32_t raw = uniform_read(vals + i);
        if ((((raw | a.quad_on) >> (kQuadShift + wave)) & 1u) == 0u) continue;  // box misses this quadrant
        const uint32_t id = (raw & a.id_mask) * (uint32_t)nv + (uint32_t)v;  // item of (Gaussian, view)
        const float4 *r = rec + (size_t)id * kRecQuads;
        const float4 q0 = r[0], q1 = r[1], q2 = r[2], q3 = r[3], q4 = r[4], q5 = r[5], q6 = r[6];
        if (STATS && !ps.done) ++n_eval;
        if (STATS) ++w_steps;
        const float dx = fxp - q5.y, dy = fyp - q5.z;
        const Eval e = eval_line(dx, dy, q0, q1, q2, q3, q4);
        const bool near = !ps.done && e.N <= q6.x * e.D;
        // wave-uniform branches from here on: the window registers are only
        // ever updated with all lanes active (no divergent copies)
        if (__builtin_amdgcn_ballot_w64(near) == 0ull) continue;
        if (STATS && near) ++n_near;
        if (STATS) ++w_near;
        const float inv = __builtin_amdgcn_rcpf(e.D);
        const float rho2 = e.N * inv;
        const float al = fminf(amax, q5.w * __builtin_amdgcn_exp2f(-(rho2 * kLog2eHalf)));
        const float z = __fmaf_rn(dy, q5.x, __fmaf_rn(dx, q4.w, q4.z)) * inv;
        const bool contrib = near && al >= amin && z >= znear;
        if (__builtin_amdgcn_ballot_w64(contrib) == 0ull) continue;
        if (STATS) ++w_contrib;
        const uint32_t my_rank = rank;
        if (contrib) ++rank;
        // the entry's own colour: scalar loads, like the rest of its record
        const float3 c_new = PASS1 ? make_float3(0.0f, 0.0f, 0.0f) : float3_of(r[7]);
        if constexpr (K == 0) {
            blend_entry<PASS1>(ps, rec, id, c_new, my_rank, contrib ? al : 0.0f, tmin, bp, cap);
        } else {
            const float ak = contrib ? al : 0.0f;
            // pop min(new, front); insert the new entry behind equal depths,
            // into the slot the front leaves
            uint32_t fs;
            bool front_out;
            uint32_t key = 0u;
            float zk = 0.0f;
            if constexpr (kKeyed) {
                // a non-contributing lane inserts key 0: below every key, so
                // the window stays as it is (at most a filler pops, a no-op)
                fs = wk[0] & 15u;
                const uint32_t doff = min(__float_as_uint(z) - zbits + 1u, (1u << 28) - 1u);
                key = contrib ? (doff << 4) | fs : 0u;
                front_out = wk[0] <= key;
            } else {
                // a non-contributing lane inserts a NaN depth: every
                // comparison is false and the window stays as it is
                zk = contrib ? z : __builtin_nanf("");
                fs = ws[0];
                front_out = wz[0] <= zk;
            }
            const uint2 fp = pay[wl][fs][lane];
            const uint32_t frk = PASS1 ? pay_rank[wl][fs][lane] : 0u;
            // forward: gather the popped entry's colour before the window
            // update, so that its latency overlaps it (the register starts as
            // the new entry's colour, which pops when the front stays; the
            // compiler then issues one load for both cases)
            float4 fc = make_float4(c_new.x, c_new.y, c_new.z, 0.0f);
            if (!PASS1 && front_out) fc = rec[(size_t)fp.x * kRecQuads + 7];
            if constexpr (kKeyed) {
                // For a sorted window the new k-th key is the median of the
                // old k-th, the new key and the old (k+1)-th; the last is the
                // larger of the old last and the new key.  (Written in place,
                // so that the compiler keeps the window registers where they
                // are.)
#pragma unroll
                for (int k = 0; k + 1 < K; ++k)
                    asm("v_med3_u32 %0, %0, %1, %2" : "+v"(wk[k]) : "v"(key), "v"(wk[k + 1]));
                wk[K - 1] = max(wk[K - 1], key);
            } else {
                // the same median rule for the depths; the slots follow with
                // two selects per position
                bool gcur = front_out;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int kn = k + 1 < K ? k + 1 : k;
                    const bool gnext = (k + 1 < K) ? (wz[kn] <= zk) : false;
                    wz[k] = (k + 1 < K) ? __builtin_amdgcn_fmed3f(wz[k], zk, wz[kn]) : (gcur ? zk : wz[k]);
                    ws[k] = gnext ? ws[kn] : (gcur ? fs : ws[k]);
                    gcur = gnext;
                }
            }
            const float pop_a = front_out ? __uint_as_float(fp.y) : ak;
            const uint32_t pop_id = front_out ? fp.x : id;
            const float3 pop_c = float3_of(fc);
            const uint32_t pop_rk = front_out ? frk : my_rank;
            if (front_out) {
                pay[wl][fs][lane] = make_uint2(id, __float_as_uint(ak));
                if (PASS1) pay_rank[wl][fs][lane] = (RankT)my_rank;
            }
            blend_entry<PASS1>(ps, rec, pop_id, pop_c, pop_rk, pop_a, tmin, bp, cap);
        }
        if (contrib && ps.done && consumed == 0) consumed = i - start + 1;
    }
    // drain the window in depth order (lanes already done only zero the
    // slots of what they hold, in pass 1)
    const bool draining = !ps.done;
    if constexpr (K > 0) {
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const uint32_t sk = kKeyed ? (wk[k] & 15u) : ws[k];
            const uint2 q = pay[wl][sk][lane];
            const uint32_t rk = PASS1 ? pay_rank[wl][sk][lane] : 0u;
            const float3 c = PASS1 ? make_float3(0.0f, 0.0f, 0.0f) : float3_of(rec[(size_t)q.x * kRecQuads + 7]);
            blend_entry<PASS1>(ps, rec, q.x, c, rk, __uint_as_float(q.y), tmin, bp, cap);
        }
    }
    if (draining) consumed = end - start;
    if (!PASS1 && inside) {
        vw.out_rgb[pix] = ps.C[0] + ps.T * vw.bg[0];
        vw.out_rgb[hw + pix] = ps.C[1] + ps.T * vw.bg[1];
        vw.out_rgb[2 * hw + pix] = ps.C[2] + ps.T * vw.bg[2];
        vw.out_T[pix] = ps.T;
        a.n_done[gpix] = consumed;
        a.n_ins[gpix] = rank;
    }
    if (STATS) {
        unsigned long long e = n_eval, c = rank, nr = n_near;
        for (int off = 32; off > 0; off >>= 1) {
            e += __shfl_down(e, off);
            c += __shfl_down(c, off);
            nr += __shfl_down(nr, off);
        }
        if (lane == 0) {
            atomicAdd(&a.counters[0], e);
            atomicAdd(&a.counters[1], c);
            atomicAdd(&a.counters[2], nr);
            atomicAdd(&a.counters[3], (unsigned long long)w_steps);
            atomicAdd(&a.counters[4], (unsigned long long)w_near);
            atomicAdd(&a.counters[5], (unsigned long long)w_contrib);
        }
    }
}

// ------------------------------------------------------ long tile lists
//
// A tile whose list is longer than a.long_list (far views: much of the scene
// in a few tiles) takes a different route.  There every Gaussian covers a
// pixel or two, so a wave that walks the list in lockstep finds one or two
// contributing lanes per entry.  Instead:
//   1. k_long_masks (many workgroups per long tile, one 64-entry word of the
//      list at a time, staged in LDS): every lane evaluates its pixel for the
//      word's entries and stores a 64-bit mask "entry contributes to this
//      pixel" (the blend's own test, without the termination state);
//   2. k_blend_long gives every lane its own walk over its pixel's set bits,
//      in list order, with the next entry's record fetched while the current
//      one is processed.  All lanes still run the window update together
//      (lanes without an entry insert a NaN depth, a no-op), so a wave step
//      serves one contribution of every pixel instead of one entry.
// Entries whose bit is clear contribute nothing to that pixel, so the result
// equals the regular kernel's.  The window slots carry alpha and colour.
//
// Mask layout: word w of the pair list for tile t sits at (w + t) * 256 +
// pixel, pixel = quadrant * 64 + lane; tile lists are in tile order, so
// (w + t) never collides between tiles.  A summary keeps one bit per
// non-empty mask word, bit (w + t) % 64 of word ((w + t) / 64) * 256 + pixel,
// so that a walk jumps over empty words with one load per 64 of them.

constexpr unsigned kMaskBlocksPerTile = 64;

// Collects the tiles with lists longer than long_list.  The long route is
// taken only when there are at most kMaxLongTiles of them: then a few tiles
// hold most of the work and the regular kernel would leave the chip idle;
// with many long tiles (a close, dense view) the regular kernel has
// parallelism enough and keeps its early termination.  Every kernel reads
// the count from device memory, so they all agree.
__global__ void k_find_long(const uint32_t *__restrict__ ranges, int ntiles, uint32_t long_list,
                            uint32_t *__restrict__ long_tiles, uint32_t *__restrict__ n_long)
{
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= ntiles) return;
    if (ranges[2 * t + 1] - ranges[2 * t] > long_list) {
        const uint32_t k = atomicAdd(n_long, 1u);
        if (k < kMaxLongTiles) long_tiles[k] = (uint32_t)t;
    }
}

// geometric contribution test of one entry at one pixel (the blend's test
// without the termination state; same arithmetic)
__device__ __forceinline__ bool contributes(float fxp, float fyp, float4 q0, float4 q1, float4 q2, float4 q3,
                                            float4 q4, float4 q5, float4 q6, float amin, float amax, float znear)
{
    const float dx = fxp - q5.y, dy = fyp - q5.z;
    const Eval e = eval_line(dx, dy, q0, q1, q2, q3, q4);
    const bool near = e.N <= q6.x * e.D;
    const float inv = __builtin_amdgcn_rcpf(e.D);
    const float rho2 = e.N * inv;
    const float al = fminf(amax, q5.w * __builtin_amdgcn_exp2f(-(rho2 * kLog2eHalf)));
    const float z = __fmaf_rn(dy, q5.x, __fmaf_rn(dx, q4.w, q4.z)) * inv;
    return near && al >= amin && z >= znear;
}

struct LongTile {
    int tile, v;
    const ViewDev *vw;
    int px, py;
    bool inside;
    uint32_t start, end;
};

__device__ __forceinline__ LongTile long_tile_setup(const BlendArgs &a, int tile, int wave)
{
    LongTile L;
    L.tile = tile;
    int v = 0;
    while (v + 1 < a.nviews && a.views[v + 1].tile_base <= tile) ++v;
    L.v = v;
    L.vw = &a.views[v];
    const int lt = tile - L.vw->tile_base;
    const int tx = lt % L.vw->cam.tiles_x, ty = lt / L.vw->cam.tiles_x;
    const int lane = threadIdx.x & 63;
    L.px = tx * kTile + (wave & 1) * 8 + (lane & 7);
    L.py = ty * kTile + (wave >> 1) * 8 + (lane >> 3);
    L.inside = L.px < L.vw->cam.width && L.py < L.vw->cam.height;
    L.start = a.ranges[2 * tile];
    L.end = a.ranges[2 * tile + 1];
    return L;
}

__global__ __launch_bounds__(256) void k_long_masks(const float4 *__restrict__ rec, const uint32_t *__restrict__ vals,
                                                    BlendArgs a, const uint32_t *__restrict__ long_tiles,
                                                    const uint32_t *__restrict__ n_long, uint64_t *__restrict__ pixmask,
                                                    uint64_t *__restrict__ summary)
{
    if (blockIdx.y >= *n_long || *n_long > kMaxLongTiles) return;
    const LongTile L = long_tile_setup(a, (int)long_tiles[blockIdx.y], (int)(threadIdx.x >> 6));
    const uint32_t nv = (uint32_t)a.nviews;
    const int t = threadIdx.x;
    const float fxp = (float)L.px + 0.5f, fyp = (float)L.py + 0.5f;
    const float amin = a.alpha_min, amax = a.alpha_max, znear = (float)L.vw->cam.znear;
    __shared__ float4 srec[64][7];
    for (uint32_t w = L.start / 64 + blockIdx.x; (uint64_t)w * 64 < L.end; w += gridDim.x) {
        for (int idx = t; idx < 64 * 7; idx += 256) {
            const uint32_t e = w * 64 + (uint32_t)(idx / 7);
            if (e >= L.start && e < L.end)
                srec[idx / 7][idx % 7] = rec[(size_t)((vals[e] & a.id_mask) * nv + (uint32_t)L.v) * kRecQuads + idx % 7];
        }
        __syncthreads();
        uint64_t bits = 0;
        for (int b = 0; b < 64; ++b) {
            const uint32_t e = w * 64 + (uint32_t)b;
            if (e < L.start || e >= L.end) continue;
            const bool c = L.inside && contributes(fxp, fyp, srec[b][0], srec[b][1], srec[b][2], srec[b][3],
                                                   srec[b][4], srec[b][5], srec[b][6], amin, amax, znear);
            bits |= c ? (1ull << b) : 0ull;
        }
        const uint64_t i = (uint64_t)w + (uint64_t)L.tile;
        pixmask[i * 256 + (uint64_t)t] = bits;
        if (bits) atomicOr((unsigned long long *)&summary[(i / 64) * 256 + (uint64_t)t], 1ull << (i % 64));
        __syncthreads();
    }
}

// One 64-thread workgroup per 8x8 quadrant of a long tile (workgroup 4j + q
// takes quadrant q of long tile j), like the forward k_blend.
template <int K, bool STATS>
__global__ __launch_bounds__(64) void k_blend_long(const float4 *__restrict__ rec, const uint32_t *__restrict__ vals,
                                                   BlendArgs a, const uint32_t *__restrict__ long_tiles,
                                                   const uint32_t *__restrict__ n_long,
                                                   const uint64_t *__restrict__ pixmask,
                                                   const uint64_t *__restrict__ summary)
{
    const uint32_t j = blockIdx.x >> 2;
    if (j >= *n_long || *n_long > kMaxLongTiles) return;
    const int wave = (int)(blockIdx.x & 3);
    const LongTile L = long_tile_setup(a, (int)long_tiles[j], wave);
    const ViewDev &vw = *L.vw;
    const uint32_t nv = (uint32_t)a.nviews;
    const int lane = (int)(threadIdx.x & 63), t = wave * 64 + lane;  // t: the pixel's column of the masks
    const float fxp = (float)L.px + 0.5f, fyp = (float)L.py + 0.5f;
    const uint32_t start = L.start, end = L.end;
    const size_t hw = (size_t)vw.cam.width * vw.cam.height;
    const size_t pix = L.inside ? (size_t)L.py * vw.cam.width + L.px : 0;
    const size_t gpix = vw.pix_base + pix;

    // The window of k_blend's keyed form (K <= 16 here: K = 32 keeps every
    // tile in k_blend): the same keys, the same median update, so both routes
    // pop the same entries in the same order, ties included (by slot).
    static_assert(K <= 16, "the long-list route serves K <= 16");
    constexpr int KS = K > 0 ? K : 1;
    __shared__ float4 pay[1][KS][64];  // (alpha, r, g, b) per slot
    uint32_t wk[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        wk[k] = (uint32_t)k;  // filler keys: depth offset 0, slot k
        if constexpr (K > 0) pay[0][k][lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    bool done = !L.inside;
    uint32_t consumed = 0, rank = 0;
    uint32_t n_eval = 0, n_near = 0, w_steps = 0, w_near = 0, w_contrib = 0;
    const float amin = a.alpha_min, amax = a.alpha_max, tmin = a.t_min, znear = (float)vw.cam.znear;
    const uint32_t zbits = __float_as_uint(znear);

    auto blend = [&](float al, float cr, float cg, float cb) {
        if (al > 0.0f && !done) {
            const float Tn = T * (1.0f - al);
            if (Tn < tmin) {
                done = true;
            } else {
                const float W = T * al;
                C0 += W * cr;
                C1 += W * cg;
                C2 += W * cb;
                T = Tn;
            }
        }
    };

    // this lane's walk over its set bits: word w (global index), bits left;
    // the summary word in hand covers positions sb * 64 .. sb * 64 + 63 of
    // (w + tile)
    const uint64_t tl = (uint64_t)L.tile;
    const uint64_t i_last = (uint64_t)((end - 1) / 64) + tl;
    uint64_t i_cur = (uint64_t)(start / 64) + tl;
    uint64_t bits = 0;
    auto word_bits = [&](uint64_t i) {
        const uint64_t ww = i - tl;
        uint64_t b = pixmask[i * 256 + (uint64_t)t];
        if (ww * 64 < start) b &= ~0ull << (start - ww * 64);
        if (i == i_last && (end & 63u)) b &= (1ull << (end & 63u)) - 1ull;
        return b;
    };
    uint64_t sb = i_cur / 64;
    uint64_t sw = summary[sb * 256 + (uint64_t)t];
    bits = L.inside ? word_bits(i_cur) : 0ull;
    // next entry of the walk, or end when the pixel has none left
    auto advance = [&]() -> uint32_t {
        while (bits == 0ull) {
            if (i_cur >= i_last) return end;
            // next non-empty word after i_cur, from the summary
            uint64_t nxt = i_cur + 1;
            if (nxt / 64 != sb) {
                sb = nxt / 64;
                sw = summary[sb * 256 + (uint64_t)t];
            }
            uint64_t m = sw & (~0ull << (nxt % 64));
            while (m == 0ull) {
                ++sb;
                if (sb * 64 > i_last) return end;
                sw = summary[sb * 256 + (uint64_t)t];
                m = sw;
            }
            i_cur = sb * 64 + (uint64_t)__builtin_ctzll(m);
            if (i_cur > i_last) return end;
            bits = word_bits(i_cur);
        }
        const uint32_t e = (uint32_t)((i_cur - tl) * 64) + (uint32_t)__builtin_ctzll(bits);
        bits &= bits - 1ull;
        return e;
    };
    uint32_t e_cur = (L.inside && !done) ? advance() : end;
    float4 r0, r1, r2, r3, r4, r5, r6, r7;
    auto fetch = [&](uint32_t e) {
        if (e < end) {
            const float4 *r = rec + (size_t)((vals[e] & a.id_mask) * nv + (uint32_t)L.v) * kRecQuads;
            r0 = r[0]; r1 = r[1]; r2 = r[2]; r3 = r[3]; r4 = r[4]; r5 = r[5]; r6 = r[6]; r7 = r[7];
        }
    };
    fetch(e_cur);
    while (__builtin_amdgcn_ballot_w64(e_cur < end && !done) != 0ull) {
        const bool has = e_cur < end && !done;
        const float4 q0 = r0, q1 = r1, q2 = r2, q3 = r3, q4 = r4, q5 = r5, q6 = r6, col = r7;
        const uint32_t e_this = e_cur;
        // the following entry of this pixel is fetched while this one is processed
        e_cur = has ? advance() : end;
        fetch(e_cur);
        if (STATS && has) ++n_eval;
        if (STATS) ++w_steps;
        const float dx = fxp - q5.y, dy = fyp - q5.z;
        const Eval ev = eval_line(dx, dy, q0, q1, q2, q3, q4);
        const bool near = has && ev.N <= q6.x * ev.D;
        if (STATS && near) ++n_near;
        const float inv = __builtin_amdgcn_rcpf(ev.D);
        const float rho2 = ev.N * inv;
        const float al = fminf(amax, q5.w * __builtin_amdgcn_exp2f(-(rho2 * kLog2eHalf)));
        const float z = __fmaf_rn(dy, q5.x, __fmaf_rn(dx, q4.w, q4.z)) * inv;
        const bool contrib = near && al >= amin && z >= znear;
        if (STATS) ++w_contrib;
        if (contrib) ++rank;
        if constexpr (K == 0) {
            blend(contrib ? al : 0.0f, col.x, col.y, col.z);
        } else {
            const float ak = contrib ? al : 0.0f;
            const uint32_t fs = wk[0] & 15u;
            const uint32_t doff = min(__float_as_uint(z) - zbits + 1u, (1u << 28) - 1u);
            const uint32_t key = contrib ? (doff << 4) | fs : 0u;
            const float4 fp = pay[0][fs][lane];
            const bool front_out = wk[0] <= key;
#pragma unroll
            for (int kk = 0; kk + 1 < K; ++kk)
                asm("v_med3_u32 %0, %0, %1, %2" : "+v"(wk[kk]) : "v"(key), "v"(wk[kk + 1]));
            wk[K - 1] = max(wk[K - 1], key);
            if (front_out) pay[0][fs][lane] = make_float4(ak, col.x, col.y, col.z);
            if (front_out)
                blend(fp.x, fp.y, fp.z, fp.w);
            else
                blend(ak, col.x, col.y, col.z);
        }
        if (contrib && done && consumed == 0) consumed = e_this - start + 1;
    }
    const bool draining = !done;
    if constexpr (K > 0) {
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const float4 q = pay[0][wk[k] & 15u][lane];
            blend(done ? 0.0f : q.x, q.y, q.z, q.w);
        }
    }
    if (draining) consumed = end - start;
    if (L.inside) {
        vw.out_rgb[pix] = C0 + T * vw.bg[0];
        vw.out_rgb[hw + pix] = C1 + T * vw.bg[1];
        vw.out_rgb[2 * hw + pix] = C2 + T * vw.bg[2];
        vw.out_T[pix] = T;
        a.n_done[gpix] = consumed;
        a.n_ins[gpix] = rank;
    }
    if (STATS) {
        unsigned long long ec = n_eval, c = rank, nr = n_near;
        for (int off = 32; off > 0; off >>= 1) {
            ec += __shfl_down(ec, off);
            c += __shfl_down(c, off);
            nr += __shfl_down(nr, off);
        }
        if (lane == 0) {
            atomicAdd(&a.counters[0], ec);
            atomicAdd(&a.counters[1], c);
            atomicAdd(&a.counters[2], nr);
            atomicAdd(&a.counters[3], (unsigned long long)w_steps);
            atomicAdd(&a.counters[4], (unsigned long long)w_near);
            atomicAdd(&a.counters[5], (unsigned long long)w_contrib);
        }
    }
}

// ----------------------------------------------------------------- pass 2

// Reduce-scatter of 22 per-lane values over a wavefront (gfx950 lane
// swaps, then DPP inside rows of 16 lanes).
//   1. v_permlane32_swap pairs values (2j, 2j+1): one register then holds
//      value 2j summed over lanes l and l+32 in lanes 0-31 and value 2j+1 in
//      lanes 32-63.
//   2. v_permlane16_swap pairs two such registers: each row of 16 lanes then
//      holds one value summed over 4 lanes; register m holds values
//      4m, 4m+2, 4m+1, 4m+3 in rows 0..3 (register 5: values 20 and 21 in rows
//      0 and 2).
//   3. DPP steps (quad swaps, half-row mirror, row mirror) leave every lane
//      of a row holding the row's total.
// Lane 16 r + t (t < 6) then returns register t's total of row r and the
// index of that value; other lanes return index -1.
__device__ __forceinline__ float swap32_add(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float swap16_add(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float row_total(float v)
{
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, true));   // quad_perm 1,0,3,2
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, true));   // quad_perm 2,3,0,1
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, true));  // row_half_mirror
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, true));  // row_mirror
    return v;
}

__device__ __forceinline__ float reduce22(const float (&x)[22], int lane, int &idx)
{
    float u[11];
#pragma unroll
    for (int j = 0; j < 11; ++j) u[j] = swap32_add(x[2 * j], x[2 * j + 1]);
    float X[6];
#pragma unroll
    for (int m = 0; m < 5; ++m) X[m] = row_total(swap16_add(u[2 * m], u[2 * m + 1]));
    X[5] = row_total(swap16_add(u[10], 0.0f));
    const int t = lane & 15, r = lane >> 4;
    float mine = X[0];
#pragma unroll
    for (int m = 1; m < 6; ++m) mine = t == m ? X[m] : mine;
    idx = t < 5 ? 4 * t + ((r & 1) << 1) + (r >> 1) : (t == 5 && (r & 1) == 0) ? 20 + (r >> 1) : -1;
    return mine;
}

// WPB: waves per workgroup (the launch uses 1: one 8x8 quadrant per
// workgroup, so a quadrant whose pixels consumed few entries frees its slot
// on the CU without waiting for the rest of its tile).
template <int WPB>
__global__ __launch_bounds__(64 * WPB) void k_grad(const float4 *__restrict__ rec, const uint32_t *__restrict__ vals,
                                                   BlendArgs a)
{
    const int ntiles = a.total_tiles;
    const int wq = (int)(blockIdx.x >> 3);  // slots dealt to the XCDs and tile order as in k_blend
    const int slot = xcd_slot(WPB == 4 ? wq : wq >> 2, (int)(blockIdx.x & 7));
    if (slot >= ntiles) return;
    const int tile = a.tile_order ? (int)uniform_read(a.tile_order + slot) : slot;
    int v = 0;
    while (v + 1 < a.nviews && a.views[v + 1].tile_base <= tile) ++v;
    const ViewDev &vw = a.views[v];
    const uint32_t nv = (uint32_t)a.nviews;
    const int lt = tile - vw.tile_base;
    const int tx = lt % vw.cam.tiles_x, ty = lt / vw.cam.tiles_x;
    const int wave = WPB == 4 ? (int)(threadIdx.x >> 6) : (wq & 3), lane = threadIdx.x & 63;
    const int px = tx * kTile + (wave & 1) * 8 + (lane & 7);
    const int py = ty * kTile + (wave >> 1) * 8 + (lane >> 3);
    const bool inside = px < vw.cam.width && py < vw.cam.height;
    const float fxp = (float)px + 0.5f, fyp = (float)py + 0.5f;
    // wave-uniform (readfirstlane): the list walk stays on scalar loads
    const int list = __builtin_amdgcn_readfirstlane(a.quad_lists ? 4 * tile + wave : tile);
    const uint32_t start = a.ranges[2 * list], end = a.ranges[2 * list + 1];
    const size_t hw = (size_t)vw.cam.width * vw.cam.height;
    const size_t pix = inside ? (size_t)py * vw.cam.width + px : 0;
    const size_t gpix = vw.pix_base + pix;
    // entries this pixel consumed in the forward, and its slots
    const uint32_t limit = inside ? start + a.n_done[gpix] : start;
    const uint32_t cap = inside ? a.n_ins[gpix] : 0;
    const float2 *slots = a.slots + (inside ? a.wave_off[4 * tile + wave] * 64 + lane : 0);
    float g[3];
    for (int c = 0; c < 3; ++c) g[c] = inside ? vw.dL_drgb[c * hw + pix] : 0.0f;
    const float amin = a.alpha_min, amax = a.alpha_max, znear = (float)vw.cam.znear;
    // A quadrant without contributors, or without an incoming gradient (every
    // slot then holds dL/dalpha = 0 and every value below is 0), adds
    // nothing.  The test also waits for `cap` and `g` here, once: the loop's
    // uses of them would otherwise each wait for every atomic in flight.
    if (__builtin_amdgcn_ballot_w64(cap != 0u && (g[0] != 0.0f || g[1] != 0.0f || g[2] != 0.0f)) == 0ull) return;
    uint32_t rank = 0;
    // The slot of this lane's next contributor is loaded one contributor
    // ahead, so that its latency overlaps the steps in between.  Every lane
    // reloads it at every wave step with a contributor (lanes without one
    // reload the same row), from a row clamped to the quadrant's rows: the
    // load is then unconditional and lands in the same registers each time
    // (no copy that would wait for it); rows at or past the pixel's own count
    // are zeroed at use.
    uint32_t wcap = cap;  // the quadrant's largest count: its slot rows (>= 1 here)
    wcap = wave_max(wcap);
    float2 s_next = slots[0];

    const uint32_t qbit = 1u << (kQuadShift + wave);
    auto step = [&](uint32_t i, uint32_t raw, const Hot &h) {
        if (((raw | a.quad_on) & qbit) == 0u) return;  // box misses this quadrant: no pixel contributes
        const uint32_t item = (raw & a.id_mask) * nv + (uint32_t)v;
        const bool active = i < limit;
        const float dx = fxp - h.xa, dy = fyp - h.ya;
        const Eval e = eval_line(dx, dy, h);
        const bool near = active && e.N <= h.tp * e.D;
        if (__builtin_amdgcn_ballot_w64(near) == 0ull) return;
        const float inv = __builtin_amdgcn_rcpf(e.D);
        const float rho2 = e.N * inv;
        const float al = fminf(amax, h.at * __builtin_amdgcn_exp2f(-(rho2 * kLog2eHalf)));
        const float z = __fmaf_rn(dy, h.l2, __fmaf_rn(dx, h.l1, h.l0)) * inv;
        const bool contrib = near && al >= amin && z >= znear;
        if (__builtin_amdgcn_ballot_w64(contrib) == 0ull) return;
        const float2 s = (contrib && rank < cap) ? s_next : make_float2(0.0f, 0.0f);
        rank += contrib ? 1u : 0u;
        s_next = slots[(size_t)min(rank, wcap - 1u) * 64];
        // 22 record gradients of this lane (zero when not blended)
        const float ga = s.x, W = s.y;
        const bool moves = contrib && al < amax && W > 0.0f;  // a clamped alpha does not move
        const float gat = moves ? ga * al * __builtin_amdgcn_rcpf(h.at) : 0.0f;  // alpha~ >= alpha_min > 0
        const float gr2 = moves ? -0.5f * ga * al : 0.0f;
        const float kw = 2.0f * gr2 * inv, kr = -2.0f * gr2 * rho2 * inv;
        float vals22[22];
        const float gr[3] = {kr * e.rx, kr * e.ry, kr * e.rz};
        const float gw[3] = {kw * e.wx, kw * e.wy, kw * e.wz};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            vals22[k] = gr[k];
            vals22[3 + k] = dx * gr[k];
            vals22[6 + k] = dy * gr[k];
            vals22[9 + k] = gw[k];
            vals22[12 + k] = dx * gw[k];
            vals22[15 + k] = dy * gw[k];
            vals22[19 + k] = W * g[k];
        }
        vals22[18] = gat;
        // wave totals, scattered over 22 lanes (one atomic instruction)
        int idx;
        const float mine = reduce22(vals22, lane, idx);
        if (idx >= 0 && mine != 0.0f) atomicAdd(&a.grad_rec[(size_t)item * kGradStride + idx], mine);
    };

    if (start < end) {
        // same software pipeline as the forward
        uint32_t raw = vals[start];
        uint32_t raw_next = vals[start + 1 < end ? start + 1 : end - 1];
        Hot h = load_hot(rec, (raw & a.id_mask) * nv + (uint32_t)v);
        for (uint32_t i = start; i < end; ++i) {
            if (__builtin_amdgcn_ballot_w64(i < limit) == 0ull) break;
            const uint32_t raw_cur = raw_next;
            raw_next = vals[i + 2 < end ? i + 2 : end - 1];
            const Hot h_next = load_hot(rec, (raw_cur & a.id_mask) * nv + (uint32_t)v);
            step(i, raw, h);
            raw = raw_cur;
            h = h_next;
        }
    }
}

template <int K>
hipError_t launch_k(const BlendArgs &a, bool stats, bool pass1, hipStream_t s)
{
    const int ntiles = a.total_tiles;
    const int per = slot_runs(ntiles);
    dim3 tiles((unsigned)(per * 8)), quads((unsigned)(per * 8 * 4));
    if (pass1 && a.rank16)
        hipLaunchKernelGGL((k_blend<K, false, true, uint16_t>), tiles, dim3(256), 0, s, a.rec, a.vals, a);
    else if (pass1)
        hipLaunchKernelGGL((k_blend<K, false, true>), tiles, dim3(256), 0, s, a.rec, a.vals, a);
    else if (stats)
        hipLaunchKernelGGL((k_blend<K, true, false, uint32_t, 1>), quads, dim3(64), 0, s, a.rec, a.vals, a);
    else
        hipLaunchKernelGGL((k_blend<K, false, false, uint32_t, 1>), quads, dim3(64), 0, s, a.rec, a.vals, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_blend(const BlendArgs &a, int K, bool stats, bool pass1, hipStream_t s)
{
    if (a.total_tiles <= 0) return hipSuccess;
    switch (K) {
    case 0: return launch_k<0>(a, stats, pass1, s);
    case 1: return launch_k<1>(a, stats, pass1, s);
    case 2: return launch_k<2>(a, stats, pass1, s);
    case 4: return launch_k<4>(a, stats, pass1, s);
    case 8: return launch_k<8>(a, stats, pass1, s);
    case 16: return launch_k<16>(a, stats, pass1, s);
    case 32: return launch_k<32>(a, stats, pass1, s);
    default: return hipErrorInvalidValue;
    }
}

template <int K>
hipError_t launch_long_k(const BlendArgs &a, bool stats, const uint32_t *long_tiles, const uint32_t *n_long,
                         unsigned grid, const uint64_t *pixmask, const uint64_t *summary, hipStream_t s)
{
    if (stats)
        hipLaunchKernelGGL((k_blend_long<K, true>), dim3(grid * 4), dim3(64), 0, s, a.rec, a.vals, a, long_tiles, n_long,
                           pixmask, summary);
    else
        hipLaunchKernelGGL((k_blend_long<K, false>), dim3(grid * 4), dim3(64), 0, s, a.rec, a.vals, a, long_tiles,
                           n_long, pixmask, summary);
    return hipGetLastError();
}

__global__ void k_zero_u64(uint64_t *__restrict__ p, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

hipError_t launch_find_long(const BlendArgs &a, uint32_t *long_tiles, uint32_t *n_long, hipStream_t s)
{
    if (a.total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_find_long, dim3((unsigned)((a.total_tiles + 255) / 256)), dim3(256), 0, s, a.ranges,
                       a.total_tiles, a.long_list, long_tiles, n_long);
    return hipGetLastError();
}

hipError_t launch_blend_long(const BlendArgs &a, int K, bool stats, const uint32_t *long_tiles, const uint32_t *n_long,
                             unsigned grid, uint64_t *pixmask, uint64_t *summary, uint64_t summary_words, hipStream_t s)
{
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)std::min<uint64_t>((summary_words + 255) / 256, 4096)), dim3(256), 0,
                       s, summary, summary_words);
    hipLaunchKernelGGL(k_long_masks, dim3(kMaskBlocksPerTile, grid), dim3(256), 0, s, a.rec, a.vals, a, long_tiles,
                       n_long, pixmask, summary);
    switch (K) {
    case 0: return launch_long_k<0>(a, stats, long_tiles, n_long, grid, pixmask, summary, s);
    case 1: return launch_long_k<1>(a, stats, long_tiles, n_long, grid, pixmask, summary, s);
    case 2: return launch_long_k<2>(a, stats, long_tiles, n_long, grid, pixmask, summary, s);
    case 4: return launch_long_k<4>(a, stats, long_tiles, n_long, grid, pixmask, summary, s);
    case 8: return launch_long_k<8>(a, stats, long_tiles, n_long, grid, pixmask, summary, s);
    case 16: return launch_long_k<16>(a, stats, long_tiles, n_long, grid, pixmask, summary, s);
    default: return hipErrorInvalidValue;  // K = 32 keeps every tile in k_blend (long_list = max)
    }
}

// One workgroup per tile, one wave per 8x8 quadrant (the pixel mapping of
// k_blend): the quadrant's largest contributor count.
__global__ __launch_bounds__(256) void k_wave_caps(const ViewDev *__restrict__ views, int nviews,
                                                   const uint32_t *__restrict__ n_ins, uint32_t *__restrict__ caps,
                                                   uint32_t *__restrict__ max_big)
{
    const int tile = (int)blockIdx.x;
    int v = 0;
    while (v + 1 < nviews && views[v + 1].tile_base <= tile) ++v;
    const ViewDev &vw = views[v];
    const int lt = tile - vw.tile_base;
    const int tx = lt % vw.cam.tiles_x, ty = lt / vw.cam.tiles_x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int px = tx * kTile + (wave & 1) * 8 + (lane & 7);
    const int py = ty * kTile + (wave >> 1) * 8 + (lane >> 3);
    const bool inside = px < vw.cam.width && py < vw.cam.height;
    uint32_t m = inside ? n_ins[vw.pix_base + (size_t)py * vw.cam.width + px] : 0u;
    m = wave_max(m);
    if (lane == 0) {
        caps[4 * tile + wave] = m;
        if (m > 0x10000u) atomicMax(max_big, m);  // rare: pixels with more than 65536 contributors
    }
}

hipError_t launch_wave_caps(const ViewDev *views, int nviews, int total_tiles, const uint32_t *n_ins, uint32_t *caps,
                            uint32_t *max_big, hipStream_t s)
{
    if (total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_wave_caps, dim3((unsigned)total_tiles), dim3(256), 0, s, views, nviews, n_ins, caps, max_big);
    return hipGetLastError();
}

hipError_t launch_grad(const BlendArgs &a, hipStream_t s)
{
    if (a.total_tiles <= 0) return hipSuccess;
    const int per = slot_runs(a.total_tiles);
    hipLaunchKernelGGL(k_grad<1>, dim3((unsigned)(per * 8 * 4)), dim3(64), 0, s, a.rec, a.vals, a);
    return hipGetLastError();
}

}  // namespace aaa
