// K5: per-tile blending.  One workgroup per 16x16 tile; each wavefront owns
// an 8x8 quadrant and walks the tile's sorted list on its own (no barriers,
// per-wave early exit).  Every lane of a wave needs the same Gaussian at the
// same time, so the list entry and its record are fetched with scalar loads
// and reach the arithmetic as SGPR operands.
//
// Per pixel and list entry (Sec. 3.1, Eq. 4-5): rho^2 and the depth of the
// maximum along the pixel line from the anchored record; alpha =
// min(alpha_max, alpha~ exp(-rho^2/2)).  Contributors (alpha >= alpha_min,
// depth >= znear) enter a per-ray window of K entries kept sorted by depth in
// registers (the per-ray level of the hierarchical re-sort, Sec. 4); when it
// overflows its front is blended front to back; blending stops before the
// first entry that would take the transmittance below t_min.
#include "aaa_internal.h"

namespace aaa {

namespace {

struct PixelState {
    float T, C[3];
    bool done;
};

__device__ __forceinline__ void blend_entry(PixelState &ps, const float4 *__restrict__ rec, uint32_t id, float a,
                                            float t_min)
{
    if (a > 0.0f) {  // window fillers carry alpha 0
        float Tn = ps.T * (1.0f - a);
        if (Tn < t_min) {
            ps.done = true;
        } else {
            float4 c = rec[(size_t)id * kRecQuads + 7];
            float wgt = ps.T * a;
            ps.C[0] += wgt * c.x;
            ps.C[1] += wgt * c.y;
            ps.C[2] += wgt * c.z;
            ps.T = Tn;
        }
    }
}

template <int K, bool STATS>
__global__ __launch_bounds__(256) void k_blend(BlendArgs a)
{
    const int ntiles = a.cam.tiles_x * a.cam.tiles_y;
    // XCD-aware order: consecutive workgroups land on different XCDs, so hand
    // each XCD a contiguous band of tiles (neighbouring tiles share records).
    const int per = (ntiles + 7) / 8;
    const int tile = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (tile >= ntiles) return;
    const int tx = tile % a.cam.tiles_x, ty = tile / a.cam.tiles_x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int px = tx * kTile + (wave & 1) * 8 + (lane & 7);
    const int py = ty * kTile + (wave >> 1) * 8 + (lane >> 3);
    const bool inside = px < a.cam.width && py < a.cam.height;
    const float fxp = (float)px + 0.5f, fyp = (float)py + 0.5f;
    const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];

    float wz[K > 0 ? K : 1];
    uint32_t wid[K > 0 ? K : 1];
    float wa[K > 0 ? K : 1];
#pragma unroll
    for (int k = 0; k < (K > 0 ? K : 1); ++k) {
        wz[k] = -INFINITY;
        wid[k] = 0u;
        wa[k] = 0.0f;
    }
    PixelState ps;
    ps.T = 1.0f;
    ps.C[0] = ps.C[1] = ps.C[2] = 0.0f;
    ps.done = !inside;
    uint32_t consumed = 0;
    uint32_t n_eval = 0, n_contrib = 0, n_near = 0;
    const float amin = a.alpha_min, amax = a.alpha_max, tmin = a.t_min, znear = a.znear;

    for (uint32_t i = start; i < end; ++i) {
        if (__ballot(!ps.done) == 0ull) break;
        const uint32_t id = a.vals[i];
        const float4 *r = a.rec + (size_t)id * kRecQuads;
        const float4 q0 = r[0], q1 = r[1], q2 = r[2], q3 = r[3], q4 = r[4], q5 = r[5], q6 = r[6];
        if (STATS && !ps.done) ++n_eval;
        const float dx = fxp - q5.y, dy = fyp - q5.z;
        const float rx = q0.x + dx * q0.w + dy * q1.z;
        const float ry = q0.y + dx * q1.x + dy * q1.w;
        const float rz = q0.z + dx * q1.y + dy * q2.x;
        const float wx = q2.y + dx * q3.x + dy * q3.w;
        const float wy = q2.z + dx * q3.y + dy * q4.x;
        const float wzz = q2.w + dx * q3.z + dy * q4.y;
        const float D = rx * rx + ry * ry + rz * rz;
        const float N = wx * wx + wy * wy + wzz * wzz;
        const bool near = !ps.done && N <= q6.x * D;
        // wave-uniform branches from here on: the window registers are only
        // ever updated with all lanes active (no divergent copies)
        if (__ballot(near) == 0ull) continue;
        if (STATS && near) ++n_near;
        const float inv = __builtin_amdgcn_rcpf(D);
        const float rho2 = N * inv;
        const float al = fminf(amax, q5.w * __builtin_amdgcn_exp2f(-rho2 * kLog2eHalf));
        const float z = (q4.z + dx * q4.w + dy * q5.x) * inv;
        const bool contrib = near && al >= amin && z >= znear;
        if (__ballot(contrib) == 0ull) continue;
        if (STATS && contrib) ++n_contrib;
        if (K == 0) {
            if (contrib) blend_entry(ps, a.rec, id, al, tmin);
        } else {
            // Non-contributing lanes insert a NaN depth: every comparison is
            // false, the window stays as it is and the popped entry is the
            // NaN one with alpha 0 (a no-op blend).
            const float zk = contrib ? z : __builtin_nanf("");
            const float ak = contrib ? al : 0.0f;
            // pop min(new, front); insert new behind equal depths
            bool gcur = wz[0] <= zk;
            const float pop_a = gcur ? wa[0] : ak;
            const uint32_t pop_id = gcur ? wid[0] : id;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int kn = k + 1 < K ? k + 1 : k;
                const bool gnext = (k + 1 < K) ? (wz[kn] <= zk) : false;
                wz[k] = gnext ? wz[kn] : (gcur ? zk : wz[k]);
                wid[k] = gnext ? wid[kn] : (gcur ? id : wid[k]);
                wa[k] = gnext ? wa[kn] : (gcur ? ak : wa[k]);
                gcur = gnext;
            }
            blend_entry(ps, a.rec, pop_id, pop_a, tmin);
        }
        if (contrib && ps.done && consumed == 0) consumed = i - start + 1;
    }
    if (!ps.done) {
        consumed = end - start;
#pragma unroll
        for (int k = 0; k < (K > 0 ? K : 1); ++k)
            if (K > 0 && !ps.done) blend_entry(ps, a.rec, wid[k], wa[k], tmin);
    }
    if (inside) {
        const size_t hw = (size_t)a.cam.width * a.cam.height;
        const size_t pix = (size_t)py * a.cam.width + px;
        a.out_rgb[pix] = ps.C[0] + ps.T * a.bg[0];
        a.out_rgb[hw + pix] = ps.C[1] + ps.T * a.bg[1];
        a.out_rgb[2 * hw + pix] = ps.C[2] + ps.T * a.bg[2];
        a.out_T[pix] = ps.T;
        a.n_done[pix] = consumed;
    }
    if (STATS) {
        unsigned long long e = n_eval, c = n_contrib, nr = n_near;
        for (int off = 32; off > 0; off >>= 1) {
            e += __shfl_down(e, off);
            c += __shfl_down(c, off);
            nr += __shfl_down(nr, off);
        }
        if (lane == 0) {
            atomicAdd(&a.counters[0], e);
            atomicAdd(&a.counters[1], c);
            atomicAdd(&a.counters[2], nr);
        }
    }
}

template <int K>
hipError_t launch_k(const BlendArgs &a, bool stats, hipStream_t s)
{
    const int ntiles = a.cam.tiles_x * a.cam.tiles_y;
    const int per = (ntiles + 7) / 8;
    dim3 grid((unsigned)(per * 8));
    if (stats)
        hipLaunchKernelGGL((k_blend<K, true>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_blend<K, false>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_blend(const BlendArgs &a, int K, bool stats, hipStream_t s)
{
    if (a.cam.tiles_x * a.cam.tiles_y <= 0) return hipSuccess;
    switch (K) {
    case 0: return launch_k<0>(a, stats, s);
    case 1: return launch_k<1>(a, stats, s);
    case 2: return launch_k<2>(a, stats, s);
    case 4: return launch_k<4>(a, stats, s);
    case 8: return launch_k<8>(a, stats, s);
    case 16: return launch_k<16>(a, stats, s);
    case 32: return launch_k<32>(a, stats, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace aaa
