// Adam update of a flat float32 parameter array in place (the optimiser step
// of a multi-view training step; Kingma & Ba, with bias correction):
//   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
//   p = p - lr (m / c1) / (sqrt(v / c2) + eps),  c1 = 1 - b1^t, c2 = 1 - b2^t.
// HBM-bound: 16 bytes read and 12 written per parameter; float4 accesses
// where the arrays allow, a scalar tail otherwise.
#include <algorithm>

#include "aaa_internal.h"

namespace aaa {

namespace {

struct AdamK {
    float lr, b1, b2, omb1, omb2, eps, c1, c2;  // omb = 1 - beta, rounded once from double
};

__device__ __forceinline__ void adam_one(float &p, float g, float &m, float &v, const AdamK &k)
{
    m = k.b1 * m + k.omb1 * g;
    v = k.b2 * v + k.omb2 * (g * g);
    const float mh = m / k.c1;
    const float vh = v / k.c2;
    p = p - k.lr * mh / (sqrtf(vh) + k.eps);
}

__global__ __launch_bounds__(256) void k_adam4(float4 *__restrict__ p, const float4 *__restrict__ g,
                                               float4 *__restrict__ m, float4 *__restrict__ v, int64_t n4, AdamK k)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
        float4 pp = p[i], mm = m[i], vv = v[i];
        const float4 gg = g[i];
        adam_one(pp.x, gg.x, mm.x, vv.x, k);
        adam_one(pp.y, gg.y, mm.y, vv.y, k);
        adam_one(pp.z, gg.z, mm.z, vv.z, k);
        adam_one(pp.w, gg.w, mm.w, vv.w, k);
        p[i] = pp;
        m[i] = mm;
        v[i] = vv;
    }
}

__global__ __launch_bounds__(256) void k_adam1(float *__restrict__ p, const float *__restrict__ g,
                                               float *__restrict__ m, float *__restrict__ v, int64_t n, AdamK k)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float pp = p[i], mm = m[i], vv = v[i];
        adam_one(pp, g[i], mm, vv, k);
        p[i] = pp;
        m[i] = mm;
        v[i] = vv;
    }
}

}  // namespace

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, double lr, double b1, double b2,
                       double eps, double c1, double c2, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    // 1 - beta from the double values: (1 - (float)0.999) would be off by 1e-5
    const AdamK k{(float)lr, (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), (float)eps, (float)c1,
                  (float)c2};
    const bool aligned = (((uintptr_t)p | (uintptr_t)g | (uintptr_t)m | (uintptr_t)v) & 15) == 0;
    int64_t head = 0;
    if (aligned) {
        const int64_t n4 = n / 4;
        if (n4 > 0) {
            const int64_t blocks = std::min<int64_t>((n4 + 255) / 256, 8192);
            hipLaunchKernelGGL(k_adam4, dim3((unsigned)blocks), dim3(256), 0, s, (float4 *)p, (const float4 *)g,
                               (float4 *)m, (float4 *)v, n4, k);
        }
        head = n4 * 4;
    }
    if (head < n) {
        const int64_t rest = n - head;
        const int64_t blocks = std::min<int64_t>((rest + 255) / 256, 8192);
        hipLaunchKernelGGL(k_adam1, dim3((unsigned)blocks), dim3(256), 0, s, p + head, g + head, m + head, v + head,
                           rest, k);
    }
    return hipGetLastError();
}

}  // namespace aaa
