// Machine rates for the roofline fractions: the FP32 fused multiply-add rate
// (non-packed, the only FP32 form the kernels here use), the v_exp_f32 rate
// and the device copy bandwidth, each measured with HIP events on the
// caller's stream.
#include <math.h>

#include "aaa_internal.h"
#include "../../include/aaa.h"

namespace {

constexpr int kThreads = 256;
constexpr int kChains = 8;      // independent dependency chains per thread
constexpr int kIters = 2048;    // loop trips per chain

// kChains independent FMA chains per lane; one result store guarded by a
// condition the data never meets (keeps the chains alive)
__global__ __launch_bounds__(kThreads) void k_fma(float *sink, float a, float b)
{
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = (float)(threadIdx.x + c);
    for (int i = 0; i < kIters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = __fmaf_rn(x[c], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    if (s == 1234.5f) sink[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_exp(float *sink, float a)
{
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = a * (float)(threadIdx.x + c) * 1e-6f;
    for (int i = 0; i < kIters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = __builtin_amdgcn_exp2f(-x[c]);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    if (s == 1234.5f) sink[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_copy(const float4 *__restrict__ src, float4 *__restrict__ dst, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kThreads)
        dst[i] = src[i];
}

}  // namespace

extern "C" int aaa_measure_peaks(void *buf, size_t bytes, int reps, void *stream, double *out)
{
    if (!buf || !out || reps < 1 || bytes < (1u << 20) || ((uintptr_t)buf & 255) != 0) return AAA_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return AAA_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return AAA_ERR_HIP;
    }
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const unsigned grid = (unsigned)(cus > 0 ? cus : 256) * 16;  // 16 workgroups of 4 waves per CU
    float *sink = (float *)buf;
    double best[3] = {0.0, 0.0, 0.0};
    const uint64_t n4 = (bytes / 2) / sizeof(float4);
    const float4 *src = (const float4 *)buf;
    float4 *dst = (float4 *)((char *)buf + n4 * sizeof(float4));
    int rc = AAA_OK;
    for (int r = 0; r < reps + 1 && rc == AAA_OK; ++r) {  // the first round warms up
        for (int k = 0; k < 3; ++k) {
            float ms = 0.0f;
            if (hipEventRecord(e0, s) != hipSuccess) rc = AAA_ERR_HIP;
            if (k == 0) hipLaunchKernelGGL(k_fma, dim3(grid), dim3(kThreads), 0, s, sink, 0.999f, 1e-3f);
            if (k == 1) hipLaunchKernelGGL(k_exp, dim3(grid), dim3(kThreads), 0, s, sink, 0.5f);
            if (k == 2) hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kThreads), 0, s, src, dst, n4);
            if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = AAA_ERR_HIP;
                break;
            }
            if (r == 0 || ms <= 0.0f) continue;
            const double threads = (double)grid * kThreads;
            double v = 0.0;
            if (k == 0) v = threads * kChains * kIters * 2.0 / (ms * 1e-3) / 1e12;   // TFLOP/s
            if (k == 1) v = threads * kChains * kIters / (ms * 1e-3) / 1e9;          // G exp/s
            if (k == 2) v = 2.0 * (double)n4 * sizeof(float4) / (ms * 1e-3) / 1e9;   // GB/s, read + write
            if (v > best[k]) best[k] = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (int k = 0; k < 3; ++k) out[k] = best[k];
    return rc;
}
