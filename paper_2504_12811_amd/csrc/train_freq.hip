// K7: training sampling frequency (Sec. 3.2).  The 3D smoothing filter's
// stored per-Gaussian frequency is the maximum of f / d over the training
// cameras, f the focal length in pixels (fx) and d the view-space depth of
// the mean; Eq. 13 clamps the render-time frequency to it.  A camera counts
// when the mean lies in front of its near plane and projects inside the
// image, border included; when no camera sees the mean, every camera with the
// mean in front of the near plane counts; with none of those the value is
// +inf (no clamp).
//
// One thread per Gaussian, cameras read as scalars (every lane walks the same
// camera).  FP64 with a fixed operation order and no fused multiply-add, so
// the result is reproducible exactly: X = ((R0 mu0 + R1 mu1) + R2 mu2) + t,
// x = cx + (fx X0) / z, y = cy + (fy X1) / z, v = fx / z; rounded to float
// once.
#include "aaa_internal.h"

namespace aaa {

namespace {

__global__ __launch_bounds__(256) void k_train_freq(const float *__restrict__ means, int64_t n,
                                                    const TrainCam *__restrict__ cams, int ncam,
                                                    float *__restrict__ out)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double m0 = means[i], m1 = means[n + i], m2 = means[2 * n + i];
    double best_in = 0.0, best_any = 0.0;
    for (int c = 0; c < ncam; ++c) {
        const TrainCam &k = cams[c];
        double X[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const double a = k.V[4 * r] * m0;
            const double b = k.V[4 * r + 1] * m1;
            const double e = k.V[4 * r + 2] * m2;
            X[r] = ((a + b) + e) + k.V[4 * r + 3];
        }
        const double z = X[2];
        if (!(z > k.znear)) continue;
        const double x = k.cx + (k.fx * X[0]) / z;
        const double y = k.cy + (k.fy * X[1]) / z;
        const double v = k.fx / z;
        best_any = v > best_any ? v : best_any;
        if (x >= 0.0 && x <= k.w && y >= 0.0 && y <= k.h && v > best_in) best_in = v;
    }
    const double r = best_in > 0.0 ? best_in : (best_any > 0.0 ? best_any : (double)INFINITY);
    out[i] = (float)r;
}

}  // namespace

hipError_t launch_train_freq(const float *means, int64_t n, const TrainCam *cams, int ncam, float *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_train_freq, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, means, n, cams, ncam, out);
    return hipGetLastError();
}

}  // namespace aaa
