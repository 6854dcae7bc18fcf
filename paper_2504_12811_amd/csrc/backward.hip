// K6b: preprocess adjoint, one thread per visible Gaussian (double precision).
//
// Input: the per-Gaussian record gradients summed by the blend adjoint
// (line coefficients c0..c2, w0..w2, alpha~, colour).  The record was built
// from the normalised-space map A = S~^-1 R^T R_V^T and the camera centre
// o_g = -A mu_view as c_i = lambda A b_i, w_i = o_g x c_i, with b_0 the anchor
// direction and b_1, b_2 the pixel steps.  rho^2 is invariant to lambda, so
// lambda is held fixed.  The chain continues through the filter (Eq. 12,
// Eq. 8 or none; Eq. 13 clamp as a fixed decision), the activations and the
// quaternion normalisation, and the SH colour.  Gradients are accumulated
// (+=) into the caller's arrays.
#include "gauss_setup.h"

namespace aaa {

namespace {

__device__ __forceinline__ void cross3(const double *a, const double *b, double *c) { cross3d(a, b, c); }

// Adjoint of the preparation of Gaussian i for view v; adds into the
// per-Gaussian sums (gsh_out is [(DEG+1)^2][3], coefficient-major).  The SH
// degree is a template parameter so that every SH loop unrolls and its
// arrays stay in registers.
template <int DEG>
__device__ __forceinline__ void preprocess_bwd_item(const PreArgs &a, int64_t i, int v, const float *gv,
                                                    double *gmu_out, double *gls_out, double *gq_out,
                                                    double &glogit_out, float *gsh_out)
{
    const int64_t n = a.n;
    const ViewDev &vw = a.views[v];
    const int64_t item = i * a.nviews + v;
    Setup S;
    if (setup_gaussian(a, i, vw, S) != kVisible) return;
    const double *A = S.A, *R = S.R, *muv = S.muv, *og = S.og, *d = S.d;
    const float4 q5 = a.rec[(size_t)item * kRecQuads + 5];
    const double xa = q5.y, ya = q5.z;
    const double ua = (xa - vw.cam.cx) / vw.cam.fx, va = (ya - vw.cam.cy) / vw.cam.fy;
    const double b[3][3] = {{ua, va, 1.0}, {1.0 / vw.cam.fx, 0.0, 0.0}, {0.0, 1.0 / vw.cam.fy, 0.0}};
    double c[3][3];
    for (int j = 0; j < 3; ++j)
        for (int r = 0; r < 3; ++r) c[j][r] = A[3 * r] * b[j][0] + A[3 * r + 1] * b[j][1] + A[3 * r + 2] * b[j][2];
    const double lam = 1.0 / sqrt(dot3(c[0], c[0]));
    for (int j = 0; j < 3; ++j)
        for (int r = 0; r < 3; ++r) c[j][r] *= lam;

    // record -> (A, o_g)
    double gog[3] = {0, 0, 0}, gA[9];
    for (int k = 0; k < 9; ++k) gA[k] = 0.0;
    for (int j = 0; j < 3; ++j) {
        const double gc[3] = {gv[3 * j], gv[3 * j + 1], gv[3 * j + 2]};
        const double gw[3] = {gv[9 + 3 * j], gv[9 + 3 * j + 1], gv[9 + 3 * j + 2]};
        double t[3], u[3];
        cross3(c[j], gw, t);   // d/d o_g of (o_g x c) . gw
        cross3(gw, og, u);     // d/d c   of (o_g x c) . gw
        for (int r = 0; r < 3; ++r) {
            gog[r] += t[r];
            const double gct = gc[r] + u[r];
            for (int col = 0; col < 3; ++col) gA[3 * r + col] += lam * gct * b[j][col];
        }
    }
    double gmuv[3] = {0, 0, 0};
    for (int r = 0; r < 3; ++r)
        for (int col = 0; col < 3; ++col) {
            gA[3 * r + col] -= gog[r] * muv[col];
            gmuv[col] -= A[3 * r + col] * gog[r];
        }
    // A[r][c] = B[r][c] / st[r],  B[r][c] = sum_k R[k][r] RV[c][k]
    double gst[3] = {0, 0, 0}, gR[9];
    for (int k = 0; k < 9; ++k) gR[k] = 0.0;
    for (int r = 0; r < 3; ++r)
        for (int col = 0; col < 3; ++col) {
            gst[r] -= gA[3 * r + col] * A[3 * r + col] / S.st[r];
            const double gB = gA[3 * r + col] / S.st[r];
            for (int k = 0; k < 3; ++k) gR[3 * k + r] += gB * vw.RV[3 * col + k];
        }

    // alpha~ (Sec. 3.2)
    const double gat = gv[18];
    double galpha = 0.0, gs2[3] = {0, 0, 0}, gshat[3] = {0, 0, 0}, gd[3] = {0, 0, 0};
    if (a.filter_mode == 1) {
        galpha = gat;
    } else if (a.filter_mode == 2) {
        galpha = gat * S.alpha_t / S.alpha;
        for (int k = 0; k < 3; ++k) {
            gs2[k] += gat * S.alpha_t / (2.0 * S.s2[k]);
            gshat[k] -= gat * S.alpha_t / (2.0 * S.shat[k]);
        }
    } else {
        galpha = gat * S.alpha_t / S.alpha;
        const double gnum = gat * S.alpha_t / (2.0 * S.num), gden = -gat * S.alpha_t / (2.0 * S.den);
        const double p[3] = {S.dp[0] * S.dp[0], S.dp[1] * S.dp[1], S.dp[2] * S.dp[2]};
        const double *s2 = S.s2, *sh = S.shat;
        const double gp[3] = {gnum * s2[1] * s2[2] + gden * sh[1] * sh[2], gnum * s2[0] * s2[2] + gden * sh[0] * sh[2],
                              gnum * s2[0] * s2[1] + gden * sh[0] * sh[1]};
        gs2[0] += gnum * (p[1] * s2[2] + p[2] * s2[1]);
        gs2[1] += gnum * (p[0] * s2[2] + p[2] * s2[0]);
        gs2[2] += gnum * (p[0] * s2[1] + p[1] * s2[0]);
        gshat[0] += gden * (p[1] * sh[2] + p[2] * sh[1]);
        gshat[1] += gden * (p[0] * sh[2] + p[2] * sh[0]);
        gshat[2] += gden * (p[0] * sh[1] + p[1] * sh[0]);
        for (int k = 0; k < 3; ++k) {
            const double gdp = 2.0 * S.dp[k] * gp[k];
            for (int j = 0; j < 3; ++j) {  // dp[k] = sum_j R[j][k] d[j]
                gR[3 * j + k] += d[j] * gdp;
                gd[j] += R[3 * j + k] * gdp;
            }
        }
    }
    double gfa = 0.0, gls[3];
    for (int k = 0; k < 3; ++k) {
        gshat[k] += gst[k] / (2.0 * S.st[k]);
        gs2[k] += gshat[k];
        gfa += gshat[k];
        gls[k] = 2.0 * S.s2[k] * gs2[k];
    }
    if (S.fa_moves) gmuv[2] += gfa * 2.0 * a.filter_k * muv[2] / (vw.cam.fx * vw.cam.fx);
    const double glogit = galpha * S.alpha * (1.0 - S.alpha);

    // colour: c = max(0, 0.5 + sum_b Y_b(d) sh_b)
    constexpr int nb = (DEG + 1) * (DEG + 1);
    double Y[16], gY[16];
    sh_eval(DEG, d[0], d[1], d[2], Y);
#pragma unroll
    for (int k = 0; k < nb; ++k) gY[k] = 0.0;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const double gcol = gv[19 + ch];
        double acc = 0.5;
#pragma unroll
        for (int k = 0; k < nb; ++k) acc += Y[k] * (double)a.sh[((int64_t)k * 3 + ch) * n + i];
        if (!(acc > 0.0) || gcol == 0.0) continue;
#pragma unroll
        for (int k = 0; k < nb; ++k) {
            gY[k] += (double)a.sh[((int64_t)k * 3 + ch) * n + i] * gcol;
            gsh_out[3 * k + ch] += (float)(Y[k] * gcol);
        }
    }
    double gdY[3];
    sh_eval_grad(DEG, d[0], d[1], d[2], gY, gdY);
    for (int k = 0; k < 3; ++k) gd[k] += gdY[k];

    // d = (mu - o) / |mu - o|;  mu_view = R_V mu + t
    double gmu[3];
    const double dg = dot3(d, gd);
    for (int k = 0; k < 3; ++k) gmu[k] = (gd[k] - d[k] * dg) / S.dn;
    for (int k = 0; k < 3; ++k)
        for (int r = 0; r < 3; ++r) gmu[k] += vw.RV[3 * r + k] * gmuv[r];

    // rotation of the unit quaternion (w, x, y, z), then the normalisation
    const double w = S.qh[0], x = S.qh[1], y = S.qh[2], z = S.qh[3];
    const double *g = gR;
    double gq[4];
    gq[0] = 2.0 * (-z * g[1] + y * g[2] + z * g[3] - x * g[5] - y * g[6] + x * g[7]);
    gq[1] = 2.0 * (y * g[1] + z * g[2] + y * g[3] - 2.0 * x * g[4] - w * g[5] + z * g[6] + w * g[7] - 2.0 * x * g[8]);
    gq[2] = 2.0 * (-2.0 * y * g[0] + x * g[1] + w * g[2] + x * g[3] + z * g[5] - w * g[6] + z * g[7] - 2.0 * y * g[8]);
    gq[3] = 2.0 * (-2.0 * z * g[0] - w * g[1] + x * g[2] + w * g[3] - 2.0 * z * g[4] + y * g[5] + x * g[6] + y * g[7]);
    const double qg = S.qh[0] * gq[0] + S.qh[1] * gq[1] + S.qh[2] * gq[2] + S.qh[3] * gq[3];

    for (int k = 0; k < 3; ++k) {
        gmu_out[k] += gmu[k];
        gls_out[k] += gls[k];
    }
    for (int k = 0; k < 4; ++k) gq_out[k] += (gq[k] - S.qh[k] * qg) / S.qn;
    glogit_out += glogit;
}

// Gaussians with a visible item in some view, compacted in increasing
// order, so that neighbouring threads of the adjoint read neighbouring
// parameters.  A block takes kTouchPer rounds of 256 consecutive Gaussians;
// each wave's visibility ballot of a round is counted, the counts are
// scanned in (round, wave) order, and the block claims its slots with one
// atomic: its slots then hold its Gaussians in increasing order.
constexpr int kTouchPer = 16;

__device__ __forceinline__ bool gauss_visible(const int32_t *status, int64_t i, int64_t n, int nviews)
{
    bool vis = false;
    if (i < n)
        for (int v = 0; v < nviews; ++v) vis |= status[i * nviews + v] == kVisible;
    return vis;
}

__global__ __launch_bounds__(256) void k_touched(const int32_t *__restrict__ status, int64_t n, int nviews,
                                                 uint32_t *__restrict__ list, uint32_t *__restrict__ count)
{
    __shared__ uint32_t pre[kTouchPer * 4 + 1];  // exclusive offsets in (round, wave) order, then the total
    __shared__ uint32_t base;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int64_t b0 = (int64_t)blockIdx.x * 256 * kTouchPer;
    uint64_t m[kTouchPer];
#pragma unroll
    for (int k = 0; k < kTouchPer; ++k) {
        m[k] = __ballot(gauss_visible(status, b0 + (int64_t)k * 256 + t, n, nviews));
        if (lane == 0) pre[k * 4 + wave] = (uint32_t)__popcll(m[k]);
    }
    __syncthreads();
    if (t == 0) {
        uint32_t acc = 0;
        for (int k = 0; k < kTouchPer * 4; ++k) {
            const uint32_t c = pre[k];
            pre[k] = acc;
            acc += c;
        }
        pre[kTouchPer * 4] = acc;
        base = acc ? atomicAdd(count, acc) : 0u;
    }
    __syncthreads();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int k = 0; k < kTouchPer; ++k) {
        if ((m[k] >> lane) & 1ull)
            list[base + pre[k * 4 + wave] + (uint32_t)__popcll(m[k] & below)] = (uint32_t)(b0 + (int64_t)k * 256 + t);
    }
}

// One thread per listed Gaussian: sums the adjoint over the views of the
// batch and adds it to the caller's gradient arrays (no atomics needed).
template <int DEG>
__global__ __launch_bounds__(256) void k_preprocess_bwd(PreArgs a, const float *__restrict__ grad_rec, GradOut go,
                                                        const uint32_t *__restrict__ list,
                                                        const uint32_t *__restrict__ count)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= (int64_t)*count) return;
    const int64_t i = list[j];
    const int64_t n = a.n;
    constexpr int nb = (DEG + 1) * (DEG + 1);
    double gmu[3] = {0, 0, 0}, gls[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, glogit = 0.0;
    float gsh[3 * nb];
#pragma unroll
    for (int k = 0; k < 3 * nb; ++k) gsh[k] = 0.0f;
    bool touched = false;
    for (int v = 0; v < a.nviews; ++v) {
        const int64_t item = i * a.nviews + v;
        if (a.status[item] != kVisible) continue;
        const float *gr = grad_rec + (size_t)item * kGradStride;
        float gv[22];
        bool any = false;
#pragma unroll
        for (int k = 0; k < 22; ++k) {
            gv[k] = gr[k];
            any |= gv[k] != 0.0f;
        }
        if (!any) continue;
        touched = true;
        preprocess_bwd_item<DEG>(a, i, v, gv, gmu, gls, gq, glogit, gsh);
    }
    if (!touched) return;
    if (go.means)
        for (int k = 0; k < 3; ++k) go.means[k * n + i] += (float)gmu[k];
    if (go.log_scales)
        for (int k = 0; k < 3; ++k) go.log_scales[k * n + i] += (float)gls[k];
    if (go.quats)
        for (int k = 0; k < 4; ++k) go.quats[k * n + i] += (float)gq[k];
    if (go.logits) go.logits[i] += (float)glogit;
    if (go.sh) {
#pragma unroll
        for (int k = 0; k < nb; ++k)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) go.sh[((int64_t)k * 3 + ch) * n + i] += gsh[3 * k + ch];
    }
}

}  // namespace

hipError_t launch_preprocess_bwd(const PreArgs &a, const float *grad_rec, GradOut g, uint32_t *list, uint32_t *count,
                                 hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((a.n + 255) / 256);
    const unsigned tgrid = (unsigned)((a.n + 256 * kTouchPer - 1) / (256 * kTouchPer));
    hipLaunchKernelGGL(k_touched, dim3(tgrid), dim3(256), 0, s, (const int32_t *)a.status, a.n, a.nviews, list, count);
    switch (a.sh_degree) {
    case 0: hipLaunchKernelGGL(k_preprocess_bwd<0>, dim3(grid), dim3(256), 0, s, a, grad_rec, g, list, count); break;
    case 1: hipLaunchKernelGGL(k_preprocess_bwd<1>, dim3(grid), dim3(256), 0, s, a, grad_rec, g, list, count); break;
    case 2: hipLaunchKernelGGL(k_preprocess_bwd<2>, dim3(grid), dim3(256), 0, s, a, grad_rec, g, list, count); break;
    default: hipLaunchKernelGGL(k_preprocess_bwd<3>, dim3(grid), dim3(256), 0, s, a, grad_rec, g, list, count); break;
    }
    return hipGetLastError();
}

}  // namespace aaa
