// Per-Gaussian setup shared by the preprocess kernel and its adjoint, so
// that both see bit-identical intermediates.
#pragma once

#include "aaa_internal.h"

namespace aaa {

__device__ __forceinline__ void cross3d(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// Real spherical harmonics up to degree 3 (Condon-Shortley phase), index l*l+l+m.
__device__ __forceinline__ void sh_eval(int deg, double x, double y, double z, double *Y)
{
    Y[0] = 0.28209479177387814;
    if (deg < 1) return;
    Y[1] = -0.48860251190291992 * y;
    Y[2] = 0.48860251190291992 * z;
    Y[3] = -0.48860251190291992 * x;
    if (deg < 2) return;
    double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = 1.0925484305920792 * x * y;
    Y[5] = -1.0925484305920792 * y * z;
    Y[6] = 0.31539156525252005 * (2.0 * zz - xx - yy);
    Y[7] = -1.0925484305920792 * x * z;
    Y[8] = 0.54627421529603959 * (xx - yy);
    if (deg < 3) return;
    Y[9] = -0.59004358992664352 * y * (3.0 * xx - yy);
    Y[10] = 2.8906114426405538 * x * y * z;
    Y[11] = -0.45704579946446572 * y * (4.0 * zz - xx - yy);
    Y[12] = 0.3731763325901154 * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = -0.45704579946446572 * x * (4.0 * zz - xx - yy);
    Y[14] = 1.4453057213202769 * z * (xx - yy);
    Y[15] = -0.59004358992664352 * x * (xx - 3.0 * yy);
}

// Gradient of sum_b gY[b] Y_b(x, y, z) with respect to (x, y, z), the
// polynomials of sh_eval differentiated term by term.
__device__ __forceinline__ void sh_eval_grad(int deg, double x, double y, double z, const double *gY, double *g)
{
    g[0] = g[1] = g[2] = 0.0;
    if (deg < 1) return;
    const double C1 = 0.48860251190291992;
    g[1] += -C1 * gY[1];
    g[2] += C1 * gY[2];
    g[0] += -C1 * gY[3];
    if (deg < 2) return;
    const double A2 = 1.0925484305920792, B2 = 0.31539156525252005, D2 = 0.54627421529603959;
    g[0] += A2 * y * gY[4];                 g[1] += A2 * x * gY[4];
    g[1] += -A2 * z * gY[5];                g[2] += -A2 * y * gY[5];
    g[0] += -2.0 * B2 * x * gY[6];          g[1] += -2.0 * B2 * y * gY[6];  g[2] += 4.0 * B2 * z * gY[6];
    g[0] += -A2 * z * gY[7];                g[2] += -A2 * x * gY[7];
    g[0] += 2.0 * D2 * x * gY[8];           g[1] += -2.0 * D2 * y * gY[8];
    if (deg < 3) return;
    const double a9 = -0.59004358992664352, a10 = 2.8906114426405538, a11 = -0.45704579946446572;
    const double a12 = 0.3731763325901154, a14 = 1.4453057213202769;
    const double xx = x * x, yy = y * y, zz = z * z;
    // Y9 = a9 y (3xx - yy)
    g[0] += a9 * 6.0 * x * y * gY[9];       g[1] += a9 * (3.0 * xx - 3.0 * yy) * gY[9];
    // Y10 = a10 x y z
    g[0] += a10 * y * z * gY[10];           g[1] += a10 * x * z * gY[10];   g[2] += a10 * x * y * gY[10];
    // Y11 = a11 y (4zz - xx - yy)
    g[0] += a11 * (-2.0 * x * y) * gY[11];  g[1] += a11 * (4.0 * zz - xx - 3.0 * yy) * gY[11];
    g[2] += a11 * 8.0 * y * z * gY[11];
    // Y12 = a12 z (2zz - 3xx - 3yy)
    g[0] += a12 * (-6.0 * x * z) * gY[12];  g[1] += a12 * (-6.0 * y * z) * gY[12];
    g[2] += a12 * (6.0 * zz - 3.0 * xx - 3.0 * yy) * gY[12];
    // Y13 = a11 x (4zz - xx - yy)
    g[0] += a11 * (4.0 * zz - 3.0 * xx - yy) * gY[13];  g[1] += a11 * (-2.0 * x * y) * gY[13];
    g[2] += a11 * 8.0 * x * z * gY[13];
    // Y14 = a14 z (xx - yy)
    g[0] += a14 * 2.0 * x * z * gY[14];     g[1] += -a14 * 2.0 * y * z * gY[14];  g[2] += a14 * (xx - yy) * gY[14];
    // Y15 = a9 x (xx - 3yy)
    g[0] += a9 * (3.0 * xx - 3.0 * yy) * gY[15];  g[1] += a9 * (-6.0 * x * y) * gY[15];
}

struct Setup {
    double mu[3], s[3], s2[3], shat[3], st[3];
    double alpha, alpha_t, tau;
    double qn, qh[4], R[9];
    double muv[3], dz, v, fa;
    bool fa_moves;          // filter variance depends on the view depth (not clamped)
    double d[3], dn, dp[3], num, den;
    double M[9], A[9], og[3], og2;
};

// Sec. 3.1 Eq. 1-3 activations, Sec. 3.2 filter (Eq. 6-13), tau, and the
// maps between normalised Gaussian space and view space.  Returns kInvalid,
// kLowOpacity or kVisible (later culls are the caller's).
__device__ __forceinline__ int setup_gaussian(const PreArgs &a, int64_t i, const ViewDev &vw, Setup &G)
{
    const int64_t n = a.n;
    double ls[3], q[4];
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
        G.mu[k] = a.means[k * n + i];
        ls[k] = a.log_scales[k * n + i];
        ok = ok && isfinite(G.mu[k]) && isfinite(ls[k]);
    }
    for (int k = 0; k < 4; ++k) {
        q[k] = a.quats[k * n + i];
        ok = ok && isfinite(q[k]);
    }
    double logit = a.logits[i];
    G.qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    ok = ok && isfinite(logit) && G.qn > 0.0;
    if (!ok) return kInvalid;
    for (int k = 0; k < 3; ++k) G.s[k] = exp(ls[k]);
    G.alpha = 1.0 / (1.0 + exp(-logit));
    for (int k = 0; k < 4; ++k) G.qh[k] = q[k] / G.qn;
    const double w = G.qh[0], x = G.qh[1], y = G.qh[2], z = G.qh[3];
    double *R = G.R;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
    for (int r = 0; r < 3; ++r)
        G.muv[r] = vw.RV[3 * r] * G.mu[0] + vw.RV[3 * r + 1] * G.mu[1] + vw.RV[3 * r + 2] * G.mu[2] + vw.tV[r];
    // filter variance k / v'^2 with v = fx / max(z, znear), v' = min(v_train, v)
    G.dz = fmax(G.muv[2], vw.cam.znear);
    G.v = vw.cam.fx / G.dz;
    G.fa_moves = a.filter_mode != 1 && G.muv[2] > vw.cam.znear;
    if (a.v_train) {
        double vt = (double)a.v_train[i];
        if (vt < G.v) {
            G.v = vt;
            G.fa_moves = false;
        }
    }
    G.fa = a.filter_mode == 1 ? 0.0 : a.filter_k / (G.v * G.v);
    for (int k = 0; k < 3; ++k) {
        G.s2[k] = G.s[k] * G.s[k];
        G.shat[k] = G.s2[k] + G.fa;
        G.st[k] = sqrt(G.shat[k]);
    }
    for (int k = 0; k < 3; ++k) G.d[k] = G.mu[k] - vw.o[k];
    G.dn = sqrt(dot3(G.d, G.d));
    for (int k = 0; k < 3; ++k) G.d[k] /= G.dn;
    for (int k = 0; k < 3; ++k) G.dp[k] = R[k] * G.d[0] + R[3 + k] * G.d[1] + R[6 + k] * G.d[2];
    if (a.filter_mode == 1) {
        G.alpha_t = G.alpha;
    } else if (a.filter_mode == 2) {
        G.alpha_t = G.alpha * sqrt((G.s2[0] * G.s2[1] * G.s2[2]) / (G.shat[0] * G.shat[1] * G.shat[2]));  // Eq. 8
    } else {
        const double p0 = G.dp[0] * G.dp[0], p1 = G.dp[1] * G.dp[1], p2 = G.dp[2] * G.dp[2];
        G.num = p0 * G.s2[1] * G.s2[2] + p1 * G.s2[0] * G.s2[2] + p2 * G.s2[0] * G.s2[1];
        G.den = p0 * G.shat[1] * G.shat[2] + p1 * G.shat[0] * G.shat[2] + p2 * G.shat[0] * G.shat[1];
        G.alpha_t = G.alpha * sqrt(G.num / G.den);  // Eq. 12
    }
    if (!(G.alpha_t >= a.alpha_min)) return kLowOpacity;
    G.tau = 2.0 * log(G.alpha_t / a.alpha_min);
    // M = R_V R S~ (normalised Gaussian space -> view); A = M^-1 = S~^-1 R^T R_V^T
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = vw.RV[3 * r] * R[c] + vw.RV[3 * r + 1] * R[3 + c] + vw.RV[3 * r + 2] * R[6 + c];
            G.M[3 * r + c] = acc * G.st[c];
            G.A[3 * c + r] = acc / G.st[c];
        }
    // camera centre (view origin) in normalised space: -A mu_v
    for (int r = 0; r < 3; ++r) G.og[r] = -(G.A[3 * r] * G.muv[0] + G.A[3 * r + 1] * G.muv[1] + G.A[3 * r + 2] * G.muv[2]);
    G.og2 = dot3(G.og, G.og);
    return kVisible;
}

}  // namespace aaa
