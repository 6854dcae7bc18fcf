"""Pins of the FP64 oracle against closed forms, brute force and invariants.

Each test checks the oracle against something other than itself: the
paper's defining formulas evaluated by an independent route (numpy linear
algebra, dense sampling, quadrature), textbook identities, or invariants.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import oracle as O
from paper_2504_12811_amd import scenes as S


def one_gaussian(mu, log_s, q, logit, colour=(1.0, 1.0, 1.0), v_train=None, deg=0):
    n = 1
    sh = np.zeros(((deg + 1) ** 2, 3, n), np.float32)
    sh[0, :, 0] = (np.asarray(colour) - 0.5) / S.SH_C0
    return S.Scene(
        means=np.asarray(mu, np.float32).reshape(3, 1),
        log_scales=np.asarray(log_s, np.float32).reshape(3, 1),
        quats=np.asarray(q, np.float32).reshape(4, 1),
        opacity_logits=np.asarray([logit], np.float32),
        sh=sh,
        v_train=None if v_train is None else np.asarray([v_train], np.float32),
    )


def rot_np(q):
    """Rodrigues rotation of the unit quaternion q=(w,x,y,z), written independently."""
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q)
    w, v = q[0], q[1:]
    ang = 2 * math.atan2(np.linalg.norm(v), w)
    if np.linalg.norm(v) < 1e-300:
        return np.eye(3)
    k = v / np.linalg.norm(v)
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def f64(a):
    return np.asarray(a, np.float32).astype(np.float64)


# ----------------------------------------------------------------------------
# Rotation (Eq.3) and spherical harmonics


def test_rotation_matches_rodrigues():
    rng = np.random.default_rng(0)
    for _ in range(20):
        q = rng.normal(size=4) * rng.uniform(0.1, 3)
        R = O.rotation(q)
        np.testing.assert_allclose(R, rot_np(q), atol=1e-13)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-13)
        assert abs(np.linalg.det(R) - 1) < 1e-12


def test_sh_orthonormal_by_quadrature():
    """Gauss-Legendre x uniform-phi quadrature of Y_i Y_j over the sphere = delta_ij (degree <= 3)."""
    xs, ws = np.polynomial.legendre.leggauss(24)
    nphi = 48
    phis = 2 * np.pi * np.arange(nphi) / nphi
    G = np.zeros((16, 16))
    for x, w in zip(xs, ws):
        st = math.sqrt(1 - x * x)
        for ph in phis:
            d = np.array([st * math.cos(ph), st * math.sin(ph), x])
            Y = O.sh_basis(3, d)
            G += w * (2 * np.pi / nphi) * np.outer(Y, Y)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_textbook_values():
    d = np.array([0.3, -0.4, 0.5])
    d = d / np.linalg.norm(d)
    x, y, z = d
    Y = O.sh_basis(3, d)
    assert Y[0] == pytest.approx(1 / (2 * math.sqrt(math.pi)), abs=1e-15)
    c1 = math.sqrt(3 / (4 * math.pi))
    # l=1 real harmonics with the Condon-Shortley phase: -c y, c z, -c x
    np.testing.assert_allclose(Y[1:4], [-c1 * y, c1 * z, -c1 * x], atol=1e-14)
    # Y_2^0 = sqrt(5/16pi) (3z^2 - 1)
    assert Y[6] == pytest.approx(math.sqrt(5 / (16 * math.pi)) * (3 * z * z - 1), abs=1e-14)
    # Y_3^0 = sqrt(7/16pi) (5z^3 - 3z)
    assert Y[12] == pytest.approx(math.sqrt(7 / (16 * math.pi)) * (5 * z ** 3 - 3 * z), abs=1e-14)


# ----------------------------------------------------------------------------
# P1: adaptive 3D filter (Sec. 3.2)


def _cam_at(dist, w=64, h=64, fov=60.0):
    return S.pinhole((0.0, 0.0, -dist), w, h, fov)


def test_filter_isotropic_closed_form():
    """Isotropic s: alpha~ = alpha s^2 / (s^2 + a), a = k / v^2, v = f / z."""
    cam = _cam_at(4.0)
    st = S.Settings()
    for ls in (-3.0, -1.5, 0.0):
        sc = one_gaussian((0.1, -0.05, 0.2), (ls, ls, ls), (0.3, 0.1, -0.7, 0.2), 0.7)
        pp = O.preprocess(sc, cam, st)
        z = pp["mu_v"][2, 0]
        a = st.filter_k / (cam.fx / z) ** 2
        s2 = math.exp(2 * float(np.float32(ls)))
        alpha = 1 / (1 + math.exp(-float(np.float32(0.7))))
        assert pp["alpha_t"][0] == pytest.approx(alpha * s2 / (s2 + a), rel=1e-12)
        np.testing.assert_allclose(pp["s_t"][:, 0], math.sqrt(s2 + a), rtol=1e-12)


def test_filter_axis_aligned_independent_of_depth_axis():
    """d along local axis 3: alpha~ = alpha s1 s2 / sqrt((s1^2+a)(s2^2+a)), independent of s3."""
    cam = _cam_at(3.0)
    st = S.Settings()
    # identity rotation, mean on the optical axis -> d = +z = local axis 3
    vals = []
    for s3 in (-6.0, -2.0, 1.0):
        sc = one_gaussian((0.0, 0.0, 0.0), (-3.0, -2.5, s3), (1, 0, 0, 0), 0.2)
        pp = O.preprocess(sc, cam, st)
        a = st.filter_k / (cam.fx / 3.0) ** 2
        s1, s2 = math.exp(float(np.float32(-3.0))), math.exp(float(np.float32(-2.5)))
        alpha = 1 / (1 + math.exp(-float(np.float32(0.2))))
        want = alpha * s1 * s2 / math.sqrt((s1 * s1 + a) * (s2 * s2 + a))
        assert pp["alpha_t"][0] == pytest.approx(want, rel=1e-12)
        vals.append(pp["alpha_t"][0])
    assert max(vals) - min(vals) < 1e-14


def _perp_det(Sig, d):
    """det of Sigma restricted to the plane orthogonal to d, via an explicit orthonormal basis."""
    d = d / np.linalg.norm(d)
    a = np.array([1.0, 0, 0]) if abs(d[0]) < 0.9 else np.array([0, 1.0, 0])
    u2 = np.cross(d, a)
    u2 /= np.linalg.norm(u2)
    u3 = np.cross(d, u2)
    U = np.stack([u2, u3], 1)
    return np.linalg.det(U.T @ Sig @ U)


def test_filter_equals_perpendicular_determinant_ratio():
    """Eq.(12) equals sqrt(det Sigma_perp / det Sigma^_perp) (Eq.9-10, appendix A) for random Gaussians."""
    sc, cam = S.small_scene(n=200, seed=7)
    st = S.Settings()
    pp = O.preprocess(sc, cam, st)
    o = cam.position
    for i in range(200):
        mu = f64(sc.means[:, i])
        s = np.exp(f64(sc.log_scales[:, i]))
        R = rot_np(f64(sc.quats[:, i]))
        Sig = R @ np.diag(s ** 2) @ R.T
        z = (cam.viewmat[:3, :3] @ mu + cam.viewmat[:3, 3])[2]
        v = cam.fx / max(z, cam.znear)
        v = min(v, float(sc.v_train[i]))
        a = st.filter_k / v ** 2
        Sh = Sig + a * np.eye(3)
        d = mu - o
        ratio = math.sqrt(_perp_det(Sig, d) / _perp_det(Sh, d))
        alpha = 1 / (1 + math.exp(-float(sc.opacity_logits[i])))
        assert pp["alpha_t"][i] == pytest.approx(alpha * ratio, rel=1e-9)


def test_volume_normalised_variant_is_eq8():
    sc, cam = S.small_scene(n=50, seed=8)
    st = S.Settings(filter_mode=2)
    pp = O.preprocess(sc, cam, st)
    for i in range(50):
        mu = f64(sc.means[:, i])
        s = np.exp(f64(sc.log_scales[:, i]))
        R = rot_np(f64(sc.quats[:, i]))
        Sig = R @ np.diag(s ** 2) @ R.T
        z = (cam.viewmat[:3, :3] @ mu + cam.viewmat[:3, 3])[2]
        v = min(cam.fx / max(z, cam.znear), float(sc.v_train[i]))
        Sh = Sig + st.filter_k / v ** 2 * np.eye(3)
        alpha = 1 / (1 + math.exp(-float(sc.opacity_logits[i])))
        want = alpha * math.sqrt(np.linalg.det(Sig) / np.linalg.det(Sh))
        assert pp["alpha_t"][i] == pytest.approx(want, rel=1e-9)


def test_filter_preserves_perpendicular_opacity_integral():
    """P4: integral over the plane orthogonal to d of alpha * max_t G(y + t d) is
    unchanged by the filter (max along each line found by brute-force sampling)."""
    cam = _cam_at(5.0)
    st = S.Settings(filter_k=30.0)  # a large filter so the effect is visible
    mu = np.array([0.05, -0.02, 0.1])
    ls = (-1.2, -2.2, -0.6)
    q = (0.8, 0.3, -0.4, 0.2)
    sc = one_gaussian(mu, ls, q, 1.1)
    pp = O.preprocess(sc, cam, st)
    s = np.exp(f64(ls))
    R = rot_np(f64(q))
    Sig = R @ np.diag(s ** 2) @ R.T
    st_ = pp["s_t"][:, 0]
    Sh = R @ np.diag(st_ ** 2) @ R.T
    d = f64(mu) - cam.position
    d /= np.linalg.norm(d)
    a_ = np.array([1.0, 0, 0])
    u2 = np.cross(d, a_); u2 /= np.linalg.norm(u2)
    u3 = np.cross(d, u2)
    alpha = 1 / (1 + math.exp(-float(np.float32(1.1))))

    def integral(Sg, amp):
        P = np.linalg.inv(Sg)
        ext = 6 * math.sqrt(np.max(np.linalg.eigvalsh(Sg)))
        n = 161
        g = np.linspace(-ext, ext, n)
        h = g[1] - g[0]
        ts = np.linspace(-ext, ext, 801)
        tot = 0.0
        for a2 in g:
            Y = a2 * u2[None, :] + g[:, None] * u3[None, :]               # (n,3)
            X = Y[:, None, :] + ts[None, :, None] * d[None, None, :]      # (n,T,3)
            q2 = np.einsum("nti,ij,ntj->nt", X, P, X)
            tot += np.exp(-0.5 * q2.min(axis=1)).sum()
        return amp * tot * h * h

    i0 = integral(Sig, alpha)
    i1 = integral(Sh, pp["alpha_t"][0])
    assert i1 == pytest.approx(i0, rel=2e-3)
    # and the closed form 2 pi alpha sqrt(det Sigma_perp)
    assert i0 == pytest.approx(2 * math.pi * alpha * math.sqrt(_perp_det(Sig, d)), rel=2e-3)


def test_training_frequency_clamp():
    """Eq.(13): v' = min(v_train, v); zooming in stops shrinking at v_train."""
    st = S.Settings()
    vt = 50.0
    sc = one_gaussian((0, 0, 0), (-3, -3, -3), (1, 0, 0, 0), 0.0, v_train=vt)
    near = O.preprocess(sc, _cam_at(0.5), st)   # v = f/0.5 > v_train: filter fixed at k/v_train^2
    far = O.preprocess(sc, _cam_at(100.0), st)  # v < v_train: filter k/v^2
    s2 = math.exp(2 * -3.0)
    assert near["s_t"][0, 0] == pytest.approx(math.sqrt(s2 + st.filter_k / vt ** 2), rel=1e-6)
    v = _cam_at(100.0).fx / 100.0
    assert far["s_t"][0, 0] == pytest.approx(math.sqrt(s2 + st.filter_k / v ** 2), rel=1e-6)


# ----------------------------------------------------------------------------
# P2: response along a pixel line (Sec. 3.1, Eq.4-5)


def _sigma_hat(sc, pp, i):
    R = rot_np(f64(sc.quats[:, i]))
    return R @ np.diag(pp["s_t"][:, i] ** 2) @ R.T


def _pixel_dir_world(cam, x, y):
    rv = np.array([(x - cam.cx) / cam.fx, (y - cam.cy) / cam.fy, 1.0])
    return cam.viewmat[:3, :3].T @ rv


def test_ray_through_mean_gives_full_amplitude():
    cam = _cam_at(3.0, 64, 48)
    st = S.Settings()
    x, y = 40.5, 11.5
    t = 2.7
    mu = cam.position + t * _pixel_dir_world(cam, x, y)
    sc = one_gaussian(mu.astype(np.float32), (-2.0, -2.6, -1.7), (0.2, 0.9, 0.1, -0.3), 2.5)
    pp = O.preprocess(sc, cam, st)
    # the float32 rounding of mu puts it ~1e-7 off the line: rho^2 ~ 1e-12
    r2, z, a = O.eval_points(sc, cam, st, [0], [x], [y])
    assert r2[0] < 1e-9
    assert z[0] == pytest.approx(t, rel=1e-6)
    assert a[0] == pytest.approx(min(0.99, pp["alpha_t"][0]), rel=1e-9)


def test_isotropic_perpendicular_distance():
    """Isotropic filtered scale s~ at perpendicular distance b: rho^2 = b^2 / s~^2."""
    cam = _cam_at(4.0)
    st = S.Settings()
    sc = one_gaussian((0.2, 0.1, 0.3), (-2.0, -2.0, -2.0), (1, 0, 0, 0), 0.0)
    pp = O.preprocess(sc, cam, st)
    mu = f64(sc.means[:, 0])
    o = cam.position
    for (x, y) in [(30.5, 30.5), (10.5, 50.5), (0.5, 0.5)]:
        d = _pixel_dir_world(cam, x, y)
        d /= np.linalg.norm(d)
        w = mu - o
        b2 = w @ w - (w @ d) ** 2
        r2, z, a = O.eval_points(sc, cam, st, [0], [x], [y])
        assert r2[0] == pytest.approx(b2 / pp["s_t"][0, 0] ** 2, rel=1e-10)


def test_response_matches_brute_force_line_search():
    sc, cam = S.small_scene(n=40, seed=11)
    st = S.Settings()
    pp = O.preprocess(sc, cam, st)
    rng = np.random.default_rng(3)
    o = cam.position
    for i in range(40):
        Sh = _sigma_hat(sc, pp, i)
        P = np.linalg.inv(Sh)
        mu = f64(sc.means[:, i])
        x, y = rng.uniform(0, 128, 2)
        rw = _pixel_dir_world(cam, x, y)
        ts = np.linspace(-8, 8, 400001)
        X = o[None, :] + ts[:, None] * rw[None, :] - mu[None, :]
        q = np.einsum("ti,ij,tj->t", X, P, X)
        k = np.argmin(q)
        r2, z, a = O.eval_points(sc, cam, st, [i], [x], [y])
        assert r2[0] == pytest.approx(q[k], rel=1e-6, abs=1e-9)
        assert z[0] == pytest.approx(ts[k], abs=1e-4)


def test_plane_form_equals_ray_form():
    """Eq.(4)-(5): transform pi_x, pi_y by T'^T = (K V T)^T and take the origin-to-line distance."""
    sc, cam = S.small_scene(n=30, seed=12)
    st = S.Settings()
    pp = O.preprocess(sc, cam, st)
    K = np.array([[cam.fx, 0, cam.cx, 0], [0, cam.fy, cam.cy, 0], [0, 0, 1, 0], [0, 0, 0, 1.0]])
    rng = np.random.default_rng(5)
    for i in range(30):
        R = rot_np(f64(sc.quats[:, i]))
        T = np.eye(4)
        T[:3, :3] = R @ np.diag(pp["s_t"][:, i])
        T[:3, 3] = f64(sc.means[:, i])
        # rows x, y, w of the screen map; pi_x = (1,0,0,-x) acts on (x w, y w, z, w)
        Tp = K @ cam.viewmat @ T
        Tp = Tp[[0, 1, 2, 3]]
        x, y = rng.uniform(0, 128, 2)
        # screen homogeneous coordinates are rows 0,1 and w=row 2 of K V T
        pa = Tp[0] - x * Tp[2]
        pb = Tp[1] - y * Tp[2]
        na, da = pa[:3], pa[3]
        nb, db = pb[:3], pb[3]
        num = da * nb - db * na
        rho2 = (num @ num) / (np.cross(na, nb) @ np.cross(na, nb))
        r2, z, a = O.eval_points(sc, cam, st, [i], [x], [y])
        assert r2[0] == pytest.approx(rho2, rel=1e-9, abs=1e-12)


# ----------------------------------------------------------------------------
# Camera-inside discard (Sec. 3.3) and whole-frustum cull (Sec. 3.4)


def test_camera_inside_is_discarded():
    cam = _cam_at(0.05)
    st = S.Settings()
    sc = one_gaussian((0, 0, 0), (-1.0, -1.0, -1.0), (1, 0, 0, 0), 3.0)
    assert O.preprocess(sc, cam, st)["status"][0] == O.CAM_INSIDE
    sc = one_gaussian((0, 0, 0), (-5.0, -5.0, -5.0), (1, 0, 0, 0), 3.0)
    assert O.preprocess(sc, cam, st)["status"][0] == O.VISIBLE


def test_whole_frustum_cull():
    cam = _cam_at(3.0)
    st = S.Settings()
    behind = one_gaussian((0, 0, -6.0), (-2, -2, -2), (1, 0, 0, 0), 3.0)
    side = one_gaussian((30.0, 0, 0), (-2, -2, -2), (1, 0, 0, 0), 3.0)
    # a big Gaussian whose mean is outside the image but whose extent reaches in
    reach = one_gaussian((2.3, 0, 0), (0.0, -3, -3), (1, 0, 0, 0), 3.0)
    assert O.preprocess(behind, cam, st)["status"][0] == O.OUTSIDE
    assert O.preprocess(side, cam, st)["status"][0] == O.OUTSIDE
    assert O.preprocess(reach, cam, st)["status"][0] == O.VISIBLE
    low = one_gaussian((0, 0, 0), (-2, -2, -2), (1, 0, 0, 0), -7.0)
    assert O.preprocess(low, cam, st)["status"][0] == O.LOW_OPACITY


# ----------------------------------------------------------------------------
# P6: exact pyramid minimum vs dense sampling


def test_cone_min_matches_dense_sampling():
    sc, cam = S.small_scene(n=16, seed=21)
    st = S.Settings()
    pp = O.preprocess(sc, cam, st)
    rng = np.random.default_rng(9)
    RV, tV = cam.viewmat[:3, :3], cam.viewmat[:3, 3]
    checked = 0
    for i in range(16):
        Sh = _sigma_hat(sc, pp, i)
        P = np.linalg.inv(Sh)
        mu = f64(sc.means[:, i])
        tx, ty = rng.integers(0, 8, 2)
        rect = (16.0 * tx, 16.0 * tx + 16, 16.0 * ty, 16.0 * ty + 16)
        m, tau = O.cone_min(sc, cam, st, [i], [rect])
        # sample the pyramid: screen points of the rectangle x depth
        xs = rng.uniform(rect[0], rect[1], 1000)
        ys = rng.uniform(rect[2], rect[3], 1000)
        xs = np.concatenate([xs, np.repeat([rect[0], rect[1]], 100), rng.uniform(rect[0], rect[1], 200)])
        ys = np.concatenate([ys, rng.uniform(rect[2], rect[3], 200), np.repeat([rect[2], rect[3]], 100)])
        zs = np.geomspace(1e-4, 50, 200)
        rv = np.stack([(xs - cam.cx) / cam.fx, (ys - cam.cy) / cam.fy, np.ones_like(xs)], 1)
        Xv = rv[:, None, :] * zs[None, :, None]
        Xw = (Xv - tV) @ RV  # R^T (Xv - t)
        D = Xw - mu
        q = np.einsum("...i,ij,...j->...", D, P, D)
        qmin = min(q.min(), float((cam.position - mu) @ P @ (cam.position - mu)))
        assert m[0] <= qmin * (1 + 1e-9) + 1e-12
        # multi-start local search over (screen x, screen y, log depth) reaches the exact minimum
        def f(p):
            p = np.clip(p, -50, 50)
            x = rect[0] + (rect[1] - rect[0]) / (1 + math.exp(-p[0]))
            y = rect[2] + (rect[3] - rect[2]) / (1 + math.exp(-p[1]))
            Xv = np.array([(x - cam.cx) / cam.fx, (y - cam.cy) / cam.fy, 1.0]) * math.exp(p[2])
            D = RV.T @ (Xv - tV) - mu
            return D @ P @ D
        best = min(minimize(f, np.array([a, b, c]), method="Nelder-Mead",
                            options=dict(xatol=1e-10, fatol=1e-13, maxiter=20000)).fun
                   for a in (-2, 2) for b in (-2, 2) for c in (-2, 0, 2))
        assert m[0] <= best * (1 + 1e-9) + 1e-12
        assert best == pytest.approx(m[0], rel=1e-3, abs=1e-6)
        checked += 1
    assert checked == 16


def test_cone_min_zero_when_mean_inside():
    cam = _cam_at(3.0)
    st = S.Settings()
    sc = one_gaussian((0, 0, 0), (-2, -2, -2), (1, 0, 0, 0), 1.0)
    m, _ = O.cone_min(sc, cam, st, [0], [(24.0, 40.0, 24.0, 40.0)])
    assert m[0] == 0.0


# ----------------------------------------------------------------------------
# P3: angular bounds of a sphere


def test_sampled_bounds_of_sphere():
    cam = _cam_at(4.0, 128, 128, 60.0)
    st = S.Settings(filter_mode=1)
    mu = np.array([0.6, -0.3, 1.0])
    ls = -1.5
    sc = one_gaussian(mu, (ls, ls, ls), (1, 0, 0, 0), 2.0)
    pp = O.preprocess(sc, cam, st)
    st_, out = O.sampled_bounds(sc, cam, st, 0, 512, 1024)
    Rr = math.sqrt(pp["tau"][0]) * pp["s_t"][0, 0]
    mv = pp["mu_v"][:, 0]
    th = math.atan2(mv[0], mv[2])
    dth = math.asin(Rr / math.hypot(mv[0], mv[2]))
    x_lo = cam.cx + cam.fx * math.tan(th - dth)
    x_hi = cam.cx + cam.fx * math.tan(th + dth)
    assert out[0] == pytest.approx(x_lo, abs=0.05)
    assert out[1] == pytest.approx(x_hi, abs=0.05)


# ----------------------------------------------------------------------------
# P5: blending invariants and brute-force per-ray ordering


def _brute_pixel(sc, cam, st, pp, x, y):
    """Per-pixel exact depth sort (by depth of maximum response, then id) and blending."""
    n = sc.n
    r2, z, a = O.eval_points(sc, cam, st, np.arange(n), np.full(n, x), np.full(n, y))
    keep = (a >= st.alpha_min) & (z >= cam.znear) & (pp["status"] == O.VISIBLE)
    idx = np.nonzero(keep)[0]
    idx = idx[np.lexsort((idx, z[idx]))]
    T, C = 1.0, np.zeros(3)
    for i in idx:
        if T * (1 - a[i]) < st.t_min:
            break
        C += T * a[i] * pp["color"][:, i]
        T *= 1 - a[i]
    return C + T * np.asarray(cam.bg), T


def tiny_scene(seed, n=8):
    rng = np.random.default_rng(seed)
    means = rng.uniform(-0.4, 0.4, size=(3, n))
    sc = S.Scene(
        means=means.astype(np.float32),
        log_scales=rng.normal(-1.6, 0.3, size=(3, n)).astype(np.float32),
        quats=rng.normal(size=(4, n)).astype(np.float32),
        opacity_logits=rng.normal(1.0, 1.0, size=n).astype(np.float32),
        sh=((rng.uniform(0, 1, size=(1, 3, n)) - 0.5) / S.SH_C0).astype(np.float32),
    )
    cam = S.pinhole((0.3, -0.2, -2.5), 16, 16, 50.0, bg=(0.1, 0.2, 0.3))
    return sc, cam


@pytest.mark.parametrize("seed", range(6))
def test_large_window_equals_brute_force_per_ray_sort(seed):
    sc, cam = tiny_scene(seed)
    st = S.Settings(ray_window=64)
    pp = O.preprocess(sc, cam, st)
    r = O.render(sc, cam, st)
    for py in range(16):
        for px in range(16):
            if r.flags[py, px]:
                continue
            C, T = _brute_pixel(sc, cam, st, pp, px + 0.5, py + 0.5)
            np.testing.assert_allclose(r.rgb[:, py, px], C, atol=1e-12)
            assert r.T[py, px] == pytest.approx(T, abs=1e-12)


@pytest.mark.parametrize("K", [0, 1, 4, 16])
def test_transmittance_monotone_and_white_identity(K):
    sc, cam = S.small_scene(n=400, seed=31)
    sc.sh[:] = 0
    sc.sh[0] = (1.0 - 0.5) / S.SH_C0  # white
    cam.bg = (0.0, 0.0, 0.0)
    st = S.Settings(ray_window=K)
    r = O.render(sc, cam, st)
    assert np.all(r.T <= 1) and np.all(r.T >= st.t_min * (1 - 1e-12))
    # sum_i a_i T_i + T_final = 1 -> white on black gives C = 1 - T
    np.testing.assert_allclose(r.rgb[0], 1 - r.T, atol=1e-12)
    np.testing.assert_allclose(r.rgb[1], 1 - r.T, atol=1e-12)


def test_window_of_one_equals_full_sort_when_tile_order_is_pixel_order():
    """Gaussians at well separated depths straight ahead: tile order = pixel order, so K=1 == K=64 == K=0."""
    n = 6
    rng = np.random.default_rng(4)
    means = np.stack([rng.uniform(-0.1, 0.1, n), rng.uniform(-0.1, 0.1, n), np.linspace(-1.0, 1.0, n)])
    sc = S.Scene(means.astype(np.float32), np.full((3, n), -1.2, np.float32), np.tile([[1], [0], [0], [0]], n).astype(np.float32),
                 np.full(n, 0.0, np.float32), ((rng.uniform(0, 1, (1, 3, n)) - 0.5) / S.SH_C0).astype(np.float32))
    cam = S.pinhole((0.0, 0.0, -4.0), 32, 32, 40.0)
    imgs = [O.render(sc, cam, S.Settings(ray_window=K)).rgb for K in (0, 1, 64)]
    np.testing.assert_allclose(imgs[0], imgs[2], atol=1e-13)
    np.testing.assert_allclose(imgs[1], imgs[2], atol=1e-13)


def test_single_gaussian_image_closed_form():
    """One Gaussian: pixel = min(0.99, alpha~ exp(-rho^2/2)) c + (1 - a) bg, rho^2 from Sigma^-1 directly."""
    cam = S.pinhole((0.2, 0.1, -3.0), 48, 40, 55.0, bg=(0.2, 0.0, 0.5))
    st = S.Settings()
    mu = np.array([0.1, -0.05, 0.2])
    q = (0.9, -0.2, 0.3, 0.1)
    sc = one_gaussian(mu, (-1.8, -2.4, -1.5), q, 1.7, colour=(0.8, 0.4, 0.1))
    pp = O.preprocess(sc, cam, st)
    r = O.render(sc, cam, st)
    R = rot_np(f64(q))
    P = np.linalg.inv(R @ np.diag(pp["s_t"][:, 0] ** 2) @ R.T)
    o = cam.position
    m = f64(sc.means[:, 0])
    bg = np.asarray(cam.bg)
    for py in range(0, 40, 3):
        for px in range(0, 48, 3):
            if r.flags[py, px]:
                continue
            d = _pixel_dir_world(cam, px + 0.5, py + 0.5)
            w = o - m
            t = -(d @ P @ w) / (d @ P @ d)
            X = w + t * d
            r2 = X @ P @ X
            a = min(0.99, pp["alpha_t"][0] * math.exp(-0.5 * r2))
            want = bg.copy()
            if a >= st.alpha_min and t >= cam.znear:
                want = a * pp["color"][:, 0] + (1 - a) * bg
            np.testing.assert_allclose(r.rgb[:, py, px], want, atol=1e-12)


def test_colour_clamped_at_zero_and_dc_encoding():
    cam = _cam_at(3.0)
    st = S.Settings()
    sc = one_gaussian((0, 0, 0), (-2, -2, -2), (1, 0, 0, 0), 0.0, colour=(0.25, 0.5, 1.0))
    pp = O.preprocess(sc, cam, st)
    np.testing.assert_allclose(pp["color"][:, 0], [0.25, 0.5, 1.0], rtol=1e-6)
    sc.sh[0, 0, 0] = -10.0
    assert O.preprocess(sc, cam, st)["color"][0, 0] == 0.0


def test_invalid_inputs_are_culled():
    cam = _cam_at(3.0)
    st = S.Settings()
    sc = one_gaussian((0, np.nan, 0), (-2, -2, -2), (1, 0, 0, 0), 0.0)
    assert O.preprocess(sc, cam, st)["status"][0] == O.INVALID
    sc = one_gaussian((0, 0, 0), (-2, -2, -2), (0, 0, 0, 0), 0.0)
    assert O.preprocess(sc, cam, st)["status"][0] == O.INVALID
