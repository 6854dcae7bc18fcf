"""ctypes front-end of the FP64 CPU oracle (aaa_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.

Inputs are duck-typed scene/camera/settings objects (attributes as in the
seeded input generators); outputs are float64 numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "aaa_oracle.c")
LIB = os.path.join(HERE, "liboracle_aaa.so")

VISIBLE, INVALID, LOW_OPACITY, CAM_INSIDE, OUTSIDE = 0, 1, 2, 3, 4

# Relative bands inside which an FP32 implementation may take a threshold
# decision the other way; pixels touched by such a decision are flagged.
# The termination band is an error bound accumulated per pixel from
# BAND_ALPHA over the blended entries (aaa_oracle.c, blend_one); BAND_T is
# its floor.
BAND_ALPHA = 3e-5
BAND_Z = 1e-5
BAND_TIE = 2e-6
BAND_T = 1e-5


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no fused multiply-add, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", tmp,
                               SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Scene(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("_pad", C.c_int32),
                ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p), ("v_train", C.c_void_p)]


class _Camera(C.Structure):
    _fields_ = [("viewmat", C.c_double * 16), ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double),
                ("cy", C.c_double), ("width", C.c_int32), ("height", C.c_int32), ("znear", C.c_double),
                ("bg", C.c_double * 3)]


class _Settings(C.Structure):
    _fields_ = [("filter_k", C.c_double), ("ray_window", C.c_int32), ("filter_mode", C.c_int32),
                ("alpha_min", C.c_double), ("alpha_max", C.c_double), ("t_min", C.c_double),
                ("band_alpha", C.c_double), ("band_z", C.c_double), ("band_tie", C.c_double), ("band_T", C.c_double),
                ("subtile_sort", C.c_int32), ("_pad", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("n_visible", C.c_int64), ("n_candidates_total", C.c_int64), ("n_contrib_total", C.c_int64),
                ("n_blended_total", C.c_int64), ("n_flagged", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
    return _lib


def _f64(a):
    # float32 inputs convert exactly; float64 inputs (finite differences) pass through
    return np.ascontiguousarray(a, dtype=np.float64)


class _SceneHolder:
    def __init__(self, scene):
        self.arrays = [_f64(scene.means), _f64(scene.log_scales), _f64(scene.quats), _f64(scene.opacity_logits),
                       _f64(scene.sh)]
        self.vt = None if scene.v_train is None else _f64(scene.v_train)
        n = self.arrays[0].shape[1]
        nb = self.arrays[4].shape[0]
        deg = int(round(np.sqrt(nb))) - 1
        assert (deg + 1) ** 2 == nb and 0 <= deg <= 3
        ptr = lambda a: a.ctypes.data_as(C.c_void_p)
        self.s = _Scene(n, deg, 0, *(ptr(a) for a in self.arrays), None if self.vt is None else ptr(self.vt))


def _camera(cam) -> _Camera:
    c = _Camera()
    vm = np.asarray(cam.viewmat, np.float64).reshape(16)
    for i in range(16):
        c.viewmat[i] = vm[i]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height, c.znear = int(cam.width), int(cam.height), float(cam.znear)
    for i in range(3):
        c.bg[i] = float(cam.bg[i])
    return c


def _settings(st) -> _Settings:
    s = _Settings()
    s.filter_k = float(st.filter_k)
    s.ray_window = int(st.ray_window)
    s.filter_mode = int(st.filter_mode)
    s.alpha_min, s.alpha_max, s.t_min = float(st.alpha_min), float(st.alpha_max), float(st.t_min)
    s.band_alpha, s.band_z, s.band_tie, s.band_T = BAND_ALPHA, BAND_Z, BAND_TIE, BAND_T
    s.subtile_sort = int(bool(getattr(st, "subtile_sort", False)))
    return s


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


@dataclass
class RenderResult:
    rgb: np.ndarray       # (3, H, W)
    T: np.ndarray         # (H, W)
    flags: np.ndarray     # (H, W) uint8
    ncontrib: np.ndarray  # (H, W) int32
    n_visible: int
    n_candidates: int
    n_contrib: int
    n_blended: int
    n_flagged: int


def render(scene, cam, settings, tile_sel=None) -> RenderResult:
    """Plain per-pixel FP64 render (rgb, final transmittance, flags)."""
    L = lib()
    sh = _SceneHolder(scene)
    c, s = _camera(cam), _settings(settings)
    H, W = int(cam.height), int(cam.width)
    rgb = np.zeros((3, H, W))
    T = np.zeros((H, W))
    flags = np.zeros((H, W), np.uint8)
    ncon = np.zeros((H, W), np.int32)
    stats = _Stats()
    sel = None
    if tile_sel is not None:
        sel = np.ascontiguousarray(tile_sel, dtype=np.uint8)
    L.or_render.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Settings), C.c_void_p, C.c_void_p,
                            C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(_Stats)]
    rc = L.or_render(C.byref(sh.s), C.byref(c), C.byref(s), None if sel is None else _p(sel), _p(rgb), _p(T),
                     _p(flags), _p(ncon), C.byref(stats))
    assert rc == 0
    return RenderResult(rgb, T, flags, ncon, stats.n_visible, stats.n_candidates_total, stats.n_contrib_total,
                        stats.n_blended_total, stats.n_flagged)


def render_alternatives(scene, cam, settings, pixels, tile_sel=None):
    """Alternative outcomes of the given pixels ((y, x) pairs): every flagged
    decision of a pixel taken the other way, one at a time (see
    pixel_alternatives in aaa_oracle.c).  Returns a list, per pixel, of an
    array [n_alt, 4] (r, g, b, T)."""
    L = lib()
    sh = _SceneHolder(scene)
    c, s = _camera(cam), _settings(settings)
    H, W = int(cam.height), int(cam.width)
    pixels = np.asarray(pixels, np.int64).reshape(-1, 2)
    slot = np.full((H, W), -1, np.int32)
    slot[pixels[:, 0], pixels[:, 1]] = np.arange(len(pixels), dtype=np.int32)
    ma = int(L.or_max_alternatives())
    out = np.zeros((max(len(pixels), 1), ma, 4))
    na = np.zeros(max(len(pixels), 1), np.int32)
    if len(pixels):
        sel = None if tile_sel is None else np.ascontiguousarray(tile_sel, dtype=np.uint8)
        L.or_render_alternatives.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Settings), C.c_void_p,
                                             C.c_void_p, C.c_void_p, C.c_void_p]
        rc = L.or_render_alternatives(C.byref(sh.s), C.byref(c), C.byref(s), None if sel is None else _p(sel),
                                      _p(slot), _p(out), _p(na))
        assert rc == 0
    return [out[k, : na[k]] for k in range(len(pixels))]


def preprocess(scene, cam, settings) -> dict:
    L = lib()
    sh = _SceneHolder(scene)
    c, s = _camera(cam), _settings(settings)
    n = sh.s.n
    out = dict(status=np.zeros(n, np.int32), ambiguous=np.zeros(n, np.int32), alpha_t=np.zeros(n), tau=np.zeros(n),
               s_t=np.zeros((3, n)), color=np.zeros((3, n)), mu_v=np.zeros((3, n)), og2=np.zeros(n))
    L.or_preprocess.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Settings)] + [C.c_void_p] * 8
    rc = L.or_preprocess(C.byref(sh.s), C.byref(c), C.byref(s), *(_p(out[k]) for k in
                                                                   ("status", "ambiguous", "alpha_t", "tau", "s_t",
                                                                    "color", "mu_v", "og2")))
    assert rc == 0
    return out


def eval_points(scene, cam, settings, ids, xs, ys):
    """rho^2, depth of maximum response and alpha for (gaussian, x, y) queries."""
    L = lib()
    sh = _SceneHolder(scene)
    c, s = _camera(cam), _settings(settings)
    ids = np.ascontiguousarray(ids, np.int64)
    xs = np.ascontiguousarray(xs, np.float64)
    ys = np.ascontiguousarray(ys, np.float64)
    nq = len(ids)
    r2, z, a = np.zeros(nq), np.zeros(nq), np.zeros(nq)
    L.or_eval_points.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Settings), C.c_int64] + [C.c_void_p] * 6
    L.or_eval_points(C.byref(sh.s), C.byref(c), C.byref(s), nq, _p(ids), _p(xs), _p(ys), _p(r2), _p(z), _p(a))
    return r2, z, a


def cone_min(scene, cam, settings, ids, rects):
    """Exact minimum of rho^2 over the pyramid of each screen rectangle (x0,x1,y0,y1)."""
    L = lib()
    sh = _SceneHolder(scene)
    c, s = _camera(cam), _settings(settings)
    ids = np.ascontiguousarray(ids, np.int64)
    rects = np.ascontiguousarray(rects, np.float64).reshape(-1, 4)
    nq = len(ids)
    m, tau = np.zeros(nq), np.zeros(nq)
    L.or_cone_min_query.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Settings), C.c_int64] + [C.c_void_p] * 4
    L.or_cone_min_query(C.byref(sh.s), C.byref(c), C.byref(s), nq, _p(ids), _p(rects), _p(m), _p(tau))
    return m, tau


def classify_pairs(scene, cam, settings, tile, ids):
    """0 not allowed, 1 allowed but not needed, 2 needed, 3 exempt (near a threshold)."""
    L = lib()
    sh = _SceneHolder(scene)
    c, s = _camera(cam), _settings(settings)
    ids = np.ascontiguousarray(ids, np.int64)
    out = np.zeros(len(ids), np.int32)
    L.or_classify_pairs.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Settings), C.c_int32, C.c_int64,
                                    C.c_void_p, C.c_void_p]
    L.or_classify_pairs(C.byref(sh.s), C.byref(c), C.byref(s), int(tile), len(ids), _p(ids), _p(out))
    return out


def sampled_bounds(scene, cam, settings, i, nt=256, np_=512):
    L = lib()
    sh = _SceneHolder(scene)
    c, s = _camera(cam), _settings(settings)
    out = np.zeros(4)
    L.or_sampled_bounds.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Settings), C.c_int64, C.c_int,
                                    C.c_int, C.c_void_p]
    st = L.or_sampled_bounds(C.byref(sh.s), C.byref(c), C.byref(s), int(i), nt, np_, _p(out))
    return st, out


def sampled_bounds_many(scene, cam, settings, ids, nt=256, np_=512):
    """sampled_bounds for several Gaussians: (status [q], bounds [q, 4])."""
    L = lib()
    sh = _SceneHolder(scene)
    c, s = _camera(cam), _settings(settings)
    ids = np.ascontiguousarray(ids, np.int64)
    out = np.zeros((len(ids), 4))
    st = np.zeros(len(ids), np.int32)
    L.or_sampled_bounds_many.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Settings), C.c_int64,
                                         C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    L.or_sampled_bounds_many(C.byref(sh.s), C.byref(c), C.byref(s), len(ids), _p(ids), nt, np_, _p(out), _p(st))
    return st, out


def sh_basis(degree, direction):
    L = lib()
    d = np.ascontiguousarray(direction, np.float64)
    Y = np.zeros(16)
    L.or_sh_basis.argtypes = [C.c_int, C.c_void_p, C.c_void_p]
    L.or_sh_basis(int(degree), _p(d), _p(Y))
    return Y[: (degree + 1) ** 2]


def rotation(q):
    L = lib()
    qq = np.ascontiguousarray(q, np.float64)
    R = np.zeros(9)
    L.or_rotation.argtypes = [C.c_void_p, C.c_void_p]
    L.or_rotation(_p(qq), _p(R))
    return R.reshape(3, 3)


def num_threads() -> int:
    return int(lib().or_num_threads())


def sh_basis_poly(degree, direction):
    """Polynomial-form real SH (the form the gradient chain uses)."""
    L = lib()
    d = np.ascontiguousarray(direction, np.float64)
    Y = np.zeros(16)
    L.or_sh_basis_poly.argtypes = [C.c_int, C.c_void_p, C.c_void_p]
    L.or_sh_basis_poly(int(degree), _p(d), _p(Y))
    return Y[: (degree + 1) ** 2]


def gauss_values(scene, cam, settings, i, complex_chain=False):
    """o_g (3), A (9), alpha~, colour (3) of Gaussian i, from the real
    preparation or from the complex-arithmetic chain used for gradients."""
    L = lib()
    sh = _SceneHolder(scene)
    c, s = _camera(cam), _settings(settings)
    out = np.zeros(16)
    f = L.or_cont_values if complex_chain else L.or_prepare_values
    f.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Settings), C.c_int64, C.c_void_p]
    st = f(C.byref(sh.s), C.byref(c), C.byref(s), int(i), _p(out))
    return out, st


@dataclass
class GradResult:
    rgb: np.ndarray
    T: np.ndarray
    flags: np.ndarray
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray


def render_backward(scene, cam, settings, dL_drgb) -> GradResult:
    """FP64 gradient of sum(dL_drgb * rgb) w.r.t. every scene parameter
    (decisions held fixed)."""
    L = lib()
    sh = _SceneHolder(scene)
    c, s = _camera(cam), _settings(settings)
    H, W = int(cam.height), int(cam.width)
    g = np.ascontiguousarray(dL_drgb, np.float64).reshape(3, H, W)
    n = sh.s.n
    nb = (sh.s.sh_degree + 1) ** 2
    rgb, T = np.zeros((3, H, W)), np.zeros((H, W))
    flags = np.zeros((H, W), np.uint8)
    gm, gl, gq, go, gs = np.zeros((3, n)), np.zeros((3, n)), np.zeros((4, n)), np.zeros(n), np.zeros((nb, 3, n))
    L.or_render_backward.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Settings)] + [C.c_void_p] * 9
    rc = L.or_render_backward(C.byref(sh.s), C.byref(c), C.byref(s), _p(g), _p(rgb), _p(T), _p(flags), _p(gm),
                              _p(gl), _p(gq), _p(go), _p(gs))
    assert rc == 0
    return GradResult(rgb, T, flags, gm, gl, gq, go, gs)


def training_frequency(means, cams):
    """Training sampling frequency per Gaussian (Sec. 3.2): the maximum of
    fx / depth over the cameras that see the mean (fallback: cameras with the
    mean in front of the near plane; else +inf).  Returns (values float64 [n],
    flags uint8 [n]); a flag marks a frustum decision within 1e-9 of its
    boundary."""
    m = _f64(means)
    n = m.shape[1]
    arr = (_Camera * max(len(cams), 1))(*[_camera(c) for c in cams])
    out = np.empty(n, np.float64)
    fl = np.zeros(n, np.uint8)
    lib().or_training_frequency(_p(m), C.c_int64(n), C.c_int(len(cams)), arr, _p(out), _p(fl))
    return out, fl


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """Adam with bias correction (Kingma & Ba, Algorithm 1), FP64: returns the
    new (p, m, v) for step t (counting from 1)."""
    p, g, m, v = (np.asarray(a, np.float64) for a in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
