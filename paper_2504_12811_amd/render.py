"""Python front-end: device scenes, the rasteriser object and autograd.

PyTorch provides device memory and streams only; every step of the path
runs in libaaa_hip.so through the C ABI.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib as L


@dataclass
class DeviceScene:
    """Scene tensors on the GPU, float32 structure-of-arrays (see include/aaa.h)."""
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    opacity_logits: torch.Tensor
    sh: torch.Tensor
    v_train: Optional[torch.Tensor] = None

    @classmethod
    def from_host(cls, scene, device="cuda") -> "DeviceScene":
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(device)
        return cls(t(scene.means), t(scene.log_scales), t(scene.quats), t(scene.opacity_logits), t(scene.sh),
                   None if scene.v_train is None else t(scene.v_train))

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    @property
    def sh_degree(self) -> int:
        return int(round(self.sh.shape[0] ** 0.5)) - 1

    def tensors(self):
        return [self.means, self.log_scales, self.quats, self.opacity_logits, self.sh]

    def abi(self) -> L.Scene:
        for t in self.tensors() + ([self.v_train] if self.v_train is not None else []):
            if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("scene tensors must be contiguous float32 CUDA tensors")
        s = L.Scene()
        s.n = self.n
        s.sh_degree = self.sh_degree
        s.means, s.log_scales, s.quats = self.means.data_ptr(), self.log_scales.data_ptr(), self.quats.data_ptr()
        s.opacity_logits, s.sh = self.opacity_logits.data_ptr(), self.sh.data_ptr()
        s.v_train = None if self.v_train is None else self.v_train.data_ptr()
        return s


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Workspace:
    """A 256-byte-aligned slice of device memory sized for one frame."""

    def __init__(self, device, nbytes: int, max_pairs: int):
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.buf.data_ptr()) % 256
        self.view = self.buf[off: off + nbytes]
        self.nbytes = nbytes
        self.max_pairs = max_pairs

    @property
    def ptr(self) -> int:
        return self.view.data_ptr()


class Rasterizer:
    """Owns a library context and a growable workspace on one device."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        ctx = C.c_void_p()
        L.check(L.lib().aaa_create(C.byref(ctx), int(device)))
        self._ctx = ctx
        self._ws: Optional[Workspace] = None
        self.last_ws: Optional[Workspace] = None
        self.max_pairs = 0
        self.last_pairs = 0

    def __del__(self):
        try:
            if getattr(self, "_ctx", None):
                L.lib().aaa_destroy(self._ctx)
        except Exception:
            pass

    # workspace --------------------------------------------------------
    def workspace_bytes(self, sc: L.Scene, cam: L.Camera, st: L.Settings, max_pairs: int) -> int:
        need = C.c_size_t()
        L.check(L.lib().aaa_workspace_size(C.byref(sc), C.byref(cam), C.byref(st), max_pairs, C.byref(need)))
        return int(need.value)

    def _fit(self, ws: Optional[Workspace], sc, cam, st, max_pairs) -> Workspace:
        need = self.workspace_bytes(sc, cam, st, max_pairs)
        if ws is not None and ws.nbytes >= need:
            ws.max_pairs = max_pairs
            return ws
        return Workspace(self.device, int(need * 1.1) + 4096, max_pairs)

    # forward ------------------------------------------------------------
    def render(self, scene: DeviceScene, cam, settings, stats: bool = False, timing: bool = False,
               max_pairs: Optional[int] = None, ws: Optional[Workspace] = None, fresh_ws: bool = False,
               flags: int = 0):
        """Render one view; returns (rgb [3,H,W], T [H,W], Stats).  Uses the
        rasteriser's own workspace unless `ws` is given or `fresh_ws` asks for
        a new one; the frame state stays in that workspace (`last_ws`), e.g.
        for a later backward."""
        sc = scene.abi()
        c = L.make_camera(cam)
        st = L.make_settings(settings, (L.AAA_STATS if stats else 0) | (L.AAA_TIMING if timing else 0) | flags)
        H, W = int(cam.height), int(cam.width)
        rgb = torch.empty((3, H, W), dtype=torch.float32, device=self.device)
        T = torch.empty((H, W), dtype=torch.float32, device=self.device)
        own = ws is None and not fresh_ws
        cur = self._ws if own else ws
        mp = max_pairs or max(cur.max_pairs if cur is not None else 0, self.max_pairs, 8 * max(scene.n, 1), 1 << 16)
        for _ in range(4):
            new = self._fit(cur, sc, c, st, mp)
            if new is not cur and cur is not None and own:
                torch.cuda.current_stream(self.device).synchronize()
            cur = new
            if own:
                self._ws = cur
            out = L.Stats()
            rc = L.lib().aaa_render(self._ctx, C.byref(sc), C.byref(c), C.byref(st), cur.ptr, cur.nbytes, mp,
                                    _stream_ptr(self.device), rgb.data_ptr(), T.data_ptr(), C.byref(out))
            if rc == L.AAA_ERR_PAIR_OVERFLOW:
                mp = min(int(out.pairs * 1.25) + 1024, (1 << 32) - 1)
                continue
            L.check(rc)
            self.last_pairs = int(out.pairs)
            self.max_pairs = max(self.max_pairs, mp)
            self.last_ws = cur
            return rgb, T, out
        raise L.AAAError(L.AAA_ERR_PAIR_OVERFLOW, "pair buffer kept overflowing")

    def batch_pair_capacity(self, scene: DeviceScene, cams, settings, nbytes: int) -> int:
        """The largest max_pairs whose workspace for this batch fits in
        `nbytes` (0 if not even an empty pair buffer fits).  The workspace
        grows linearly with max_pairs."""
        sc = scene.abi()
        V = len(cams)
        carr = (L.Camera * V)(*[L.make_camera(c) for c in cams])
        st = L.make_settings(settings)
        a, b = C.c_size_t(), C.c_size_t()
        m1 = 1 << 20
        L.check(L.lib().aaa_workspace_size_batch(C.byref(sc), V, carr, C.byref(st), 1, C.byref(a)))
        L.check(L.lib().aaa_workspace_size_batch(C.byref(sc), V, carr, C.byref(st), m1 + 1, C.byref(b)))
        if a.value > nbytes:
            return 0
        per = (b.value - a.value) / m1
        mp = min(int((nbytes - a.value) / per), (1 << 32) - 1)
        while mp > 1:  # alignment padding: step down until it fits
            L.check(L.lib().aaa_workspace_size_batch(C.byref(sc), V, carr, C.byref(st), mp, C.byref(a)))
            if a.value <= nbytes:
                break
            mp -= max(1, mp // 1000)
        return mp

    def render_batch(self, scene: DeviceScene, cams, settings, stats: bool = False, max_pairs: Optional[int] = None,
                     fresh_ws: bool = False, flags: int = 0, ws: Optional[Workspace] = None):
        """Render several views of one scene in one launch sequence; returns
        ([rgb_v], [T_v], Stats).  Each view equals its single-view render.
        With `ws` (and max_pairs) the batch renders into that workspace and
        nothing is allocated beyond the output images: a batch that does not
        fit raises AAAError (AAA_ERR_WORKSPACE or AAA_ERR_PAIR_OVERFLOW)."""
        sc = scene.abi()
        V = len(cams)
        carr = (L.Camera * V)(*[L.make_camera(c) for c in cams])
        st = L.make_settings(settings, (L.AAA_STATS if stats else 0) | flags)
        rgbs = [torch.empty((3, int(c.height), int(c.width)), dtype=torch.float32, device=self.device) for c in cams]
        Ts = [torch.empty((int(c.height), int(c.width)), dtype=torch.float32, device=self.device) for c in cams]
        prgb = (C.c_void_p * V)(*[t.data_ptr() for t in rgbs])
        pT = (C.c_void_p * V)(*[t.data_ptr() for t in Ts])
        if ws is not None:
            mp = max_pairs if max_pairs is not None else ws.max_pairs
            out = L.Stats()
            L.check(L.lib().aaa_render_batch(self._ctx, C.byref(sc), V, carr, C.byref(st), ws.ptr, ws.nbytes, mp,
                                             _stream_ptr(self.device), prgb, pT, C.byref(out)))
            self.last_pairs = int(out.pairs)
            self.last_ws = ws
            ws.max_pairs = mp
            return rgbs, Ts, out
        own = not fresh_ws
        cur = self._ws if own else None
        npix = sum(int(c.width) * int(c.height) for c in cams)
        mp = max_pairs or max(self.max_pairs, 2 * npix, 1 << 16)
        for _ in range(4):
            need = C.c_size_t()
            L.check(L.lib().aaa_workspace_size_batch(C.byref(sc), V, carr, C.byref(st), mp, C.byref(need)))
            if cur is None or cur.nbytes < need.value:
                if cur is not None and own:
                    torch.cuda.current_stream(self.device).synchronize()
                cur = Workspace(self.device, int(need.value * 1.1) + 4096, mp)
            cur.max_pairs = mp
            if own:
                self._ws = cur
            out = L.Stats()
            rc = L.lib().aaa_render_batch(self._ctx, C.byref(sc), V, carr, C.byref(st), cur.ptr, cur.nbytes, mp,
                                          _stream_ptr(self.device), prgb, pT, C.byref(out))
            if rc == L.AAA_ERR_PAIR_OVERFLOW:
                mp = min(int(out.pairs * 1.25) + 1024, (1 << 32) - 1)
                continue
            L.check(rc)
            self.last_pairs = int(out.pairs)
            self.max_pairs = max(self.max_pairs, mp)
            self.last_ws = cur
            return rgbs, Ts, out
        raise L.AAAError(L.AAA_ERR_PAIR_OVERFLOW, "pair buffer kept overflowing")

    def backward_batch(self, scene: DeviceScene, cams, settings, ws: Workspace, out_rgbs, grad_rgbs,
                       flags: int = 0) -> dict:
        """Gradients of sum_v sum(grad_rgbs[v] * rgb_v) for the batch held in `ws`."""
        sc = scene.abi()
        V = len(cams)
        carr = (L.Camera * V)(*[L.make_camera(c) for c in cams])
        st = L.make_settings(settings, flags)
        grads = {k: torch.zeros_like(t) for k, t in zip(["means", "log_scales", "quats", "opacity_logits", "sh"],
                                                        scene.tensors())}
        g = L.SceneGrad()
        g.means, g.log_scales, g.quats = grads["means"].data_ptr(), grads["log_scales"].data_ptr(), grads["quats"].data_ptr()
        g.opacity_logits, g.sh = grads["opacity_logits"].data_ptr(), grads["sh"].data_ptr()
        grs = [t.contiguous().float() for t in grad_rgbs]
        prgb = (C.c_void_p * V)(*[t.data_ptr() for t in out_rgbs])
        pg = (C.c_void_p * V)(*[t.data_ptr() for t in grs])
        scr, nscr = self._backward_scratch(sc, V, carr, st, ws)
        L.check(L.lib().aaa_render_backward_batch(self._ctx, C.byref(sc), V, carr, C.byref(st), ws.ptr, ws.nbytes,
                                                  ws.max_pairs, _stream_ptr(self.device), prgb, pg, scr, nscr,
                                                  C.byref(g)))
        return grads

    def _backward_scratch(self, sc, V, carr, st, ws: Workspace):
        need = C.c_size_t()
        L.check(L.lib().aaa_backward_scratch_size(self._ctx, C.byref(sc), V, carr, C.byref(st), ws.ptr, ws.nbytes,
                                                  ws.max_pairs, _stream_ptr(self.device), C.byref(need)))
        buf = getattr(self, "_bwd_scratch", None)
        if buf is None or buf.numel() < need.value + 256:
            self._bwd_scratch = buf = torch.empty(int(need.value * 1.2) + 512, dtype=torch.uint8, device=self.device)
        ptr = buf.data_ptr() + ((-buf.data_ptr()) % 256)
        return ptr, int(need.value)

    def backward(self, scene: DeviceScene, cam, settings, ws: Workspace, out_rgb: torch.Tensor,
                 grad_rgb: torch.Tensor, flags: int = 0) -> dict:
        """Gradients of sum(grad_rgb * rgb) for the frame held in `ws`."""
        sc = scene.abi()
        c = L.make_camera(cam)
        st = L.make_settings(settings, flags)
        grads = {k: torch.zeros_like(t) for k, t in zip(["means", "log_scales", "quats", "opacity_logits", "sh"],
                                                        scene.tensors())}
        g = L.SceneGrad()
        g.means, g.log_scales, g.quats = grads["means"].data_ptr(), grads["log_scales"].data_ptr(), grads["quats"].data_ptr()
        g.opacity_logits, g.sh = grads["opacity_logits"].data_ptr(), grads["sh"].data_ptr()
        gr = grad_rgb.contiguous().float()
        scr, nscr = self._backward_scratch(sc, 1, C.pointer(c), st, ws)
        L.check(L.lib().aaa_render_backward(self._ctx, C.byref(sc), C.byref(c), C.byref(st), ws.ptr, ws.nbytes,
                                            ws.max_pairs, _stream_ptr(self.device), out_rgb.data_ptr(), gr.data_ptr(),
                                            scr, nscr, C.byref(g)))
        return grads

    def training_frequency(self, means: torch.Tensor, cams) -> torch.Tensor:
        """Per-Gaussian training sampling frequency over `cams` (float32 [n]);
        means: device float32 [3, n]."""
        m = means.contiguous().float()
        assert m.is_cuda and m.dim() == 2 and m.shape[0] == 3
        n = m.shape[1]
        out = torch.empty(n, dtype=torch.float32, device=m.device)
        arr = (L.Camera * max(len(cams), 1))(*[L.make_camera(c) for c in cams])
        L.check(L.lib().aaa_training_frequency(self._ctx, m.data_ptr(), n, arr, len(cams), _stream_ptr(self.device),
                                               out.data_ptr()))
        return out

    def stage_times(self, reset: bool = True):
        """(dict stage -> accumulated ms, frames) of the renders made with timing=True."""
        ms = (C.c_double * len(L.STAGES))()
        frames = C.c_uint64()
        L.check(L.lib().aaa_stage_times(self._ctx, ms, C.byref(frames), int(reset)))
        return {k: ms[i] for i, k in enumerate(L.STAGES)}, int(frames.value)

    def read_gaussians(self, scene: DeviceScene, cam):
        n = scene.n
        dev = self.device
        status = torch.empty(n, dtype=torch.int32, device=dev)
        alpha_t = torch.empty(n, dtype=torch.float32, device=dev)
        tau = torch.empty(n, dtype=torch.float32, device=dev)
        color = torch.empty((3, n), dtype=torch.float32, device=dev)
        rect = torch.empty((4, n), dtype=torch.int32, device=dev)
        ws = self.last_ws
        L.check(L.lib().aaa_read_gaussians(C.byref(scene.abi()), C.byref(L.make_camera(cam)), ws.max_pairs,
                                           ws.ptr, ws.nbytes, _stream_ptr(dev), status.data_ptr(),
                                           alpha_t.data_ptr(), tau.data_ptr(), color.data_ptr(), rect.data_ptr()))
        return dict(status=status, alpha_t=alpha_t, tau=tau, color=color, rect=rect)

    def read_pairs(self, scene: DeviceScene, cam):
        dev = self.device
        cap = max(self.last_pairs, 1)
        keys = torch.empty(cap, dtype=torch.int64, device=dev)
        vals = torch.empty(cap, dtype=torch.int32, device=dev)
        tx, ty = (int(cam.width) + 15) // 16, (int(cam.height) + 15) // 16
        ranges = torch.empty((tx * ty, 2), dtype=torch.int32, device=dev)
        n = C.c_uint64()
        ws = self.last_ws
        L.check(L.lib().aaa_read_pairs(C.byref(scene.abi()), C.byref(L.make_camera(cam)), ws.max_pairs,
                                       ws.ptr, ws.nbytes, _stream_ptr(dev), keys.data_ptr(),
                                       vals.data_ptr(), ranges.data_ptr(), cap, C.byref(n)))
        P = int(n.value)
        return keys[:P], vals[:P], ranges


def sort_pairs(keys: torch.Tensor, vals: torch.Tensor, key_bits: int):
    """Stable radix sort in place of int64 keys (as uint64 bit patterns) and int32 values."""
    assert keys.is_cuda and vals.is_cuda and keys.dtype == torch.int64 and vals.dtype == torch.int32
    n = keys.numel()
    need = C.c_size_t()
    L.check(L.lib().aaa_sort_tmp_size(n, C.byref(need)))
    buf = torch.empty(need.value + 256, dtype=torch.uint8, device=keys.device)
    off = (-buf.data_ptr()) % 256
    L.check(L.lib().aaa_sort_pairs(keys.data_ptr(), vals.data_ptr(), n, int(key_bits), buf.data_ptr() + off,
                                   need.value, _stream_ptr(keys.device)))
    return keys, vals


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, v_train, cam, settings, ras):
        scene = DeviceScene(means.detach().contiguous(), log_scales.detach().contiguous(), quats.detach().contiguous(),
                            opacity_logits.detach().contiguous(), sh.detach().contiguous(),
                            None if v_train is None else v_train.detach().contiguous())
        # a workspace of its own, kept alive for the backward of this call
        rgb, T, _ = ras.render(scene, cam, settings, fresh_ws=True)
        ctx.scene, ctx.cam, ctx.settings, ctx.ras = scene, cam, settings, ras
        ctx.ws = ras.last_ws
        ctx.save_for_backward(rgb)
        ctx.mark_non_differentiable(T)
        return rgb, T

    @staticmethod
    def backward(ctx, grad_rgb, grad_T):
        (rgb,) = ctx.saved_tensors
        g = ctx.ras.backward(ctx.scene, ctx.cam, ctx.settings, ctx.ws, rgb, grad_rgb)
        return g["means"], g["log_scales"], g["quats"], g["opacity_logits"], g["sh"], None, None, None, None


def render(means, log_scales, quats, opacity_logits, sh, cam, settings, ras: Rasterizer, v_train=None):
    """Differentiable render of one view: returns (rgb [3,H,W], T [H,W]).
    Gradients flow to means, log_scales, quats, opacity_logits and sh."""
    return _RenderFn.apply(means, log_scales, quats, opacity_logits, sh, v_train, cam, settings, ras)
