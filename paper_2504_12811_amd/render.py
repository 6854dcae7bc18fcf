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


class Rasterizer:
    """Owns a library context and a growable workspace on one device."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        ctx = C.c_void_p()
        L.check(L.lib().aaa_create(C.byref(ctx), int(device)))
        self._ctx = ctx
        self._ws = None
        self._ws_bytes = 0
        self.max_pairs = 0
        self.last_pairs = 0

    def __del__(self):
        try:
            if getattr(self, "_ctx", None):
                L.lib().aaa_destroy(self._ctx)
        except Exception:
            pass

    # workspace --------------------------------------------------------
    def _ensure_ws(self, sc: L.Scene, cam: L.Camera, st: L.Settings, max_pairs: int):
        need = C.c_size_t()
        L.check(L.lib().aaa_workspace_size(C.byref(sc), C.byref(cam), C.byref(st), max_pairs, C.byref(need)))
        if self._ws is None or self._ws_bytes < need.value:
            self._ws = None
            torch.cuda.synchronize(self.device)
            nbytes = int(need.value * 1.1) + 4096
            buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-buf.data_ptr()) % 256
            self._ws_buf = buf
            self._ws = buf[off: off + nbytes]
            self._ws_bytes = nbytes
        self.max_pairs = max_pairs

    def workspace(self):
        return self._ws.data_ptr(), self._ws_bytes, self.max_pairs

    # forward ------------------------------------------------------------
    def render(self, scene: DeviceScene, cam, settings, stats: bool = False, timing: bool = False,
               max_pairs: Optional[int] = None):
        """Render one view; returns (rgb [3,H,W], T [H,W], Stats)."""
        sc = scene.abi()
        c = L.make_camera(cam)
        st = L.make_settings(settings, (L.AAA_STATS if stats else 0) | (L.AAA_TIMING if timing else 0))
        H, W = int(cam.height), int(cam.width)
        rgb = torch.empty((3, H, W), dtype=torch.float32, device=self.device)
        T = torch.empty((H, W), dtype=torch.float32, device=self.device)
        mp = max_pairs or max(self.max_pairs, 8 * max(scene.n, 1), 1 << 16)
        for _ in range(4):
            self._ensure_ws(sc, c, st, mp)
            out = L.Stats()
            rc = L.lib().aaa_render(self._ctx, C.byref(sc), C.byref(c), C.byref(st), self._ws.data_ptr(),
                                    self._ws_bytes, mp, _stream_ptr(self.device), rgb.data_ptr(), T.data_ptr(),
                                    C.byref(out))
            if rc == L.AAA_ERR_PAIR_OVERFLOW:
                mp = min(int(out.pairs * 1.25) + 1024, (1 << 32) - 1)
                continue
            L.check(rc)
            self.last_pairs = int(out.pairs)
            return rgb, T, out
        raise L.AAAError(L.AAA_ERR_PAIR_OVERFLOW, "pair buffer kept overflowing")

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
        L.check(L.lib().aaa_read_gaussians(C.byref(scene.abi()), C.byref(L.make_camera(cam)), self.max_pairs,
                                           self._ws.data_ptr(), self._ws_bytes, _stream_ptr(dev), status.data_ptr(),
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
        L.check(L.lib().aaa_read_pairs(C.byref(scene.abi()), C.byref(L.make_camera(cam)), self.max_pairs,
                                       self._ws.data_ptr(), self._ws_bytes, _stream_ptr(dev), keys.data_ptr(),
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
