"""Multi-view training step: one batched forward over V views, an L1 loss,
one batched backward, and an Adam update of every parameter array in place.

The rasterisation, its adjoint and the optimiser update all run in
libaaa_hip.so; PyTorch holds the tensors and computes the loss gradient
(an elementwise sign).
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional, Sequence

import torch

from . import _lib as L
from .render import DeviceScene, Rasterizer, _stream_ptr

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")

# per-group learning rates of the 3DGS training lineage (positions scaled by
# the scene extent by the caller if wanted)
DEFAULT_LR = {"means": 1.6e-4, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2, "sh": 2.5e-3}


class Adam:
    """Adam state (first and second moments) for the parameter arrays of a
    DeviceScene; `step(grads)` updates the scene tensors in place."""

    def __init__(self, scene: DeviceScene, lr: Optional[Dict[str, float]] = None, betas=(0.9, 0.999), eps=1e-15):
        self.scene = scene
        self.lr = dict(DEFAULT_LR if lr is None else lr)
        self.b1, self.b2 = float(betas[0]), float(betas[1])
        self.eps = float(eps)
        self.t = 0
        self.m = {k: torch.zeros_like(getattr(scene, k)) for k in GROUPS}
        self.v = {k: torch.zeros_like(getattr(scene, k)) for k in GROUPS}

    def step(self, grads: Dict[str, torch.Tensor]):
        self.t += 1
        lib = L.lib()
        for k in GROUPS:
            p, g = getattr(self.scene, k), grads[k]
            assert p.is_contiguous() and g.is_contiguous() and g.shape == p.shape and g.dtype == torch.float32
            L.check(lib.aaa_adam_step(p.data_ptr(), g.data_ptr(), self.m[k].data_ptr(), self.v[k].data_ptr(),
                                      p.numel(), self.t, float(self.lr[k]), self.b1, self.b2, self.eps,
                                      _stream_ptr(p.device)))


def l1_grad(rgb: torch.Tensor, target: torch.Tensor, scale: float) -> torch.Tensor:
    """dL/drgb of L = scale * sum |rgb - target| (0 at ties)."""
    return torch.sign(rgb - target) * scale


def train_step(ras: Rasterizer, scene: DeviceScene, cams: Sequence, targets: Sequence[torch.Tensor], settings,
               opt: Adam) -> float:
    """One step over the views `cams` (one batch): returns the mean L1 loss
    before the update."""
    rgbs, _, _ = ras.render_batch(scene, cams, settings)
    npix = sum(r.numel() for r in rgbs)
    dl = [l1_grad(r, t, 1.0 / npix) for r, t in zip(rgbs, targets)]
    loss = sum(float((r - t).abs().sum()) for r, t in zip(rgbs, targets)) / npix
    grads = ras.backward_batch(scene, cams, settings, ras.last_ws, rgbs, dl)
    opt.step(grads)
    return loss
