"""Imaging major cycle on the library's kernels.

Deconvolution follows imaging in the processing chain the paper describes
(Sec. 1): CLEAN in Hogbom's form, inside the major / minor cycle split of
Clark and Schwab.  ``MajorCycle`` drives the C ABI: the dirty beam once
(ws_dirty_beam), then per major cycle the residual image of the current
model (ws_residual_image: degridding of the model, residual visibilities,
gridding, FFT, w-screen and plane sum) and a Hogbom minor cycle on the GPU
(ws_clean_minor).  Every step runs in the HIP kernels; this module only
holds the device buffers and loops.
"""
from __future__ import annotations

from typing import List, Optional

import torch

from . import _abi
from .api import WStackPlan, _ptr


class MajorCycle:
    """Cotton-Schwab deconvolution of one visibility set on one plan.

    ``uvw``, ``vis``, ``weight`` are device tensors of the plan's
    precision (vis Hermitian-paired for a real sky).  ``run`` returns the
    model image; ``residual`` holds the residual image of that model,
    ``picks`` the pixel indices taken in each major cycle.
    """

    def __init__(self, plan: WStackPlan, uvw, vis, weight=None):
        self.plan = plan
        m = int(uvw.shape[0])
        plan._check(uvw, torch.float64, (m, 3), "uvw")
        plan._check(vis, plan.cdtype, (m,), "vis")
        plan._check(weight, torch.float32, (m,), "weight")
        self.uvw, self.vis, self.weight, self.m = uvw, vis, weight, m
        nv, nu = plan.params.nv, plan.params.nu
        d = plan.device
        self.image_scratch = torch.empty((nv, nu), dtype=plan.cdtype,
                                         device=d)
        self.vis_scratch = torch.empty(max(m, 1), dtype=plan.cdtype, device=d)
        self.beam = torch.empty((nv, nu), dtype=plan.rdtype, device=d)
        self.beta = torch.zeros(1, dtype=torch.float64, device=d)
        self.model = torch.zeros((nv, nu), dtype=plan.rdtype, device=d)
        self.residual = torch.empty((nv, nu), dtype=plan.rdtype, device=d)
        self.n_done = torch.zeros(1, dtype=torch.int32, device=d)
        self.picks: List[torch.Tensor] = []
        plan.reset()
        plan._bind()
        _abi.call("ws_dirty_beam", plan._h, m, _ptr(uvw), _ptr(weight),
                  _ptr(self.image_scratch), _ptr(self.beam), _ptr(self.beta))

    def residual_image(self) -> torch.Tensor:
        """Recompute ``residual`` for the current model."""
        self.plan._bind()
        _abi.call("ws_residual_image", self.plan._h, self.m, _ptr(self.uvw),
                  _ptr(self.vis), _ptr(self.weight), _ptr(self.model),
                  _ptr(self.beta), _ptr(self.vis_scratch),
                  _ptr(self.image_scratch), _ptr(self.residual))
        return self.residual

    def minor(self, niter: int, gain: float, threshold: float = 0.0,
              picks: Optional[torch.Tensor] = None):
        """One Hogbom minor cycle on ``residual`` (adds to ``model``)."""
        self.plan._bind()
        _abi.call("ws_clean_minor", self.plan._h, _ptr(self.residual),
                  _ptr(self.beam), _ptr(self.model), int(niter), float(gain),
                  float(threshold), _ptr(picks), _ptr(self.n_done))

    def run(self, n_major: int, n_minor: int, gain: float = 0.1,
            threshold: float = 0.0) -> torch.Tensor:
        for _ in range(n_major):
            self.residual_image()
            pk = torch.full((max(n_minor, 1),), -1, dtype=torch.int32,
                            device=self.plan.device)
            self.minor(n_minor, gain, threshold, pk)
            self.picks.append(pk)
        self.residual_image()
        return self.model
