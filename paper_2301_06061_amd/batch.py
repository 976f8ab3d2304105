"""Many images in one launch sequence (frequency channels, observations).

``BatchedImager`` owns one ``WStackPlan`` per channel (each with its own
grid, planes, w range and visibility count) and images them together
through ws_batch_image: per-plan binning, one persistent gridding kernel
over the work items of every channel, then each channel's FFT, w-screen
and plane sum.  ``capture()`` records that sequence into a HIP graph once;
``replay()`` relaunches it with a single call.  Launch parameters (tile
edge, records per work item) can come from the autotuner per shape class.
"""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import torch

from . import _abi
from .api import WStackPlan, _ptr


class BatchedImager:
    def __init__(self, workloads: Sequence, uvw: Sequence[torch.Tensor],
                 vis: Sequence[torch.Tensor],
                 weight: Optional[Sequence[Optional[torch.Tensor]]] = None,
                 precision: str = "fp32", tune: bool = False,
                 params: Optional[Sequence[tuple]] = None):
        """One plan per workload geometry; uvw/vis/weight are the device
        inputs of each channel (kept referenced; their contents may change
        between runs, their shapes may not)."""
        n = len(workloads)
        if not (1 <= n <= 64):
            raise ValueError("a batch holds 1..64 channels")
        self.device = uvw[0].device
        self.stream = torch.cuda.Stream(device=self.device)
        self.uvw = list(uvw)
        self.vis = list(vis)
        self.weight = list(weight) if weight is not None else [None] * n
        self.plans: List[WStackPlan] = []
        self.tuned = []
        with torch.cuda.stream(self.stream):
            for i, wl in enumerate(workloads):
                tile, chunk = 0, 0
                if params is not None:
                    tile, chunk = params[i]
                elif tune:
                    from .autotune import tune as _tune
                    tile, chunk = _tune(wl, self.uvw[i], self.vis[i],
                                        self.weight[i], precision)
                self.tuned.append((tile, chunk))
                p = WStackPlan(wl.nu, wl.nv, wl.nw, wl.fov_l, wl.fov_m,
                               wl.w_min, wl.w_max, wl.support,
                               getattr(wl, "sigma", 0.0), precision,
                               max_vis=max(1, int(self.uvw[i].shape[0])),
                               tile=tile, chunk=chunk, device=self.device,
                               kernel=getattr(wl, "kernel", "gauss"),
                               beta=getattr(wl, "beta", 0.0),
                               correct=bool(getattr(wl, "correct", False)))
                self.plans.append(p)
            self.images = [p.new_image() for p in self.plans]
        wb = C.c_size_t(0)
        _abi.call("ws_batch_workspace_bytes", n, C.byref(wb))
        self.work = torch.empty(wb.value, dtype=torch.uint8,
                                device=self.device)
        handles = (C.c_void_p * n)(*[p._h for p in self.plans])
        for p in self.plans:
            _abi.call("ws_set_stream", p._h, C.c_void_p(self.stream.cuda_stream))
        h = C.c_void_p()
        _abi.call("ws_batch_create", n, handles, _ptr(self.work), wb.value,
                  C.byref(h))
        self._h = h
        self._args = self._marshal()
        self.captured = False

    def _marshal(self):
        n = len(self.plans)
        for i, p in enumerate(self.plans):
            m = int(self.uvw[i].shape[0])
            p._check(self.uvw[i], torch.float64, (m, 3), f"uvw[{i}]")
            p._check(self.vis[i], p.cdtype, (m,), f"vis[{i}]")
            p._check(self.weight[i], torch.float32, (m,), f"weight[{i}]")
        m = (C.c_int64 * n)(*[int(u.shape[0]) for u in self.uvw])
        uvw = (C.c_void_p * n)(*[u.data_ptr() for u in self.uvw])
        vis = (C.c_void_p * n)(*[v.data_ptr() for v in self.vis])
        wt = (C.c_void_p * n)(*[0 if w is None else w.data_ptr()
                                for w in self.weight])
        img = (C.c_void_p * n)(*[t.data_ptr() for t in self.images])
        return m, uvw, vis, wt, img

    def run(self) -> List[torch.Tensor]:
        """Image every channel now (eager launches); returns the images."""
        with torch.cuda.stream(self.stream):
            for t in self.images:
                t.zero_()
            _abi.call("ws_batch_image", self._h, *self._args)
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return self.images

    def capture(self) -> None:
        """Record the batch into a HIP graph (nothing runs yet)."""
        torch.cuda.synchronize(self.device)
        _abi.call("ws_batch_capture", self._h, *self._args)
        self.captured = True

    def replay(self) -> List[torch.Tensor]:
        """Zero the images and relaunch the captured graph."""
        if not self.captured:
            raise RuntimeError("call capture() first")
        with torch.cuda.stream(self.stream):
            for t in self.images:
                t.zero_()
            _abi.call("ws_batch_replay", self._h)
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return self.images

    def close(self):
        if getattr(self, "_h", None) is not None:
            _abi.lib().ws_batch_destroy(self._h)
            self._h = None
        for p in getattr(self, "plans", []):
            p.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
