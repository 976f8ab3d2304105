"""Python face of libwstack.so: a plan object over torch-owned device memory.

PyTorch supplies the device buffers (the plane stack and the workspace) and
the HIP stream; every step of the imaging path runs in the library's HIP
kernels.  Arguments are checked here only for what ctypes cannot express
(device, dtype, contiguity, shapes); the library checks the rest.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import torch

from . import _abi

_PREC = {"fp32": _abi.WS_FP32, "fp64": _abi.WS_FP64,
         0: _abi.WS_FP32, 1: _abi.WS_FP64}
_KERN = {"gauss": _abi.WS_KERNEL_GAUSS, "es": _abi.WS_KERNEL_ES,
         0: _abi.WS_KERNEL_GAUSS, 1: _abi.WS_KERNEL_ES}
_BIN = {"auto": _abi.WS_BINNING_AUTO, "partition": _abi.WS_BINNING_PARTITION,
        "hashed": _abi.WS_BINNING_HASHED, 0: 0, 1: 1, 2: 2}


def make_params(nu, nv, nw, fov_l, fov_m, w_min, w_max, support=7,
                sigma=0.0, precision="fp32", tile=0, chunk=0,
                kernel="gauss", beta=0.0, correct=False,
                binning="auto") -> _abi.Params:
    return _abi.Params(int(nu), int(nv), int(nw), float(fov_l), float(fov_m),
                       float(w_min), float(w_max), int(support), float(sigma),
                       _PREC[precision], int(tile), int(chunk),
                       _KERN[kernel], float(beta), int(bool(correct)),
                       _BIN[binning])


def kernel_transform(params: _abi.Params, f):
    """(psi(f), c): the library's 1-D kernel transform at the frequencies f
    (cycles per cell) and its kernel norm (host only)."""
    import numpy as np
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
    psi = np.empty_like(f)
    c = C.c_double(0.0)
    _abi.call("ws_kernel_transform", C.byref(params), int(f.size),
              f.ctypes.data_as(C.c_void_p), psi.ctypes.data_as(C.c_void_p),
              C.byref(c))
    return psi, c.value


def workspace_bytes(params: _abi.Params, max_vis: int):
    """(plane stack bytes, workspace bytes) for a parameter set (host only)."""
    pb = C.c_size_t(0)
    wb = C.c_size_t(0)
    _abi.call("ws_workspace_bytes", C.byref(params), int(max_vis),
              C.byref(pb), C.byref(wb))
    return pb.value, wb.value


def validate(params: _abi.Params) -> None:
    _abi.call("ws_validate_params", C.byref(params))


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def grid_image_noalloc(params: _abi.Params, uvw, vis, weight=None,
                       image=None, dropped=None):
    """ws_grid_image_noalloc: grid and image with the library's static
    scratch (no plan, no stack or workspace tensors).  Adds into ``image``
    (a new zero image if None, the only allocation here, made by torch
    before the call) on the current stream and returns it."""
    fp64 = params.precision == _abi.WS_FP64
    cdt = torch.complex128 if fp64 else torch.complex64
    m = int(uvw.shape[0])
    if image is None:
        image = torch.zeros((params.nv, params.nu), dtype=cdt,
                            device=uvw.device)
    for t, dt, shape, name in ((uvw, torch.float64, (m, 3), "uvw"),
                               (vis, cdt, (m,), "vis"),
                               (weight, torch.float32, (m,), "weight"),
                               (image, cdt, (params.nv, params.nu), "image"),
                               (dropped, torch.int64, (1,), "dropped")):
        if t is None:
            continue
        if t.dtype != dt or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"{name}: need a contiguous {dt} of shape "
                             f"{shape}")
        if t.device != image.device:
            raise ValueError(f"{name} is not on {image.device}")
    with torch.cuda.device(image.device):
        stream = torch.cuda.current_stream(image.device).cuda_stream
        _abi.call("ws_grid_image_noalloc", C.byref(params), m, _ptr(uvw),
                  _ptr(vis), _ptr(weight), _ptr(image), _ptr(dropped),
                  C.c_void_p(stream))
    return image


class WStackPlan:
    """One imaging geometry bound to a plane stack and a workspace.

    ``precision`` is "fp32" (complex64 data, FP64 positions and phases) or
    "fp64" (complex128 throughout).  ``max_vis`` bounds the visibilities of
    one ``grid``/``degrid`` call.
    """

    def __init__(self, nu, nv, nw, fov_l, fov_m, w_min, w_max, support=7,
                 sigma=0.0, precision="fp32", max_vis=1 << 20, tile=0,
                 chunk=0, device=None, kernel="gauss", beta=0.0,
                 correct=False, binning="auto"):
        self.params = make_params(nu, nv, nw, fov_l, fov_m, w_min, w_max,
                                  support, sigma, precision, tile, chunk,
                                  kernel, beta, correct, binning)
        self.fp64 = self.params.precision == _abi.WS_FP64
        self.cdtype = torch.complex128 if self.fp64 else torch.complex64
        self.rdtype = torch.float64 if self.fp64 else torch.float32
        self.max_vis = int(max_vis)
        self.device = torch.device("cuda", torch.cuda.current_device()) \
            if device is None else torch.device(device)
        pb, wb = workspace_bytes(self.params, self.max_vis)
        self.planes = torch.empty((nw, nv, nu), dtype=self.cdtype,
                                  device=self.device)
        assert self.planes.numel() * self.planes.element_size() == pb
        self.work = torch.empty(wb, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _abi.call("ws_grid_init", C.byref(self.params), self.max_vis,
                      _ptr(self.planes), pb, _ptr(self.work), wb,
                      C.c_void_p(self._stream()), C.byref(h))
        self._h = h

    @classmethod
    def from_workload(cls, wl, max_vis=None, precision=None, **kw):
        prec = precision if precision is not None else (
            "fp64" if wl.precision == 1 else "fp32")
        kw.setdefault("kernel", getattr(wl, "kernel", "gauss"))
        kw.setdefault("beta", getattr(wl, "beta", 0.0))
        kw.setdefault("correct", bool(getattr(wl, "correct", False)))
        return cls(wl.nu, wl.nv, wl.nw, wl.fov_l, wl.fov_m, wl.w_min,
                   wl.w_max, wl.support, wl.sigma, prec,
                   max_vis=max(1, wl.m) if max_vis is None else max_vis, **kw)

    # -- helpers ---------------------------------------------------------
    def _stream(self) -> int:
        return torch.cuda.current_stream(self.device).cuda_stream

    def _bind(self):
        if self._h is None:
            raise RuntimeError("plan is closed")
        _abi.call("ws_set_stream", self._h, C.c_void_p(self._stream()))

    def _check(self, t, dtype, shape, name):
        if t is None:
            return None
        if t.device != self.device:
            raise ValueError(f"{name} must be on {self.device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, "
                             f"expected {tuple(shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    # -- the imaging steps ---------------------------------------------------
    def grid(self, uvw, vis, weight=None, dropped=None):
        """Grid visibilities onto the plane stack (additive)."""
        m = int(uvw.shape[0])
        self._check(uvw, torch.float64, (m, 3), "uvw")
        self._check(vis, self.cdtype, (m,), "vis")
        self._check(weight, torch.float32, (m,), "weight")
        self._check(dropped, torch.int64, (1,), "dropped")
        self._bind()
        _abi.call("ws_grid_visibilities", self._h, m, _ptr(uvw), _ptr(vis),
                  _ptr(weight), _ptr(dropped))

    def fft(self, direction: int = +1):
        self._bind()
        _abi.call("ws_fft_planes", self._h, int(direction))

    def wcorrect(self, image):
        self._check(image, self.cdtype, (self.params.nv, self.params.nu),
                    "image")
        self._bind()
        _abi.call("ws_wcorrect_accumulate", self._h, _ptr(image))

    def image_accumulate(self, image):
        """Fused FFT + screen + plane sum into ``image``; resets the stack."""
        self._check(image, self.cdtype, (self.params.nv, self.params.nu),
                    "image")
        self._bind()
        _abi.call("ws_image_accumulate", self._h, _ptr(image))

    def grid_image(self, uvw, vis, weight=None, image=None, dropped=None):
        """Grid and image in one call (the stack must be empty, e.g. after
        ``reset()``); adds into ``image`` (a new zero image if None) and
        returns it.  The stack is scratch: afterwards its contents are
        unspecified and the plan is empty."""
        m = int(uvw.shape[0])
        if image is None:
            image = self.new_image()
        self._check(uvw, torch.float64, (m, 3), "uvw")
        self._check(vis, self.cdtype, (m,), "vis")
        self._check(weight, torch.float32, (m,), "weight")
        self._check(image, self.cdtype, (self.params.nv, self.params.nu),
                    "image")
        self._check(dropped, torch.int64, (1,), "dropped")
        self._bind()
        _abi.call("ws_grid_image", self._h, m, _ptr(uvw), _ptr(vis),
                  _ptr(weight), _ptr(image), _ptr(dropped))
        return image

    def _rows_args(self, uvw_m, freq_hz, vis, weight, pol_coeff):
        if vis.dim() != 3:
            raise ValueError("vis must be [nrows, nchan, npol]")
        nrows, nchan, npol = (int(x) for x in vis.shape)
        self._check(uvw_m, torch.float64, (nrows, 3), "uvw_m")
        self._check(freq_hz, torch.float64, (nchan,), "freq_hz")
        self._check(vis, self.cdtype, None, "vis")
        self._check(weight, torch.float32, (nrows, npol), "weight")
        import numpy as np
        coeff = np.ascontiguousarray(
            np.asarray(pol_coeff, dtype=np.complex128).reshape(npol))
        pc = np.ascontiguousarray(
            np.stack([coeff.real, coeff.imag], axis=1), dtype=np.float64)
        return nrows, nchan, npol, pc

    def grid_rows(self, uvw_m, freq_hz, vis, weight, pol_coeff, dropped=None):
        """Baseline-major gridding (additive): uvw_m [R, 3] metres, freq_hz
        [C], vis [R, C, P], weight [R, P] or None, pol_coeff P complex
        coefficients of the gridded combination (host values)."""
        nrows, nchan, npol, pc = self._rows_args(uvw_m, freq_hz, vis, weight,
                                                 pol_coeff)
        self._check(dropped, torch.int64, (1,), "dropped")
        self._bind()
        _abi.call("ws_grid_rows", self._h, nrows, nchan, npol, _ptr(uvw_m),
                  _ptr(freq_hz), _ptr(vis), _ptr(weight),
                  pc.ctypes.data_as(C.c_void_p), _ptr(dropped))

    def grid_image_rows(self, uvw_m, freq_hz, vis, weight, pol_coeff,
                        image=None, dropped=None):
        """Baseline-major input through the one-call path (the stack must
        be empty); adds into ``image`` (a new zero image if None)."""
        nrows, nchan, npol, pc = self._rows_args(uvw_m, freq_hz, vis, weight,
                                                 pol_coeff)
        if image is None:
            image = self.new_image()
        self._check(image, self.cdtype, (self.params.nv, self.params.nu),
                    "image")
        self._check(dropped, torch.int64, (1,), "dropped")
        self._bind()
        _abi.call("ws_grid_image_rows", self._h, nrows, nchan, npol,
                  _ptr(uvw_m), _ptr(freq_hz), _ptr(vis), _ptr(weight),
                  pc.ctypes.data_as(C.c_void_p), _ptr(image), _ptr(dropped))
        return image

    def new_image(self):
        return torch.zeros((self.params.nv, self.params.nu), dtype=self.cdtype,
                           device=self.device)

    def dirty_image(self, uvw, vis, weight=None, fused=True, dropped=None):
        """Reset, grid, transform, screen and sum: a fresh dirty image
        (``fused``: one ws_grid_image call; else grid, FFT and the separate
        screen + sum)."""
        self.reset()
        img = self.new_image()
        if fused:
            self.grid_image(uvw, vis, weight, img, dropped)
        else:
            self.grid(uvw, vis, weight, dropped)
            self.fft(+1)
            self.wcorrect(img)
            self.reset()
        return img

    def degrid(self, image, uvw, weight=None, out=None):
        """Visibilities of ``image`` (real or complex): the adjoint operator."""
        m = int(uvw.shape[0])
        is_real = not image.is_complex()
        self._check(image, self.rdtype if is_real else self.cdtype,
                    (self.params.nv, self.params.nu), "image")
        self._check(uvw, torch.float64, (m, 3), "uvw")
        self._check(weight, torch.float32, (m,), "weight")
        if out is None:
            out = torch.empty(m, dtype=self.cdtype, device=self.device)
        self._check(out, self.cdtype, (m,), "out")
        self._bind()
        _abi.call("ws_degrid", self._h, _ptr(image), int(is_real), m,
                  _ptr(uvw), _ptr(weight), _ptr(out))
        return out

    def reset(self):
        _abi.call("ws_plan_reset", self._h)

    def sync(self):
        self._bind()
        _abi.call("ws_sync", self._h)

    def tile_stats(self) -> dict:
        """Work counts of the last binning call (waits for the stream)."""
        out = (C.c_int64 * 7)()
        _abi.call("ws_tile_stats", self._h, out)
        return {"tile": out[0], "busy": out[1], "idle": out[2],
                "split": out[3], "extra_items": out[4], "strips": out[5],
                "record_reads": out[6]}

    def set_profiling(self, enable: bool):
        _abi.call("ws_set_profiling", self._h, int(bool(enable)))

    def kernel_times(self, reset: bool = False) -> dict:
        """{kernel name: (total ms, launches)} since the last reset."""
        cap = 64
        names = (C.c_char_p * cap)()
        ms = (C.c_double * cap)()
        cnt = (C.c_int64 * cap)()
        n = C.c_int32(0)
        self._bind()
        _abi.call("ws_kernel_times", self._h, cap, names, ms, cnt,
                  C.byref(n), int(bool(reset)))
        return {names[i].decode(): (ms[i], cnt[i]) for i in range(n.value)}

    def close(self):
        if getattr(self, "_h", None) is not None:
            _abi.lib().ws_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
