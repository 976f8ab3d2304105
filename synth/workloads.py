"""Synthetic stand-ins for the paper's LOFAR Medium/Large workloads.

The paper images a LOFAR HBA observation (Sec. 4, Tables 2 and 3) that is not
available here, so every workload is drawn from a seeded PCG64 generator with
the shapes and structure the paper describes: a core-dense (u, v) coverage
(Sec. 3.1), w growing with baseline length, complex visibilities and weights
(Sec. 2), and a mesh of N_u x N_v x N_w cells.

Units: u, v, w are in wavelengths; the field of view is the full image width
in radians.  Positions are drawn in grid cells of width 1/fov and converted to
wavelengths with that factor; a margin of (support+1)/2 cells keeps every
kernel tap of every visibility inside the grid.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np


@dataclass
class Workload:
    """Grid geometry plus one batch of visibilities.

    ``uvw`` is float64 [m, 3]; ``vis`` complex64 or complex128 [m];
    ``weight`` float32 [m] or None (unit weights).
    """

    nu: int
    nv: int
    nw: int
    fov_l: float
    fov_m: float
    w_min: float
    w_max: float
    support: int
    sigma: float = 0.0
    precision: int = 0  # 0 = FP32 path (complex64 data), 1 = FP64 path
    uvw: Optional[np.ndarray] = None
    vis: Optional[np.ndarray] = None
    weight: Optional[np.ndarray] = None
    name: str = ""
    extra: dict = field(default_factory=dict)
    kernel: str = "gauss"   # gridding kernel: "gauss" or "es"
    beta: float = 0.0       # ES kernel shape (<= 0: the default)
    correct: bool = False   # divide the image by the kernel's transform

    @property
    def m(self) -> int:
        return 0 if self.uvw is None else int(self.uvw.shape[0])

    def geometry(self) -> dict:
        return dict(nu=self.nu, nv=self.nv, nw=self.nw, fov_l=self.fov_l,
                    fov_m=self.fov_m, w_min=self.w_min, w_max=self.w_max,
                    support=self.support, sigma=self.sigma,
                    precision=self.precision, kernel=self.kernel,
                    beta=self.beta, correct=self.correct)

    def as_precision(self, precision: int) -> "Workload":
        """Same draw in the other precision path (values upcast/downcast)."""
        cdt = np.complex128 if precision == 1 else np.complex64
        return replace(self, precision=precision,
                       vis=None if self.vis is None else self.vis.astype(cdt))


def _margin(support: int) -> int:
    return (support - 1) // 2 + 1


def _cn01(rng: np.random.Generator, m: int, dtype) -> np.ndarray:
    """Circular complex normal CN(0, 1): (a + ib)/sqrt(2), a, b ~ N(0, 1)."""
    a = rng.standard_normal(m)
    b = rng.standard_normal(m)
    out = np.empty(m, dtype=dtype)
    out.real = a / math.sqrt(2.0)
    out.imag = b / math.sqrt(2.0)
    return out


def _gauss_disk(rng, m, sigma_cells, radius_cells):
    """(u, v) in cells ~ N(0, sigma^2) each, rejection-resampled into a disk."""
    us = np.empty(0)
    vs = np.empty(0)
    while us.size < m:
        need = m - us.size
        draw = max(1024, int(need * 1.3) + 16)
        u = rng.standard_normal(draw) * sigma_cells
        v = rng.standard_normal(draw) * sigma_cells
        keep = u * u + v * v <= radius_cells * radius_cells
        us = np.concatenate([us, u[keep]])
        vs = np.concatenate([vs, v[keep]])
    return us[:m], vs[:m]


def _dense_core(rng, m, radius_cells):
    """Core-dense coverage: r = R U^2, theta ~ U[0, 2 pi).

    The surface density of r = R U^2 falls as r^-1.5, integrable at the
    centre, so a few per cent of the visibilities land within a cell of
    (u, v) = (0, 0), like the dense inner stations of a real array.
    """
    r = radius_cells * rng.random(m) ** 2
    th = 2.0 * math.pi * rng.random(m)
    return r * np.cos(th), r * np.sin(th), r


def config1(seed: int = 0, m: int = 200_000, precision: int = 1) -> Workload:
    """Plain FP64 w-stacking: 512^2 x 8 planes, K=7, 1 deg, Gaussian (u, v)."""
    n, nw, k = 512, 8, 7
    fov = math.radians(1.0)
    du = 1.0 / fov
    rng = np.random.default_rng(seed)
    uc, vc = _gauss_disk(rng, m, 0.25 * n / 2, n / 2 - _margin(k))
    wmax = (n / 2) * du
    w = rng.uniform(-wmax, wmax, m)
    uvw = np.stack([uc * du, vc * du, w], axis=1)
    cdt = np.complex128 if precision == 1 else np.complex64
    vis = _cn01(rng, m, cdt)
    return Workload(n, n, nw, fov, fov, -wmax, wmax, k, 0.0, precision,
                    uvw, vis, np.ones(m, np.float32), name="config1")


def _dense_core_workload(seed, m, n, nw, k, fov_deg, precision, name,
                         scale=1.0, rng=None):
    fov = math.radians(fov_deg)
    du = 1.0 / fov
    rng = np.random.default_rng(seed) if rng is None else rng
    radius = (n / 2 - _margin(k)) * scale
    uc, vc, r = _dense_core(rng, m, radius)
    wmax = (n / 2) * du * scale
    w = wmax * r / radius + rng.standard_normal(m) * (0.1 * wmax)
    uvw = np.stack([uc * du, vc * du, w], axis=1)
    cdt = np.complex128 if precision == 1 else np.complex64
    vis = _cn01(rng, m, cdt)
    return Workload(n, n, nw, fov, fov, float(w.min()), float(w.max()), k,
                    0.0, precision, uvw, vis, np.ones(m, np.float32),
                    name=name)


def config2(seed: int = 0, m: int = 10_000_000, precision: int = 0) -> Workload:
    """Dense-core array: 4096^2 x 32 planes, K=7, 5 deg, 1e7 visibilities.

    w = wmax r/R + N(0, (0.1 wmax)^2) with wmax the largest |u| on the grid;
    the planes span the data's [min w, max w].
    """
    return _dense_core_workload(seed, m, 4096, 32, 7, 5.0, precision,
                                "config2")


def config3(seed: int = 0, m: int = 100_000_000, precision: int = 0) -> Workload:
    """Large single image: 16384^2 x 32 planes, K=9, 8 deg, 1e8 visibilities."""
    return _dense_core_workload(seed, m, 16384, 32, 9, 8.0, precision,
                                "config3")


def config4(seed: int = 0, channels: int = 64, m_scale: float = 1.0):
    """Batched channels: 64 channels, log-uniform counts in [1e5, 5e6].

    Channel c draws from ``default_rng([seed, c])``: its count, its grid size
    N_c (uniform over 1024, 2048, 4096), N_w = 16 below 4096 else 32, and a
    config-2 style dense core whose radius scales with f_c / 200 MHz,
    f_c = 100 + 100 c / 63 MHz.  FP32 path.  ``m_scale`` shrinks every count
    (tests use it for small batches).
    """
    out = []
    for c in range(channels):
        rng = np.random.default_rng([seed, c])
        mc = int(round(math.exp(rng.uniform(math.log(1e5), math.log(5e6)))))
        mc = max(1, int(round(mc * m_scale)))
        n = int(rng.choice([1024, 2048, 4096]))
        nw = 16 if n < 4096 else 32
        f = 100.0 + 100.0 * c / (channels - 1 if channels > 1 else 1)
        wl = _dense_core_workload(None, mc, n, nw, 7, 5.0, 0,
                                  f"config4.ch{c}", scale=f / 200.0, rng=rng)
        wl.extra["freq_mhz"] = f
        out.append(wl)
    return out


def config5(seed: int = 0, m: int = 10_000_000, n: int = 4096,
            nsrc: int = 1000):
    """Differentiable imaging: a sparse real image and config-1 style data.

    Returns (workload, x) with x a float32 [n, n] image of ``nsrc`` distinct
    point sources with N(0, 1) amplitudes; visibilities follow config 1's
    Gaussian law scaled to n, w ~ U[-wmax, wmax], V ~ CN(0, 1) complex64.
    """
    k, nw = 7, 32
    fov = math.radians(5.0)
    du = 1.0 / fov
    rng = np.random.default_rng(seed)
    x = np.zeros(n * n, np.float32)
    idx = rng.choice(n * n, size=nsrc, replace=False)
    x[idx] = rng.standard_normal(nsrc).astype(np.float32)
    uc, vc = _gauss_disk(rng, m, 0.25 * n / 2, n / 2 - _margin(k))
    wmax = (n / 2) * du
    w = rng.uniform(-wmax, wmax, m)
    uvw = np.stack([uc * du, vc * du, w], axis=1)
    vis = _cn01(rng, m, np.complex64)
    wl = Workload(n, n, nw, fov, fov, -wmax, wmax, k, 0.0, 0, uvw, vis,
                  np.ones(m, np.float32), name="config5")
    return wl, x.reshape(n, n)


def random_case(seed: int, n: int = 64, nw: int = 4, support: int = 7,
                m: int = 1000, fov_deg: float = 2.0, precision: int = 1,
                law: str = "gauss", weights: bool = True, nv: int = None,
                sigma: float = 0.0) -> Workload:
    """Small seeded case for tests: any grid, plane count and support.

    ``law`` is "gauss" (config-1 style) or "core" (config-2 style); weights
    are U[0.5, 1.5] float32 when ``weights`` is set, else None (unit).
    """
    nv = n if nv is None else nv
    fov_l = math.radians(fov_deg)
    fov_m = fov_l * nv / n
    du = 1.0 / fov_l
    dv = 1.0 / fov_m
    rng = np.random.default_rng(seed)
    half = min(n, nv) / 2 - _margin(support)
    if law == "gauss":
        uc, vc = _gauss_disk(rng, m, 0.25 * min(n, nv) / 2, half)
        wmax = (min(n, nv) / 2) * du
        w = rng.uniform(-wmax, wmax, m)
    else:
        uc, vc, r = _dense_core(rng, m, half)
        wmax = (min(n, nv) / 2) * du
        w = wmax * r / max(half, 1e-9) + rng.standard_normal(m) * 0.1 * wmax
    uvw = np.stack([uc * du, vc * dv, w], axis=1)
    cdt = np.complex128 if precision == 1 else np.complex64
    vis = _cn01(rng, m, cdt)
    wt = rng.uniform(0.5, 1.5, m).astype(np.float32) if weights else None
    w_min, w_max = (-wmax, wmax) if law == "gauss" else (float(w.min()),
                                                          float(w.max()))
    return Workload(n, nv, nw, fov_l, fov_m, w_min, w_max, support, sigma,
                    precision, uvw, vis, wt, name=f"random{seed}")


def hermitian_pairs(wl: Workload) -> Workload:
    """Append the conjugate mirror (-u, -v, -w, conj V) of every visibility.

    With planes symmetric about w = 0 the dirty image of such data is real.
    """
    uvw = np.concatenate([wl.uvw, -wl.uvw], axis=0)
    vis = np.concatenate([wl.vis, np.conj(wl.vis)])
    wt = None if wl.weight is None else np.concatenate([wl.weight, wl.weight])
    return replace(wl, uvw=uvw, vis=vis, weight=wt, name=wl.name + "+herm")


CONFIGS = {1: config1, 2: config2, 3: config3}


def edge_case(seed: int, n: int = 128, nv: int = None, nw: int = 4,
              support: int = 7, m: int = 3000, fov_deg: float = 2.0,
              precision: int = 1, bad: bool = True) -> Workload:
    """Footprints that hang off every edge and corner of the grid, and w
    values outside the plane range and exactly on plane boundaries.

    Positions (in cells, then wavelengths):
      * a quarter near the low or high u edge, a quarter near the low or high
        v edge, a quarter near a corner: the nearest cell lies within h + 1
        cells of the edge on either side, so that anywhere from none to all
        but one column (row) of the K x K taps is on the grid;
      * the rest uniform over the whole grid.
    w: the planes span [-2048, 2048] wavelengths (dw an exact power of two
    for nw a power of two); an eighth of the visibilities each below w_min,
    above w_max, and exactly at w_min + k dw (k = 0 .. nw, both ends
    included); the rest uniform in the range.
    With ``bad``, four visibilities get a NaN, an infinite or a far-off
    coordinate.  Weights U[0.5, 1.5].
    """
    nv = n if nv is None else nv
    fov_l = math.radians(fov_deg)
    fov_m = fov_l * nv / n
    h = (support - 1) // 2
    rng = np.random.default_rng(seed)

    def near_edge(size, cnt):
        # Offset of the nearest cell from the edge in [-(h+1), h+1], plus a
        # fraction of a cell, on the low or the high side.
        off = rng.integers(-(h + 1), h + 2, cnt) + rng.uniform(-0.45, 0.45, cnt)
        high = rng.random(cnt) < 0.5
        return np.where(high, size - 1 - off, off)

    q = m // 4
    xs = rng.uniform(-0.5, n - 0.5, m)
    ys = rng.uniform(-0.5, nv - 0.5, m)
    xs[:q] = near_edge(n, q)
    ys[q:2 * q] = near_edge(nv, q)
    xs[2 * q:3 * q] = near_edge(n, q)
    ys[2 * q:3 * q] = near_edge(nv, q)
    w_min, w_max = -2048.0, 2048.0
    dw = (w_max - w_min) / nw
    w = rng.uniform(w_min, w_max, m)
    e = m // 8
    w[:e] = w_min - rng.uniform(0.0, 3.0 * dw, e)
    w[e:2 * e] = w_max + rng.uniform(0.0, 3.0 * dw, e)
    w[2 * e:3 * e] = w_min + rng.integers(0, nw + 1, e) * dw
    perm = rng.permutation(m)
    xs, ys = xs[perm], ys[perm]
    uvw = np.stack([(xs - n / 2) / fov_l, (ys - nv / 2) / fov_m, w], axis=1)
    if bad and m >= 8:
        uvw[0, 0] = np.nan
        uvw[1, 1] = np.inf
        uvw[2, 2] = np.nan
        uvw[3, 0] = 1e30
    cdt = np.complex128 if precision == 1 else np.complex64
    vis = _cn01(rng, m, cdt)
    wt = rng.uniform(0.5, 1.5, m).astype(np.float32)
    return Workload(n, nv, nw, fov_l, fov_m, w_min, w_max, support, 0.0,
                    precision, np.ascontiguousarray(uvw), vis, wt,
                    name=f"edge{seed}")


@dataclass
class RowsWorkload:
    """Baseline-major data (one row per baseline and time): uvw in metres
    per row, channel frequencies, visibilities per (row, channel,
    correlation), weights per (row, correlation).  ``geo`` is a Workload
    holding the grid geometry (its uvw/vis are None)."""

    geo: Workload
    uvw_m: np.ndarray      # float64 [R, 3]
    freq_hz: np.ndarray    # float64 [C]
    vis: np.ndarray        # complex64 / complex128 [R, C, P]
    weight: np.ndarray     # float32 [R, P]


C0 = 299_792_458.0  # m/s


def rows_case(seed: int, n: int = 128, nw: int = 4, support: int = 7,
              nrows: int = 500, nchan: int = 8, npol: int = 4,
              f_lo: float = 100e6, f_hi: float = 200e6, fov_deg: float = 2.0,
              precision: int = 1, law: str = "core") -> RowsWorkload:
    """Seeded baseline-major case: rows drawn like ``random_case`` in cells
    at the highest channel frequency (so every channel's footprint stays on
    the grid), converted to metres; channels spaced evenly in [f_lo, f_hi];
    CN(0, 1) correlations; U[0.5, 1.5] weights.  The plane range covers the
    w of every channel."""
    fov = math.radians(fov_deg)
    du = 1.0 / fov
    rng = np.random.default_rng(seed)
    half = n / 2 - _margin(support)
    if law == "gauss":
        uc, vc = _gauss_disk(rng, nrows, 0.25 * n / 2, half)
        wmax = (n / 2) * du
        w = rng.uniform(-wmax, wmax, nrows)
    else:
        uc, vc, r = _dense_core(rng, nrows, half)
        wmax = (n / 2) * du
        w = wmax * r / max(half, 1e-9) + rng.standard_normal(nrows) * 0.1 * wmax
    freq = np.linspace(f_lo, f_hi, nchan) if nchan > 1 else np.array([f_hi])
    to_m = C0 / freq.max()
    uvw_m = np.stack([uc * du, vc * du, w], axis=1) * to_m
    cdt = np.complex128 if precision == 1 else np.complex64
    vis = _cn01(rng, nrows * nchan * npol, cdt).reshape(nrows, nchan, npol)
    wt = rng.uniform(0.5, 1.5, (nrows, npol)).astype(np.float32)
    w_lambda = uvw_m[:, 2][:, None] * (freq[None, :] / C0)
    lo, hi = ((float(w_lambda.min()), float(w_lambda.max()))
              if nrows > 0 and nw > 1 else (-1.0, 1.0))
    geo = Workload(n, n, nw, fov, fov, lo, hi, support, 0.0, precision,
                   name=f"rows{seed}")
    return RowsWorkload(geo, uvw_m, freq, vis, wt)
