"""FP64 CPU oracle for the w-stacking imaging path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this module; only the tests, the smoke check and the benchmark's CPU baseline
do.  It shares no code with the HIP library: it is a plain, slow, obviously
correct NumPy restatement of the method, written from the paper's Sec. 2
(Eqs. 1-3) in float64 throughout, with NumPy's FFT and ``bincount`` as the only
library primitives.

The paper leaves several conventions open (kernel width and normalisation,
the grid-to-wavelength map, the plane placement, the FFT centring, what
happens to taps that fall off the grid).  The readings taken here are:

* grid cell size du = 1/fov (fov = full image width in radians), so that
  du * dl = 1/N with dl = fov/N; the zero spacing sits at cell N/2;
* visibility m lands at x = u fov + N_u/2, y = v fov_m + N_v/2, its kernel is
  centred on the nearest cell i0 = floor(x + 1/2), j0 = floor(y + 1/2);
* nearest w-plane (Sec. 2): k = clamp(floor((w - w_min)/dw), 0, N_w - 1) with
  dw = (w_max - w_min)/N_w and plane centres w_k = w_min + (k + 1/2) dw
  (N_w = 1: a single plane at (w_min + w_max)/2);
* Gaussian kernel of support K cells (Sec. 2): sigma = K/7 cells unless given,
  G = c g(i - x) g(j - y), g(d) = exp(-d^2 / (2 sigma^2)), c = 1/(2 pi sigma^2);
  the visibility is multiplied by its weight (natural weighting);
* taps that fall outside the grid are dropped and counted;
* each plane is transformed with the unnormalised, centred, backward
  (e^{+2 pi i}) 2-D DFT of Eq. (2);
* the phase screen is exp(+2 pi i w_k (n - 1)) with n - 1 = sqrt(1 - l^2 - m^2)
  - 1 evaluated as -r^2 / (1 + sqrt(1 - r^2)) (no cancellation near r = 0);
* the dirty image is the plain sum over planes (the right-hand side of
  Eq. (2), no 1/n or (w_max - w_min) factor).

Production kernels (Sec. 2 names the Gaussian as the paper's choice and
better kernels as the alternative; Sec. 5 lists them as future work): the
"exponential of semicircle" kernel phi(z) = exp(beta (sqrt(1 - z^2) - 1)),
z = 2 d / K, over the same K x K support, normalised so that its continuous
2-D integral is one.  With ``correct`` the image is divided by the gridding
kernel's 2-D Fourier transform c psi(f_p) psi(f_q) (the grid correction),
where psi is the transform of the 1-D kernel truncated to its support and
f_p = (p - N/2)/N; the degridder multiplies its input image by the same
factor (the correction is real and diagonal, so it is its own adjoint).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Params:
    nu: int
    nv: int
    nw: int
    fov_l: float
    fov_m: float
    w_min: float
    w_max: float
    support: int
    sigma: float = 0.0
    kernel: str = "gauss"     # "gauss" or "es" (exponential of semicircle)
    beta: float = 0.0         # ES shape; <= 0 selects 2.3 K
    correct: bool = False     # divide the image by the kernel's transform

    @classmethod
    def of(cls, wl) -> "Params":
        """Take the geometry fields from any object that carries them."""
        return cls(wl.nu, wl.nv, wl.nw, wl.fov_l, wl.fov_m, wl.w_min,
                   wl.w_max, wl.support, getattr(wl, "sigma", 0.0),
                   getattr(wl, "kernel", "gauss"), getattr(wl, "beta", 0.0),
                   bool(getattr(wl, "correct", False)))


# ---------------------------------------------------------------------------
# Kernel (Sec. 2, Eq. (3): Gaussian convolution function of support K cells)
# ---------------------------------------------------------------------------

def kernel_sigma(p: Params) -> float:
    """Gaussian width in cells; the paper gives only the support (7 cells)."""
    return float(p.sigma) if p.sigma > 0 else p.support / 7.0


def kernel_norm(p: Params) -> float:
    """c: the continuous 2-D kernel c phi(x) phi(y) integrates to one.

    Gaussian: c = 1/(2 pi sigma^2) (the untruncated integral).  ES kernel:
    c = 1 / (integral of phi(2 d / K) over |d| <= K/2)^2, by quadrature.
    """
    if p.kernel == "es":
        return 1.0 / float(kernel_ft(p, 0.0)) ** 2
    s = kernel_sigma(p)
    return 1.0 / (2.0 * math.pi * s * s)


def gauss(d, sigma):
    """One-dimensional Gaussian factor g(d) = exp(-d^2 / (2 sigma^2))."""
    d = np.asarray(d, dtype=np.float64)
    return np.exp(-(d * d) / (2.0 * sigma * sigma))


def es_beta(p: Params) -> float:
    """Shape of the exponential-of-semicircle kernel; 2.3 K unless given."""
    return float(p.beta) if p.beta > 0 else 2.3 * p.support


def es(d, support, beta):
    """phi(2 d / K) = exp(beta (sqrt(1 - z^2) - 1)), zero for |z| > 1."""
    z = 2.0 * np.asarray(d, dtype=np.float64) / support
    inside = np.abs(z) <= 1.0
    r = np.sqrt(np.where(inside, 1.0 - z * z, 0.0))
    return np.where(inside, np.exp(beta * (r - 1.0)), 0.0)


def kernel_1d(p: Params, d):
    """The 1-D factor of the separable gridding kernel at offset d (cells)."""
    if p.kernel == "es":
        return es(d, p.support, es_beta(p))
    if p.kernel != "gauss":
        raise ValueError(f"unknown kernel {p.kernel!r}")
    return gauss(d, kernel_sigma(p))


_QUAD_NODES = 96


def kernel_ft(p: Params, f):
    """psi(f) = integral over |d| <= K/2 of phi(d) cos(2 pi f d) dd: the
    Fourier transform of the truncated 1-D kernel (f in cycles per cell).

    Gauss-Legendre quadrature: on d directly for the Gaussian; for the ES
    kernel after z = 2 d / K = sin(t), which makes the integrand smooth
    (phi has a square-root edge at |z| = 1).
    """
    f = np.asarray(f, dtype=np.float64)
    x, w = np.polynomial.legendre.leggauss(_QUAD_NODES)
    half = p.support / 2.0
    if p.kernel == "es":
        t = x * (math.pi / 2)
        g = np.exp(es_beta(p) * (np.cos(t) - 1.0)) * np.cos(t)
        d = half * np.sin(t)
        wt = w * (math.pi / 2) * half * g
    else:
        d = x * half
        wt = w * half * gauss(d, kernel_sigma(p))
    return np.cos(2.0 * math.pi * f[..., None] * d) @ wt


def grid_correction(p: Params):
    """1 / (c psi(f_p) psi(f_q)) at pixel [q][p]: the factor that divides
    the image by the gridding kernel's 2-D Fourier transform."""
    fp = (np.arange(p.nu) - p.nu / 2) / p.nu
    fq = (np.arange(p.nv) - p.nv / 2) / p.nv
    c = kernel_norm(p)
    return 1.0 / (c * kernel_ft(p, fq)[:, None] * kernel_ft(p, fp)[None, :])


# ---------------------------------------------------------------------------
# w-planes (Sec. 2: visibilities go to the closest w-plane)
# ---------------------------------------------------------------------------

def plane_spacing(p: Params) -> float:
    if p.nw == 1:
        return 1.0
    return (p.w_max - p.w_min) / p.nw


def plane_centres(p: Params) -> np.ndarray:
    """w_k, the w value each plane stands for."""
    if p.nw == 1:
        return np.array([0.5 * (p.w_min + p.w_max)])
    dw = plane_spacing(p)
    return p.w_min + (np.arange(p.nw) + 0.5) * dw


def plane_index(p: Params, w) -> np.ndarray:
    """Index of the closest plane centre, clamped to the end planes."""
    w = np.asarray(w, dtype=np.float64)
    if p.nw == 1:
        return np.zeros(w.shape, dtype=np.int64)
    k = np.floor((w - p.w_min) / plane_spacing(p))
    return np.clip(k, 0, p.nw - 1).astype(np.int64)


# ---------------------------------------------------------------------------
# Step 1 - coordinates of each visibility on the mesh (Sec. 2)
# ---------------------------------------------------------------------------

_FAR = 1.0e9  # a cell position far off any grid


def coordinates(p: Params, uvw):
    """Continuous cell position (x, y), nearest cell (i0, j0) and plane k.

    A visibility with a non-finite coordinate, or one so far off the grid
    that none of its taps can land on it, is parked at a position far off
    the grid, so that all of its taps are dropped.
    """
    uvw = np.asarray(uvw, dtype=np.float64)
    x = uvw[:, 0] * p.fov_l + p.nu / 2
    y = uvw[:, 1] * p.fov_m + p.nv / 2
    ok = np.isfinite(uvw).all(axis=1) & (np.abs(x) < _FAR) & (np.abs(y) < _FAR)
    x = np.where(ok, x, -_FAR)
    y = np.where(ok, y, -_FAR)
    i0 = np.floor(x + 0.5).astype(np.int64)
    j0 = np.floor(y + 0.5).astype(np.int64)
    k = plane_index(p, np.where(ok, uvw[:, 2], p.w_min))
    return x, y, i0, j0, k


def _weights(weight, m):
    if weight is None:
        return np.ones(m, dtype=np.float64)
    return np.asarray(weight, dtype=np.float64)


# ---------------------------------------------------------------------------
# Step 2 - convolutional gridding onto the plane stack (Eq. (3))
# ---------------------------------------------------------------------------

def grid(p: Params, uvw, vis, weight=None):
    """Grid visibilities onto P[k][j][i] (complex128) with the kernel.

    For every tap (a, b) in [-h, h]^2 around the nearest cell, the cell
    (i0 + a, j0 + b) of plane k receives w V c phi(i - x) phi(j - y) when it
    lies on the grid (phi the Gaussian g, or the ES kernel); taps off the
    grid are dropped and counted.
    Returns (planes, n_dropped_taps).
    """
    vis = np.asarray(vis).astype(np.complex128)
    m = vis.shape[0]
    x, y, i0, j0, k = coordinates(p, uvw)
    wv = _weights(weight, m) * vis
    h = (p.support - 1) // 2
    c = kernel_norm(p)
    ncell = p.nw * p.nv * p.nu
    re = np.zeros(ncell)
    im = np.zeros(ncell)
    dropped = 0
    for b in range(-h, h + 1):
        j = j0 + b
        gy = kernel_1d(p, j - y)
        for a in range(-h, h + 1):
            i = i0 + a
            on = (i >= 0) & (i < p.nu) & (j >= 0) & (j < p.nv)
            dropped += int(m - np.count_nonzero(on))
            val = wv[on] * (c * kernel_1d(p, i[on] - x[on]) * gy[on])
            flat = (k[on] * p.nv + j[on]) * p.nu + i[on]
            re += np.bincount(flat, weights=val.real, minlength=ncell)
            im += np.bincount(flat, weights=val.imag, minlength=ncell)
    planes = (re + 1j * im).reshape(p.nw, p.nv, p.nu)
    return planes, dropped


# ---------------------------------------------------------------------------
# Step 3 - per-plane 2-D FFT (Sec. 2, Eq. (2) inner integral)
# ---------------------------------------------------------------------------

def fft_planes(p: Params, planes, direction: int = +1):
    """Centred, unnormalised 2-D DFT of every plane.

    direction +1 (imaging, Eq. (2)):
      F[q][p] = sum_{j,i} P[j][i] exp(+2 pi i [(i - Nu/2)(p - Nu/2)/Nu
                                               + (j - Nv/2)(q - Nv/2)/Nv])
    direction -1 uses exp(-2 pi i ...), the adjoint transform.
    """
    planes = np.asarray(planes, dtype=np.complex128)
    shifted = np.fft.ifftshift(planes, axes=(-2, -1))
    if direction > 0:
        out = np.fft.ifft2(shifted, axes=(-2, -1)) * (p.nu * p.nv)
    else:
        out = np.fft.fft2(shifted, axes=(-2, -1))
    return np.fft.fftshift(out, axes=(-2, -1))


# ---------------------------------------------------------------------------
# Step 4 - w-screen and plane sum (Eq. (2) outer integral)
# ---------------------------------------------------------------------------

def sky_coords(p: Params):
    """Direction cosines (l, m) of pixel centres, l_p = (p - Nu/2) fov_l/Nu."""
    l = (np.arange(p.nu) - p.nu / 2) * (p.fov_l / p.nu)
    mm = (np.arange(p.nv) - p.nv / 2) * (p.fov_m / p.nv)
    return l, mm


def n_minus_one(l, m):
    """sqrt(1 - l^2 - m^2) - 1 without cancellation: -r^2/(1 + sqrt(1 - r^2))."""
    r2 = np.asarray(l, np.float64) ** 2 + np.asarray(m, np.float64) ** 2
    return -r2 / (1.0 + np.sqrt(1.0 - r2))


def screen_nm1(p: Params):
    """n - 1 on the image grid, indexed [q][p]."""
    l, mm = sky_coords(p)
    return n_minus_one(l[None, :], mm[:, None])


def wcorrect(p: Params, fplanes):
    """I[q][p] = sum_k F_k[q][p] exp(+2 pi i w_k (n_pq - 1)), times the
    grid correction when ``p.correct``."""
    nm1 = screen_nm1(p)
    img = np.zeros((p.nv, p.nu), dtype=np.complex128)
    for k, wk in enumerate(plane_centres(p)):
        img += fplanes[k] * np.exp(2j * math.pi * wk * nm1)
    if p.correct:
        img = img * grid_correction(p)
    return img


def image(p: Params, uvw, vis, weight=None):
    """Dirty image: gridding -> per-plane FFT -> w-screen and sum."""
    planes, _ = grid(p, uvw, vis, weight)
    return wcorrect(p, fft_planes(p, planes, +1))


# ---------------------------------------------------------------------------
# Adjoint: degridding (the paper's future work, Sec. 5)
# ---------------------------------------------------------------------------

def degrid(p: Params, img, uvw, weight=None):
    """Exact adjoint of ``image``: image -> visibilities.

    Q_k = FFT^-(conj(screen_k) X); V_m = w_m sum_taps c phi phi Q_{k(m)}[j][i],
    taps off the grid contributing nothing (X first multiplied by the grid
    correction when ``p.correct``).
    """
    img = np.asarray(img).astype(np.complex128)
    if p.correct:
        img = img * grid_correction(p)
    nm1 = screen_nm1(p)
    wks = plane_centres(p)
    q = np.stack([img * np.exp(-2j * math.pi * wk * nm1) for wk in wks])
    q = fft_planes(p, q, -1)
    m = np.asarray(uvw).shape[0]
    x, y, i0, j0, k = coordinates(p, uvw)
    h = (p.support - 1) // 2
    c = kernel_norm(p)
    out = np.zeros(m, dtype=np.complex128)
    qflat = q.reshape(-1)
    for b in range(-h, h + 1):
        j = j0 + b
        gy = kernel_1d(p, j - y)
        for a in range(-h, h + 1):
            i = i0 + a
            on = (i >= 0) & (i < p.nu) & (j >= 0) & (j < p.nv)
            flat = (k[on] * p.nv + j[on]) * p.nu + i[on]
            out[on] += c * kernel_1d(p, i[on] - x[on]) * gy[on] * qflat[flat]
    return _weights(weight, m) * out


# ---------------------------------------------------------------------------
# Direct forms for sampled outputs at full size (no FFT, no plane stack)
# ---------------------------------------------------------------------------

def grid_cells_direct(p: Params, uvw, vis, weight, cells):
    """P[k][j][i] at the given (k, j, i) cells, summed visibility by visibility."""
    vis = np.asarray(vis).astype(np.complex128)
    x, y, i0, j0, kk = coordinates(p, uvw)
    wv = _weights(weight, vis.shape[0]) * vis
    h = (p.support - 1) // 2
    c = kernel_norm(p)
    out = []
    for (k, j, i) in cells:
        sel = (kk == k) & (np.abs(i0 - i) <= h) & (np.abs(j0 - j) <= h)
        out.append(np.sum(wv[sel] * c * kernel_1d(p, i - x[sel])
                          * kernel_1d(p, j - y[sel])))
    return np.array(out, dtype=np.complex128)


def image_pixels_direct(p: Params, uvw, vis, weight, pixels, block=1 << 20):
    """Dirty-image pixels I[q][p] from the definition, without an FFT.

    Each visibility contributes w V exp(2 pi i w_k (n - 1)) times the DFT of
    its own on-grid taps; the tap sum separates into a u factor and a v
    factor.  ``pixels`` is a list of (q, p) pairs.
    """
    uvw = np.asarray(uvw, np.float64)
    vis = np.asarray(vis).astype(np.complex128)
    m = vis.shape[0]
    wts = _weights(weight, m)
    h = (p.support - 1) // 2
    c = kernel_norm(p)
    wks = plane_centres(p)
    l_all, m_all = sky_coords(p)
    res = np.zeros(len(pixels), dtype=np.complex128)
    for start in range(0, m, block):
        sl = slice(start, min(m, start + block))
        x, y, i0, j0, k = coordinates(p, uvw[sl])
        wv = wts[sl] * vis[sl]
        for t, (qq, pp) in enumerate(pixels):
            fu = (pp - p.nu / 2) / p.nu
            fv = (qq - p.nv / 2) / p.nv
            su = np.zeros(x.shape, np.complex128)
            sv = np.zeros(x.shape, np.complex128)
            for a in range(-h, h + 1):
                i = i0 + a
                onu = (i >= 0) & (i < p.nu)
                su += np.where(onu, kernel_1d(p, i - x), 0.0) * np.exp(
                    2j * math.pi * (i - p.nu / 2) * fu)
                j = j0 + a
                onv = (j >= 0) & (j < p.nv)
                sv += np.where(onv, kernel_1d(p, j - y), 0.0) * np.exp(
                    2j * math.pi * (j - p.nv / 2) * fv)
            nm1 = n_minus_one(l_all[pp], m_all[qq])
            ph = np.exp(2j * math.pi * wks[k] * nm1)
            res[t] += np.sum(wv * c * su * sv * ph)
    if p.correct:
        corr = grid_correction(p)
        res *= np.array([corr[qq, pp] for qq, pp in pixels])
    return res


def dft_image(p: Params, uvw, vis, weight, pixels=None):
    """Ideal dirty image from Eqs. (1)-(2) with no gridding at all.

    I(l, m) = sum_m w V exp(+2 pi i (u l + v m + w (n - 1))).  The w-stacked
    image equals this times the kernel's Fourier taper when every w sits on a
    plane centre, up to the kernel's aliasing and truncation.
    """
    uvw = np.asarray(uvw, np.float64)
    wv = _weights(weight, uvw.shape[0]) * np.asarray(vis).astype(np.complex128)
    l_all, m_all = sky_coords(p)
    if pixels is None:
        pixels = [(q, pp) for q in range(p.nv) for pp in range(p.nu)]
    out = np.empty(len(pixels), dtype=np.complex128)
    for t, (q, pp) in enumerate(pixels):
        l, mm = l_all[pp], m_all[q]
        ph = uvw[:, 0] * l + uvw[:, 1] * mm + uvw[:, 2] * n_minus_one(l, mm)
        out[t] = np.sum(wv * np.exp(2j * math.pi * ph))
    return out


def kernel_taper(p: Params):
    """Continuous Fourier transform of c g(x) g(y) at pixel (q, p), [q][p].

    exp(-2 pi^2 sigma^2 (f_p^2 + f_q^2)) with f_p = (p - Nu/2)/Nu.
    """
    s = kernel_sigma(p)
    fp = (np.arange(p.nu) - p.nu / 2) / p.nu
    fq = (np.arange(p.nv) - p.nv / 2) / p.nv
    return np.exp(-2 * math.pi ** 2 * s * s * (fp[None, :] ** 2
                                                + fq[:, None] ** 2))


# ---------------------------------------------------------------------------
# Cost bookkeeping (Sec. 4.2)
# ---------------------------------------------------------------------------

def grid_point_additions(p: Params, uvw) -> int:
    """Number of on-grid kernel taps: the paper's grid-point additions."""
    x, y, i0, j0, k = coordinates(p, uvw)
    h = (p.support - 1) // 2
    cols = np.clip(np.minimum(i0 + h, p.nu - 1) - np.maximum(i0 - h, 0) + 1,
                   0, None)
    rows = np.clip(np.minimum(j0 + h, p.nv - 1) - np.maximum(j0 - h, 0) + 1,
                   0, None)
    return int(np.sum(cols * rows))


def mesh_bytes(nu: int, nv: int, nw: int, complex_bytes: int = 16) -> int:
    """Bytes of one N_u x N_v x N_w complex mesh (real + imaginary parts)."""
    return nu * nv * nw * complex_bytes


# ---------------------------------------------------------------------------
# Baseline-major data (Sec. 2: the data structures; Sec. 3.4.2: one GPU
# thread per measurement convolves all of its frequencies and polarisations)
# ---------------------------------------------------------------------------

SPEED_OF_LIGHT = 299_792_458.0  # m/s


def stokes_coefficients(stokes: str, feeds: str = "linear"):
    """Coefficients a_p over the four correlations that give one Stokes
    parameter as sum_p a_p V_p.

    Reading: linear feeds correlate as XX = I + Q, XY = U + iV, YX = U - iV,
    YY = I - Q; circular feeds as RR = I + V, RL = Q + iU, LR = Q - iU,
    LL = I - V.  Solving for the Stokes parameters gives the rows below.
    """
    h = 0.5
    lin = {"I": [h, 0, 0, h], "Q": [h, 0, 0, -h], "U": [0, h, h, 0],
           "V": [0, -0.5j, 0.5j, 0]}
    circ = {"I": [h, 0, 0, h], "V": [h, 0, 0, -h], "Q": [0, h, h, 0],
            "U": [0, -0.5j, 0.5j, 0]}
    table = lin if feeds == "linear" else circ
    return np.array(table[stokes], dtype=np.complex128)


def expand_rows(uvw_m, freq_hz, vis, weight, pol_coeff):
    """Flatten baseline-major data to one visibility per (row, channel).

    uvw_m [R, 3] in metres per (baseline, time) row; freq_hz [C]; vis
    [R, C, P] complex; weight [R, P] (per measurement and polarisation) or
    None (unit); pol_coeff [P] complex.  Returns (uvw [R*C, 3] in
    wavelengths, vis [R*C], None): u_lambda = u_m (f / c) and the gridded
    value sum_p a_p w_p V_p, each with unit weight.  Row r, channel c is
    entry r*C + c.
    """
    uvw_m = np.asarray(uvw_m, dtype=np.float64)
    scale = np.asarray(freq_hz, dtype=np.float64) / SPEED_OF_LIGHT
    nr, nc = uvw_m.shape[0], scale.shape[0]
    uvw = (uvw_m[:, None, :] * scale[None, :, None]).reshape(nr * nc, 3)
    vis = np.asarray(vis).astype(np.complex128)
    coeff = np.asarray(pol_coeff, dtype=np.complex128)
    npol = coeff.shape[0]
    w = (np.ones((nr, npol)) if weight is None
         else np.asarray(weight, dtype=np.float64))
    comb = np.zeros((nr, nc), dtype=np.complex128)
    for p in range(npol):
        comb += (coeff[p] * w[:, p])[:, None] * vis[:, :, p]
    return uvw, comb.reshape(nr * nc), None


# ---------------------------------------------------------------------------
# Imaging major cycle (Sec. 1: imaging is followed by deconvolution with the
# CLEAN algorithm and its variants - Hogbom's image-plane loop, and the
# major / minor cycle split of Clark and of Schwab, in which the model is
# subtracted from the visibilities, not from the image, between minor
# cycles).
#
# Readings (the paper cites these methods but does not restate them):
# * the measurement operator predicts model visibilities with unit weights
#   (degrid(model) with weight None); the weights enter when the residual
#   visibilities are imaged (natural weighting, as for the dirty image);
# * images are real: the real part of the w-stacked image (the input is
#   taken to be Hermitian, so the imaginary part is rounding);
# * dirty beam: b = Re(image of unit visibilities), normalised by its value
#   at the centre pixel (N_v/2, N_u/2), beta; residual images are divided by
#   the same beta, so that a point source of flux S shows a peak of ~S;
# * minor cycle (Hogbom): the pixel of largest |D| (the first in row-major
#   order on ties) gets gain * D there added to the model, and gain * D
#   times b centred on that pixel (b[q - q* + N_v/2][p - p* + N_u/2], where
#   that index lies on the grid; the rest of the beam is truncated) is
#   subtracted from D; the cycle stops after niter components or when the
#   peak falls below the threshold;
# * major cycle: residual visibilities R = V - degrid(model), residual
#   image D = Re(image(R, weights)) / beta, then a minor cycle, n_major
#   times; the returned residual image is that of the final model.
# ---------------------------------------------------------------------------

def dirty_beam(p: Params, uvw, weight=None):
    """(b, beta): the normalised dirty beam and its centre value."""
    ones = np.ones(np.asarray(uvw).shape[0], dtype=np.complex128)
    img = image(p, uvw, ones, weight).real
    beta = float(img[p.nv // 2, p.nu // 2])
    return img / beta, beta


def hogbom(residual, beam, niter, gain, threshold=0.0, picks=None):
    """Hogbom minor cycle on a real residual image (modified copy returned).

    Returns (model, residual, components): ``components`` lists
    (q, p, value) for each step, the value being the residual at the pixel
    before the step.  With ``picks`` (a list of (q, p)), those pixels are
    taken in turn instead of the argmax (to replay a sequence chosen in
    another precision); the argmax is still what a free run would take.
    """
    d = np.array(residual, dtype=np.float64, copy=True)
    b = np.asarray(beam, dtype=np.float64)
    nv, nu = d.shape
    model = np.zeros_like(d)
    comps = []
    steps = niter if picks is None else min(niter, len(picks))
    for t in range(steps):
        if picks is None:
            flat = int(np.argmax(np.abs(d)))
            q, pp = divmod(flat, nu)
        else:
            q, pp = picks[t]
        a = float(d[q, pp])
        if abs(a) < threshold:
            break
        comps.append((q, pp, a))
        model[q, pp] += gain * a
        # beam centred on (q, pp), truncated at the grid edges
        q0, q1 = max(0, q - nv // 2), min(nv, q + nv // 2)
        p0, p1 = max(0, pp - nu // 2), min(nu, pp + nu // 2)
        d[q0:q1, p0:p1] -= gain * a * b[q0 - q + nv // 2:q1 - q + nv // 2,
                                        p0 - pp + nu // 2:p1 - pp + nu // 2]
    return model, d, comps


def residual_image(p: Params, uvw, vis, weight, model, beta):
    """Re(image(V - degrid(model), weights)) / beta."""
    pred = degrid(p, model, uvw, None)
    r = np.asarray(vis).astype(np.complex128) - pred
    return image(p, uvw, r, weight).real / beta


def major_cycle(p: Params, uvw, vis, weight, n_major, n_minor, gain,
                threshold=0.0, picks=None):
    """Cotton-Schwab major cycles with Hogbom minor cycles.

    Returns (model, residual image of the final model, components per
    major cycle, beam, beta).  ``picks``: per major cycle, a forced pixel
    sequence (see ``hogbom``).
    """
    b, beta = dirty_beam(p, uvw, weight)
    model = np.zeros((p.nv, p.nu))
    history = []
    for j in range(n_major):
        d = residual_image(p, uvw, vis, weight, model, beta)
        dm, _, comps = hogbom(d, b, n_minor, gain, threshold,
                              None if picks is None else picks[j])
        model = model + dm
        history.append(comps)
    return model, residual_image(p, uvw, vis, weight, model, beta), \
        history, b, beta
