"""Baseline-major input on the GPU (ws_grid_rows, ws_grid_image_rows)
against the oracle.

Paper passages: Sec. 2, data structures ((u, v, w) per baseline and time,
visibilities per frequency channel and polarisation, weights per
measurement and polarisation); Sec. 3.4.2 (one thread per measurement
convolves all of its frequencies and polarisations); Sec. 5 (full
multi-wavelength and polarisation support as future work).

The oracle flattens the rows (``expand_rows``: u_lambda = u_m f / c, value
sum_p a_p w_p V_p with unit weight) and grids the result; the library
scales and combines on the fly inside its binning kernels.  Tolerances as
in the other parity tests; dropped-tap counts exact.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import wstack as o  # noqa: E402
import paper_2301_06061_amd as ws  # noqa: E402

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def _err(got, ref, fp64):
    got = np.asarray(got, np.complex128)
    ref = np.asarray(ref, np.complex128)
    if fp64:
        return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def _dev(rw):
    d = torch.device("cuda", 0)
    return (torch.from_numpy(rw.uvw_m).to(d),
            torch.from_numpy(rw.freq_hz).to(d),
            torch.from_numpy(np.ascontiguousarray(rw.vis)).to(d),
            torch.from_numpy(rw.weight).to(d))


COEFFS = {
    "I-linear": o.stokes_coefficients("I", "linear"),
    "V-linear": o.stokes_coefficients("V", "linear"),
    "U-circular": o.stokes_coefficients("U", "circular"),
    "two-pol": np.array([0.3, -2.0j]),
    "one-pol": np.array([1.0]),
}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(COEFFS))
def test_grid_rows_matches_oracle(precision, name):
    coef = COEFFS[name]
    npol = coef.shape[0]
    fp64 = precision == "fp64"
    rw = synth.rows_case(3, n=128, nw=4, support=7, nrows=600, nchan=6,
                         npol=npol, precision=1 if fp64 else 0)
    uvw, vis, _ = o.expand_rows(rw.uvw_m, rw.freq_hz, rw.vis, rw.weight, coef)
    p = o.Params.of(rw.geo)
    ref, drop_ref = o.grid(p, uvw, vis, None)
    du, df, dv, dw = _dev(rw)
    plan = ws.WStackPlan.from_workload(rw.geo, max_vis=600 * 6)
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    plan.grid_rows(du, df, dv, dw, coef, dropped)
    torch.cuda.synchronize()
    err = _err(plan.planes.cpu().numpy(), ref, fp64)
    assert err <= (TOL64 if fp64 else TOL32), err
    assert int(dropped.item()) == drop_ref
    # and the one-call image
    img_ref = o.image(p, uvw, vis, None)
    plan.reset()
    img = plan.grid_image_rows(du, df, dv, dw, coef)
    torch.cuda.synchronize()
    err = _err(img.cpu().numpy(), img_ref, fp64)
    assert err <= (TOL64 if fp64 else TOL32), err


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_grid_rows_unit_weights_and_lazy_path(precision):
    """No weights (unit), ES kernel with correction, 512^2 so the one-call
    path leaves tiles without records unwritten; additive gridding of two
    row batches equals the oracle image of both."""
    fp64 = precision == "fp64"
    rw = synth.rows_case(8, n=512, nw=3, support=7, nrows=3000, nchan=5,
                         npol=2, precision=1 if fp64 else 0)
    rw.geo.kernel = "es"
    coef = np.array([0.5, 0.5])
    uvw, vis, _ = o.expand_rows(rw.uvw_m, rw.freq_hz, rw.vis, None, coef)
    p = o.Params.of(rw.geo)
    ref = o.image(p, uvw, vis, None)
    du, df, dv, _ = _dev(rw)
    plan = ws.WStackPlan.from_workload(rw.geo, max_vis=3000 * 5)
    img = plan.grid_image_rows(du, df, dv, None, coef)
    torch.cuda.synchronize()
    assert _err(img.cpu().numpy(), ref, fp64) <= (TOL64 if fp64 else TOL32)
    # two batches of rows, additive, then the fused image pass
    plan.reset()
    plan.grid_rows(du[:1200], df, dv[:1200], None, coef)
    plan.grid_rows(du[1200:], df, dv[1200:], None, coef)
    img2 = plan.new_image()
    plan.image_accumulate(img2)
    torch.cuda.synchronize()
    assert _err(img2.cpu().numpy(), ref, fp64) <= (TOL64 if fp64 else TOL32)


def test_grid_rows_edges_and_errors():
    """A channel scaling that pushes footprints off the grid (exact dropped
    counts), no rows, and the refused argument sets."""
    rw = synth.rows_case(4, n=64, nw=2, support=7, nrows=300, nchan=3,
                         npol=1, precision=1)
    # the last channel at twice the highest drawn frequency: positions
    # double, many footprints leave the grid
    rw.freq_hz = np.array([rw.freq_hz[0], rw.freq_hz[-1],
                           2.0 * rw.freq_hz[-1]])
    coef = np.array([1.0])
    uvw, vis, _ = o.expand_rows(rw.uvw_m, rw.freq_hz, rw.vis, rw.weight, coef)
    p = o.Params.of(rw.geo)
    ref, drop_ref = o.grid(p, uvw, vis, None)
    assert drop_ref > 0
    du, df, dv, dw = _dev(rw)
    plan = ws.WStackPlan.from_workload(rw.geo, max_vis=900)
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    plan.grid_rows(du, df, dv, dw, coef, dropped)
    torch.cuda.synchronize()
    assert _err(plan.planes.cpu().numpy(), ref, True) <= TOL64
    assert int(dropped.item()) == drop_ref
    # no rows: nothing added
    plan.reset()
    img = plan.grid_image_rows(du[:0], df, dv[:0], dw[:0], coef)
    torch.cuda.synchronize()
    assert float(img.abs().max()) == 0.0
    # refused: too many correlations, too many visibilities, NaN coefficient
    big = torch.zeros((400, 3, 1), dtype=plan.cdtype, device="cuda")
    with pytest.raises(ws.WStackError) as e:
        plan.grid_rows(torch.zeros((400, 3), dtype=torch.float64,
                                   device="cuda"), df, big,
                       None, coef)
    assert e.value.status == -3
    five = torch.zeros((10, 3, 5), dtype=plan.cdtype, device="cuda")
    with pytest.raises(ws.WStackError) as e:
        plan.grid_rows(du[:10], df, five, None, np.ones(5))
    assert e.value.status == -1
    with pytest.raises(ws.WStackError) as e:
        plan.grid_rows(du, df, dv, dw, np.array([np.nan]))
    assert e.value.status == -1


@pytest.mark.parametrize("feeds", ["linear", "circular"])
def test_rows_point_source_stokes_on_gpu(feeds):
    """A point source at a pixel centre, its correlations synthesised from
    the measurement equation (Eq. 1) per channel with each Stokes
    parameter's coefficients: the ES-corrected GPU image at that pixel
    equals S x (sum of weights), per Stokes parameter, to the kernel's
    aliasing (the oracle's pin of the same relation)."""
    n, nw = 128, 1
    fov = np.radians(2.0)
    rng = np.random.default_rng(5)
    nr, freqs = 200, np.array([100e6, 130e6, 170e6])
    half = n / 2 - 5
    cells = rng.uniform(-half, half, (nr, 2)) * 0.5
    uvw_m = np.zeros((nr, 3))
    uvw_m[:, :2] = cells / fov * (synth.workloads.C0 / freqs.max())
    pq = (n // 2 + 9, n // 2 - 14)   # pixel (p, q)
    l0 = (pq[0] - n / 2) * fov / n
    m0 = (pq[1] - n / 2) * fov / n
    S = {"I": 2.0, "Q": 0.5, "U": -0.7, "V": 0.3}
    I, Q, U, V = S["I"], S["Q"], S["U"], S["V"]
    corr = ([I + Q, U + 1j * V, U - 1j * V, I - Q] if feeds == "linear"
            else [I + V, Q + 1j * U, Q - 1j * U, I - V])
    lam = uvw_m[:, None, :] * (freqs / synth.workloads.C0)[None, :, None]
    # Eq. (1) with the image's sign convention: the source at (l0, m0)
    ph = np.exp(-2j * np.pi * (lam[..., 0] * l0 + lam[..., 1] * m0))
    vis = ph[:, :, None] * np.array(corr)[None, None, :]
    wt = np.ones((nr, 4), np.float32)
    geo = synth.Workload(n, n, nw, fov, fov, -1.0, 1.0, 7, precision=1)
    geo.kernel = "es"
    geo.correct = True
    d = torch.device("cuda", 0)
    plan = ws.WStackPlan.from_workload(geo, max_vis=nr * len(freqs))
    for s, val in S.items():
        a = o.stokes_coefficients(s, feeds)
        plan.reset()
        img = plan.grid_image_rows(torch.from_numpy(uvw_m).to(d),
                                   torch.from_numpy(freqs).to(d),
                                   torch.from_numpy(vis).to(d),
                                   torch.from_numpy(wt).to(d), a)
        torch.cuda.synchronize()
        got = img[pq[1], pq[0]].item()
        want = val * nr * len(freqs)
        assert abs(got - want) <= 1e-5 * nr * len(freqs), (s, got, want)
