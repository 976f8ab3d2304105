"""Edge cases of the method on the GPU, element by element against the oracle.

Footprints that hang off each edge and corner of the grid (taps dropped and
counted; the degridder's halo cells off the grid read as zero), footprints
wholly off the grid, non-finite coordinates, w below w_min and above w_max
(clamped to the end planes) and w exactly on a plane boundary
w_min + k dw (plane k; the boundary values are exact in FP64 here, so both
sides take the same floor).  Each case runs through gridding alone, the
one-call grid + image and degridding (real and complex images).

Tolerances as in test_gpu_parity: FP64 rel-max 1e-12, FP32 rel-L2 1e-5;
dropped-tap counts exact.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import wstack as o  # noqa: E402
import paper_2301_06061_amd as ws  # noqa: E402

from test_gpu_parity import assert_close, dev, host  # noqa: E402

pytestmark = pytest.mark.gpu


def _run_all(wl, tile, precision):
    p = o.Params.of(wl)
    fp64 = precision == "fp64"
    plan = ws.WStackPlan.from_workload(wl, tile=tile)
    uvw, vis, wt = dev(wl)
    d = torch.device("cuda", 0)
    # gridding alone
    ref_planes, ref_drop = o.grid(p, wl.uvw, wl.vis, wl.weight)
    dropped = torch.zeros(1, dtype=torch.int64, device=d)
    plan.reset()
    plan.grid(uvw, vis, wt, dropped)
    assert_close(host(plan.planes), ref_planes, fp64, "edge planes")
    assert int(dropped.item()) == ref_drop
    # one-call grid + image
    dropped.zero_()
    plan.reset()
    img = plan.grid_image(uvw, vis, wt, dropped=dropped)
    ref_img = o.wcorrect(p, o.fft_planes(p, ref_planes, +1))
    assert_close(host(img), ref_img, fp64, "edge image")
    assert int(dropped.item()) == ref_drop
    # degridding, real and complex images; entries with no tap on the grid
    # must come back as exact zeros (the output starts as NaN here)
    rng = np.random.default_rng(wl.support * 100 + tile)
    for real in (True, False):
        x = rng.standard_normal((wl.nv, wl.nu))
        if not real:
            x = x + 1j * rng.standard_normal((wl.nv, wl.nu))
        xt = torch.from_numpy(x).to(d).to(plan.rdtype if real else plan.cdtype)
        out = torch.full((wl.m,), complex(float("nan"), float("nan")),
                         dtype=plan.cdtype, device=d)
        got = host(plan.degrid(xt, uvw, wt, out=out))
        ref = o.degrid(p, x, wl.uvw, wl.weight)
        assert np.all(np.isfinite(got)), "degrid left entries unwritten"
        assert np.all(got[ref == 0] == 0)
        assert_close(got, ref, fp64, f"edge degrid real={real}")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("tile", [16, 32, 64])
@pytest.mark.parametrize("support", [1, 7, 9, 15])
def test_footprints_off_every_edge(precision, tile, support):
    wl = synth.edge_case(10 + support, n=128, nw=4, support=support,
                         m=3000, precision=1 if precision == "fp64" else 0)
    _run_all(wl, tile, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(512, 256), (64, 128)])
def test_edges_non_square_and_lazy_image(precision, shape):
    """Non-square grids; (512, 256) with 64-cell tiles takes the one-call
    form that never writes tiles without records."""
    nu, nv = shape
    wl = synth.edge_case(77, n=nu, nv=nv, nw=8, support=7, m=4000,
                         precision=1 if precision == "fp64" else 0)
    _run_all(wl, 64 if nu >= 512 else 32, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_w_clamp_and_plane_boundaries(precision):
    """Only w matters here: every visibility well inside the grid, w below,
    above and exactly on plane boundaries (including w_max itself, which
    belongs to the last plane)."""
    wl = synth.edge_case(5, n=64, nw=8, support=7, m=4000, bad=False,
                         precision=1 if precision == "fp64" else 0)
    rng = np.random.default_rng(1)
    fov = wl.fov_l
    uvw = wl.uvw.copy()
    uvw[:, 0] = rng.uniform(-20, 20, wl.m) / fov
    uvw[:, 1] = rng.uniform(-20, 20, wl.m) / fov
    dw = (wl.w_max - wl.w_min) / wl.nw
    uvw[:16, 2] = wl.w_min + np.arange(16) % (wl.nw + 1) * dw
    wl.uvw = np.ascontiguousarray(uvw)
    p = o.Params.of(wl)
    k = o.coordinates(p, wl.uvw)[4]
    # every plane holds data, and the boundary values went to plane k
    assert np.all(np.bincount(k, minlength=wl.nw) > 0)
    assert list(k[:9]) == [0, 1, 2, 3, 4, 5, 6, 7, 7]
    _run_all(wl, 16, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_narrow_kernel_small_sigma(precision):
    """Support 15 with sigma 0.15 cells: the far taps underflow to zero in
    FP64 (the gridder's tap recurrence must not turn them into NaN)."""
    wl = synth.random_case(91, n=64, nw=2, support=15, m=2000, law="gauss",
                           sigma=0.15,
                           precision=1 if precision == "fp64" else 0)
    p = o.Params.of(wl)
    plan = ws.WStackPlan.from_workload(wl, tile=16)
    uvw, vis, wt = dev(wl)
    plan.reset()
    plan.grid(uvw, vis, wt)
    got = host(plan.planes)
    ref, _ = o.grid(p, wl.uvw, wl.vis, wl.weight)
    assert np.all(np.isfinite(got))
    assert_close(got, ref, precision == "fp64", "narrow kernel planes")
