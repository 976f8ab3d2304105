"""Whole images and whole degridded outputs at the widths the benchmark and
the differentiable workload run (2048 and 4096 cells), element by element
against the oracle.

At these widths the fused row kernels take their widest instances (the
row transform + screen + plane sum of the imaging path, and the conjugate
screen + row transform of degridding); the one-call path leaves tiles
without records unwritten and the column transform reads by tile counts.
A few thousand visibilities and 2-3 planes keep the oracle to seconds.
Tolerances: FP64 rel-max 1e-12, FP32 rel-L2 1e-5.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import wstack as o  # noqa: E402
import paper_2301_06061_amd as ws  # noqa: E402

from test_gpu_parity import assert_close, dev, host  # noqa: E402

pytestmark = pytest.mark.gpu

SHAPES = {2048: 3, 4096: 2}
_cache = {}


def _case(n, precision):
    key = (n, precision)
    if key not in _cache:
        wl = synth.random_case(60 + n // 1024, n=n, nw=SHAPES[n], support=7,
                               m=4000, law="core", fov_deg=5.0,
                               precision=1 if precision == "fp64" else 0)
        p = o.Params.of(wl)
        planes, drop = o.grid(p, wl.uvw, wl.vis, wl.weight)
        img = o.wcorrect(p, o.fft_planes(p, planes, +1))
        del planes
        _cache[key] = (wl, img, drop)
    return _cache[key]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("n", [2048, 4096])
def test_wide_grid_image(n, precision):
    """The benchmark's call (ws_grid_image) and the two-call form."""
    wl, ref, drop = _case(n, precision)
    plan = ws.WStackPlan.from_workload(wl)
    uvw, vis, wt = dev(wl)
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    plan.reset()
    img = plan.grid_image(uvw, vis, wt, dropped=dropped)
    assert_close(host(img), ref, precision == "fp64", f"grid_image {n}")
    assert int(dropped.item()) == drop
    img2 = plan.dirty_image(uvw, vis, wt, fused=False)
    assert_close(host(img2), ref, precision == "fp64", f"unfused {n}")
    plan.reset()
    plan.grid(uvw, vis, wt)
    img3 = plan.new_image()
    plan.image_accumulate(img3)
    assert_close(host(img3), ref, precision == "fp64",
                 f"grid + image_accumulate {n}")


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("n", [2048, 4096])
@pytest.mark.parametrize("real", [True, False])
def test_wide_degrid(n, precision, real):
    wl, _, _ = _case(n, precision)
    p = o.Params.of(wl)
    rng = np.random.default_rng(n + int(real))
    x = rng.standard_normal((n, n))
    if not real:
        x = x + 1j * rng.standard_normal((n, n))
    ref = o.degrid(p, x, wl.uvw, wl.weight)
    plan = ws.WStackPlan.from_workload(wl)
    uvw, _, wt = dev(wl)
    xt = torch.from_numpy(x).to("cuda").to(plan.rdtype if real
                                           else plan.cdtype)
    got = host(plan.degrid(xt, uvw, wt))
    assert_close(got, ref, precision == "fp64", f"degrid {n} real={real}")
