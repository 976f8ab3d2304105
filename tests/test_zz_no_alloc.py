"""The allocation-free entry point (ws_grid_image_noalloc) against the
plan-based one (ws_grid_init + ws_grid_image) on the same inputs, through
the C ABI: two calls in a row, the second with a smaller input (and a
different grid), so that the second reads a scratch the first left dirty.
Bar: FP64 rel-max 1e-12, FP32 rel-L2 1e-5; dropped-tap counts exact."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
import paper_2301_06061_amd as ws  # noqa: E402
from paper_2301_06061_amd import api  # noqa: E402

pytestmark = pytest.mark.gpu


def _rel(a, b, fp64):
    a = a.to(torch.complex128)
    b = b.to(torch.complex128)
    if fp64:
        return float((a - b).abs().max() / b.abs().max())
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_matches_plan_path_twice(precision):
    d = torch.device("cuda", 0)
    prec = 1 if precision == "fp64" else 0
    cases = [synth.random_case(71, n=512, nw=6, support=7, m=200_000,
                               law="core", precision=prec),
             synth.edge_case(72, n=256, nv=128, nw=4, support=9, m=3000,
                             precision=prec),
             synth.random_case(73, n=128, nw=3, support=7, m=1000,
                               law="core", precision=prec)]
    # The third call: the ES kernel with grid correction (its table also
    # lives in the scratch).
    cases[2].kernel = "es"
    cases[2].correct = True
    for wl in cases:
        params = api.make_params(wl.nu, wl.nv, wl.nw, wl.fov_l, wl.fov_m,
                                 wl.w_min, wl.w_max, wl.support, wl.sigma,
                                 precision, kernel=wl.kernel,
                                 correct=wl.correct)
        uvw = torch.from_numpy(wl.uvw).to(d)
        vis = torch.from_numpy(wl.vis).to(d)
        wt = torch.from_numpy(wl.weight).to(d)
        drop_a = torch.zeros(1, dtype=torch.int64, device=d)
        got = api.grid_image_noalloc(params, uvw, vis, wt, dropped=drop_a)
        plan = ws.WStackPlan.from_workload(wl)
        drop_b = torch.zeros(1, dtype=torch.int64, device=d)
        plan.reset()
        ref = plan.grid_image(uvw, vis, wt, dropped=drop_b)
        torch.cuda.synchronize()
        err = _rel(got, ref, precision == "fp64")
        assert err <= (1e-12 if precision == "fp64" else 1e-5), err
        assert int(drop_a.item()) == int(drop_b.item())
        plan.close()


def test_noalloc_refuses_oversized_problems():
    d = torch.device("cuda", 0)
    params = api.make_params(4096, 4096, 32, 0.08, 0.08, -1.0, 1.0, 7, 0.0,
                             "fp32")
    uvw = torch.zeros((10, 3), dtype=torch.float64, device=d)
    vis = torch.zeros(10, dtype=torch.complex64, device=d)
    img = torch.zeros((4096, 4096), dtype=torch.complex64, device=d)
    with pytest.raises(ws.WStackError) as e:
        api.grid_image_noalloc(params, uvw, vis, image=img)
    assert e.value.status == -3
    assert float(img.abs().max()) == 0.0
