"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: the FP64 path must match the oracle to 1e-12 relative (max
error over the output, divided by its largest magnitude); the FP32 path to a
relative L2 error of 1e-5 over all complex outputs, the target the imaging
path is built to (FP32 data, FFT and accumulation; FP64 positions, plane
index and phase).  Integer outputs (dropped-tap counts) must match exactly.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import wstack as o  # noqa: E402
import paper_2301_06061_amd as ws  # noqa: E402

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def rel_l2(got, ref):
    got = np.asarray(got, np.complex128)
    ref = np.asarray(ref, np.complex128)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def rel_max(got, ref):
    got = np.asarray(got, np.complex128)
    ref = np.asarray(ref, np.complex128)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def assert_close(got, ref, fp64, what=""):
    if fp64:
        err = rel_max(got, ref)
        assert err <= TOL64, f"{what}: FP64 rel-max error {err:.3e}"
    else:
        err = rel_l2(got, ref)
        assert err <= TOL32, f"{what}: FP32 rel-L2 error {err:.3e}"


def dev(wl):
    d = torch.device("cuda", 0)
    uvw = torch.from_numpy(np.ascontiguousarray(wl.uvw)).to(d)
    vis = torch.from_numpy(np.ascontiguousarray(wl.vis)).to(d)
    wt = None if wl.weight is None else torch.from_numpy(
        np.ascontiguousarray(wl.weight)).to(d)
    return uvw, vis, wt


def plan_for(wl, **kw):
    return ws.WStackPlan.from_workload(wl, **kw)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


CASES = [
    dict(n=64, nw=3, support=7, m=3000, law="core"),
    dict(n=32, nw=1, support=15, m=500, law="gauss"),
    dict(n=128, nw=4, support=9, m=5000, law="core", tile=32),
    dict(n=64, nv=32, nw=2, support=5, m=2000, law="gauss"),
    dict(n=64, nw=2, support=1, m=1000, law="gauss"),
    dict(n=16, nw=5, support=3, m=300, law="core"),
    dict(n=256, nw=6, support=7, m=20000, law="core"),
]


def _case(c, precision, seed=3):
    kw = {k: v for k, v in c.items() if k not in ("tile",)}
    wl = synth.random_case(seed, precision=1 if precision == "fp64" else 0,
                           **kw)
    if c["nw"] == 1:
        wl.w_max = wl.w_min
    return wl


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("ci", range(len(CASES)))
def test_grid_matches_oracle(precision, ci):
    c = CASES[ci]
    wl = _case(c, precision)
    p = o.Params.of(wl)
    ref, ref_drop = o.grid(p, wl.uvw, wl.vis, wl.weight)
    plan = plan_for(wl, tile=c.get("tile", 0))
    uvw, vis, wt = dev(wl)
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    plan.grid(uvw, vis, wt, dropped)
    got = host(plan.planes)
    assert_close(got, ref, precision == "fp64", "planes")
    assert int(dropped.item()) == ref_drop


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(16, 16, 1), (64, 32, 3), (512, 512, 2),
                                   (32, 4096, 1), (4096, 16, 1),
                                   (16, 8192, 2), (32, 16384, 1),
                                   (8192, 16, 1), (16384, 16, 1),
                                   (32768, 16, 1), (16, 32768, 1)])
@pytest.mark.parametrize("direction", [1, -1])
def test_fft_planes_matches_oracle(precision, shape, direction):
    """One-pass and four-step columns; rows in LDS, split in two halves
    when a row exceeds LDS (FP64 at 16384, FP32 at 32768), or in four
    quarters through scratch rows (FP64 at 32768)."""
    nu, nv, nw = shape
    rng = np.random.default_rng(nu + nv + nw)
    cdt = np.complex128 if precision == "fp64" else np.complex64
    data = (rng.standard_normal((nw, nv, nu)) +
            1j * rng.standard_normal((nw, nv, nu))).astype(cdt)
    p = o.Params(nu, nv, nw, 0.02, 0.02, -1.0, 1.0, 7)
    plan = ws.WStackPlan(nu, nv, nw, p.fov_l, p.fov_m, -1.0, 1.0, 7,
                         precision=precision, max_vis=16,
                         tile=16 if min(nu, nv) < 64 else 0)
    e = torch.empty((0, 3), dtype=torch.float64, device="cuda")
    plan.grid(e, torch.empty(0, dtype=plan.cdtype, device="cuda"))
    plan.planes.copy_(torch.from_numpy(data))
    plan.fft(direction)
    got = host(plan.planes)
    ref = o.fft_planes(p, data, direction)
    assert_close(got, ref, precision == "fp64", "fft")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("fov_deg", [1.0, 8.0, 30.0])
def test_wcorrect_matches_oracle(precision, fov_deg):
    nu, nv, nw = 64, 32, 5
    rng = np.random.default_rng(5)
    cdt = np.complex128 if precision == "fp64" else np.complex64
    fov = math.radians(fov_deg)
    p = o.Params(nu, nv, nw, fov, fov * nv / nu, -3.0e4, 5.0e4, 7)
    data = (rng.standard_normal((nw, nv, nu)) +
            1j * rng.standard_normal((nw, nv, nu))).astype(cdt)
    plan = ws.WStackPlan(nu, nv, nw, p.fov_l, p.fov_m, p.w_min, p.w_max, 7,
                         precision=precision, max_vis=16, tile=16)
    # An empty plan transformed: zero planes in the transformed state, which
    # the screen then reads (here with arbitrary data written in).
    plan.reset()
    plan.fft(+1)
    plan.planes.copy_(torch.from_numpy(data))
    img = plan.new_image()
    img += 1.0  # accumulation adds to what is there
    plan.wcorrect(img)
    ref = o.wcorrect(p, data.astype(np.complex128)) + 1.0
    assert_close(host(img), ref, precision == "fp64", "wcorrect")


LARGE = [dict(n=16, nv=8192, nw=2, support=7, m=2000, law="core",
              fov_deg=0.005),
         dict(n=32, nv=16384, nw=3, support=9, m=2000, law="gauss",
              fov_deg=0.005),
         dict(n=8192, nv=16, nw=2, support=5, m=2000, law="core"),
         dict(n=16384, nv=16, nw=2, support=7, m=1000, law="gauss"),
         dict(n=32768, nv=16, nw=2, support=7, m=1000, law="gauss"),
         dict(n=16, nv=32768, nw=2, support=5, m=1000, law="core",
              fov_deg=0.005)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("ci", range(len(LARGE)))
def test_large_grid_image_and_degrid(precision, fused, ci):
    """Grids beyond the one-pass column FFT (four-step columns, transposed
    row order undone by the screen and gather kernels)."""
    c = LARGE[ci]
    wl = _case(c, precision, seed=21)
    p = o.Params.of(wl)
    plan = plan_for(wl)
    uvw, vis, wt = dev(wl)
    img = plan.dirty_image(uvw, vis, wt, fused=fused)
    assert_close(host(img), o.image(p, wl.uvw, wl.vis, wl.weight),
                 precision == "fp64", "large image")
    rng = np.random.default_rng(ci)
    x = rng.standard_normal((wl.nv, wl.nu))
    xt = torch.from_numpy(x).to("cuda").to(plan.rdtype)
    got = host(plan.degrid(xt, uvw, wt))
    assert_close(got, o.degrid(p, x, wl.uvw, wl.weight), precision == "fp64",
                 "large degrid")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("ci", [0, 2, 3, 5, 6])
def test_dirty_image_matches_oracle(precision, fused, ci):
    c = CASES[ci]
    wl = _case(c, precision, seed=8)
    p = o.Params.of(wl)
    ref = o.image(p, wl.uvw, wl.vis, wl.weight)
    plan = plan_for(wl, tile=c.get("tile", 0))
    uvw, vis, wt = dev(wl)
    img = plan.dirty_image(uvw, vis, wt, fused=fused)
    assert_close(host(img), ref, precision == "fp64", "image")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("real", [True, False])
@pytest.mark.parametrize("ci", [0, 1, 2, 3, 5])
def test_degrid_matches_oracle(precision, real, ci):
    c = CASES[ci]
    wl = _case(c, precision, seed=9)
    p = o.Params.of(wl)
    rng = np.random.default_rng(ci)
    x = rng.standard_normal((wl.nv, wl.nu))
    if not real:
        x = x + 1j * rng.standard_normal((wl.nv, wl.nu))
    ref = o.degrid(p, x, wl.uvw, wl.weight)
    plan = plan_for(wl, tile=c.get("tile", 0))
    uvw, _, wt = dev(wl)
    xt = torch.from_numpy(x).to("cuda").to(plan.rdtype if real else plan.cdtype)
    got = host(plan.degrid(xt, uvw, wt))
    assert_close(got, ref, precision == "fp64", "degrid")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_grid_is_additive_over_calls(precision):
    wl = _case(CASES[0], precision, seed=4)
    p = o.Params.of(wl)
    ref, _ = o.grid(p, wl.uvw, wl.vis, wl.weight)
    plan = plan_for(wl)
    uvw, vis, wt = dev(wl)
    plan.grid(uvw[:1000], vis[:1000], wt[:1000])
    plan.grid(uvw[1000:], vis[1000:], wt[1000:])
    assert_close(host(plan.planes), ref, precision == "fp64", "two calls")
    # a reset starts a new image
    plan.reset()
    plan.grid(uvw[:10], vis[:10], wt[:10])
    ref10, _ = o.grid(p, wl.uvw[:10], wl.vis[:10], wl.weight[:10])
    assert_close(host(plan.planes), ref10, precision == "fp64", "after reset")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_image_over_calls_and_reset_skips_only_empty_strips(precision):
    """The image path transforms only the column strips that gridding calls
    since the reset reached: two calls on opposite halves of the uv plane,
    then a reset and a call on one quarter, each imaged against the
    oracle."""
    wl = _case(dict(n=256, nw=4, support=7, m=6000, law="gauss"), precision,
               seed=31)
    p = o.Params.of(wl)
    plan = plan_for(wl, tile=32)
    uvw, vis, wt = dev(wl)
    left = wl.uvw[:, 0] < 0
    il = torch.from_numpy(np.nonzero(left)[0]).to("cuda")
    ir = torch.from_numpy(np.nonzero(~left)[0]).to("cuda")
    plan.grid(uvw[il], vis[il], wt[il])
    plan.grid(uvw[ir], vis[ir], wt[ir])
    img = plan.new_image()
    plan.image_accumulate(img)
    assert_close(host(img), o.image(p, wl.uvw, wl.vis, wl.weight),
                 precision == "fp64", "two calls")
    quarter = (wl.uvw[:, 0] > 0) & (wl.uvw[:, 1] > 0)
    iq = torch.from_numpy(np.nonzero(quarter)[0]).to("cuda")
    plan.reset()
    plan.grid(uvw[iq], vis[iq], wt[iq])
    img = plan.new_image()
    plan.image_accumulate(img)
    assert_close(host(img), o.image(p, wl.uvw[quarter], wl.vis[quarter],
                                    wl.weight[quarter]),
                 precision == "fp64", "after reset")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(512, 512, 4), (1024, 512, 3),
                                   (256, 256, 2)])
@pytest.mark.parametrize("law", ["core", "gauss"])
def test_grid_image_matches_oracle(precision, shape, law):
    """The one-call grid + image: the form that never zeroes the tiles
    without visibilities (tile edge 64, nu >= 512) and the plain form
    (nu = 256)."""
    nu, nv, nw = shape
    wl = synth.random_case(41, n=nu, nv=nv, nw=nw, support=7, m=20000,
                           law=law, precision=1 if precision == "fp64" else 0)
    plan = plan_for(wl, tile=64)
    uvw, vis, wt = dev(wl)
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = plan.grid_image(uvw, vis, wt, dropped=dropped)
    p = o.Params.of(wl)
    assert_close(host(img), o.image(p, wl.uvw, wl.vis, wl.weight),
                 precision == "fp64", "grid_image")
    assert int(dropped.item()) == o.grid(p, wl.uvw, wl.vis, wl.weight)[1]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_grid_image_reuses_a_dirty_stack(precision):
    """Same plan, same geometry, two data sets: the second call's idle
    tiles still hold the first call's sums and must not be read."""
    wl1 = synth.random_case(51, n=512, nw=4, support=7, m=30000, law="core",
                            precision=1 if precision == "fp64" else 0)
    wl2 = synth.random_case(52, n=512, nw=4, support=7, m=500, law="gauss",
                            precision=1 if precision == "fp64" else 0)
    wl2.w_min, wl2.w_max = wl1.w_min, wl1.w_max
    wl2.uvw[:, 2] = np.clip(wl2.uvw[:, 2], wl1.w_min, wl1.w_max)
    plan = plan_for(wl1, tile=64)
    for wl in (wl1, wl2, wl1):
        uvw, vis, wt = dev(wl)
        img = plan.grid_image(uvw, vis, wt)
        ref = o.image(o.Params.of(wl), wl.uvw, wl.vis, wl.weight)
        assert_close(host(img), ref, precision == "fp64", "reuse")
    with pytest.raises(ws.WStackError):
        plan.grid(uvw, vis, wt)
        plan.grid_image(uvw, vis, wt)


@pytest.mark.parametrize("precision,shape", [
    ("fp64", (8192, 512, 2)), ("fp32", (8192, 512, 2)),
    ("fp64", (512, 8192, 2)), ("fp32", (512, 8192, 2)),
    ("fp32", (8192, 8192, 2)), ("fp64", (16384, 512, 2)),
    ("fp32", (32768, 512, 2)), ("fp32", (1024, 8192, 2)),
    ("fp64", (2048, 8192, 2))])
def test_grid_image_beyond_4096_reuses_a_dirty_stack(precision, shape):
    """The one-call path beyond 4096 (rows wider than 4096 through the
    plain row transform and w-correction, columns longer than 4096 through
    the four-step transform) leaves the tiles without records unwritten
    from 1024 columns on: the column transform reads by tile record counts
    and the row transform (fused up to 4096 columns, else one-pass rows,
    or the two-half rows of FP64 at 16384 and FP32 at 32768) reads
    unmarked strips as zero; at 512 columns the idle tiles are zeroed.
    Three calls on one plan (the second with far fewer visibilities, so
    most of its idle tiles still hold the first call's sums), each image
    against the oracle."""
    nu, nv, nw = shape
    fp = 1 if precision == "fp64" else 0
    wl1 = synth.random_case(61, n=nu, nv=nv, nw=nw, support=7, m=20000,
                            law="core", precision=fp)
    wl2 = synth.random_case(62, n=nu, nv=nv, nw=nw, support=7, m=500,
                            law="gauss", precision=fp)
    wl2.w_min, wl2.w_max = wl1.w_min, wl1.w_max
    wl2.uvw[:, 2] = np.clip(wl2.uvw[:, 2], wl1.w_min, wl1.w_max)
    plan = plan_for(wl1, tile=64)
    for wl in (wl1, wl2, wl1):
        uvw, vis, wt = dev(wl)
        img = plan.grid_image(uvw, vis, wt)
        ref = o.image(o.Params.of(wl), wl.uvw, wl.vis, wl.weight)
        assert_close(host(img), ref, precision == "fp64",
                     "reuse beyond 4096")


def _with_hot_spot(wl, seed, count, cell_u, cell_v):
    """wl with its first `count` visibilities moved to within a few cells
    of (cell_u, cell_v): that tile gets more records than a chunk."""
    rng = np.random.default_rng(seed)
    uvw = wl.uvw.copy()
    uvw[:count, 0] = (cell_u + rng.normal(0, 2.0, count) - wl.nu / 2) / wl.fov_l
    uvw[:count, 1] = (cell_v + rng.normal(0, 2.0, count) - wl.nv / 2) / wl.fov_m
    return synth.Workload(wl.nu, wl.nv, wl.nw, wl.fov_l, wl.fov_m, wl.w_min,
                          wl.w_max, wl.support, wl.sigma, wl.precision,
                          np.ascontiguousarray(uvw), wl.vis, wl.weight,
                          name=wl.name + "+hot")


@pytest.mark.parametrize("chunk", [64, 0])
def test_busy_tile_store_matches_the_stack_path(chunk):
    """FP32 one-call path on 4096-row columns, tile edge 64: the tiles with
    records are gridded into a store of their own (split tiles merged into
    it) and the column transform reads them from there.  Its image matches
    that of the same data gridded into the stack and imaged by a separate
    call to 1e-6 (the same sums and transforms; only the partial tiles of
    split tiles, FP32 roundings of FP64 LDS sums whose order varies from
    run to run, can differ in the last bit), and the oracle's.  Three calls
    on one plan with different data: the second has far fewer busy tiles,
    so most slots and slot numbers of the first are stale."""
    wl1 = _with_hot_spot(
        synth.random_case(71, n=512, nv=4096, nw=2, support=7, m=20000,
                          law="core", precision=0), 72, 6000, 300.5, 1900.5)
    wl2 = synth.random_case(73, n=512, nv=4096, nw=2, support=7, m=2000,
                            law="gauss", precision=0)
    wl2.w_min, wl2.w_max = wl1.w_min, wl1.w_max
    wl2.uvw[:, 2] = np.clip(wl2.uvw[:, 2], wl1.w_min, wl1.w_max)
    plan = plan_for(wl1, tile=64, chunk=chunk)
    stack = plan_for(wl1, tile=64, chunk=chunk)
    for i, wl in enumerate((wl1, wl2, wl1)):
        uvw, vis, wt = dev(wl)
        img = plan.grid_image(uvw, vis, wt)
        st = plan.tile_stats()
        assert st["busy"] > 0 and st["idle"] > st["busy"]
        if i != 1 and chunk == 64:
            assert st["split"] > 0
        stack.reset()
        ref_img = stack.new_image()
        stack.grid(uvw, vis, wt)
        stack.image_accumulate(ref_img)
        got = host(img)
        err = rel_l2(got, host(ref_img))
        assert err <= 1e-6, f"call {i}: one-call vs stack path {err:.3e}"
        assert_close(got, o.image(o.Params.of(wl), wl.uvw, wl.vis, wl.weight),
                     False, f"busy-tile store, call {i}")


def test_busy_tile_store_overflow_goes_to_the_stack():
    """Visibilities spread over the whole 512 x 4096 grid: every tile has
    records, more than the busy-tile store holds (half the tiles), so the
    tiles past its last slot are gridded into the stack and read from
    there.  Image against the stack path and the oracle, twice in a row."""
    wl = synth.random_case(75, n=512, nv=4096, nw=2, support=7, m=20000,
                           law="gauss", precision=0)
    rng = np.random.default_rng(76)
    uvw = wl.uvw.copy()
    uvw[:, 0] = (rng.uniform(8, wl.nu - 8, wl.m) - wl.nu / 2) / wl.fov_l
    uvw[:, 1] = (rng.uniform(8, wl.nv - 8, wl.m) - wl.nv / 2) / wl.fov_m
    wl = synth.Workload(wl.nu, wl.nv, wl.nw, wl.fov_l, wl.fov_m, wl.w_min,
                        wl.w_max, wl.support, wl.sigma, wl.precision,
                        np.ascontiguousarray(uvw), wl.vis, wl.weight,
                        name="uniform")
    plan = plan_for(wl, tile=64)
    stack = plan_for(wl, tile=64)
    uvw_d, vis, wt = dev(wl)
    ref = o.image(o.Params.of(wl), wl.uvw, wl.vis, wl.weight)
    for i in range(2):
        img = plan.grid_image(uvw_d, vis, wt)
        st = plan.tile_stats()
        assert st["busy"] > (8 * 64 * 2) // 2, st
        stack.reset()
        ref_img = stack.new_image()
        stack.grid(uvw_d, vis, wt)
        stack.image_accumulate(ref_img)
        got = host(img)
        err = rel_l2(got, host(ref_img))
        assert err <= 1e-6, f"call {i}: one-call vs stack path {err:.3e}"
        assert_close(got, ref, False, f"store overflow, call {i}")


def test_busy_tile_store_empty_call_then_data():
    """An empty one-call on a plan with the busy-tile store adds nothing to
    the image (no tile has records, no strip is marked); the next call with
    data still matches the oracle."""
    wl = synth.random_case(77, n=512, nv=4096, nw=2, support=7, m=3000,
                           law="core", precision=0)
    plan = plan_for(wl, tile=64)
    uvw, vis, wt = dev(wl)
    img = plan.new_image()
    img.fill_(1.0)
    plan.grid_image(uvw[:0], vis[:0], None if wt is None else wt[:0],
                    image=img)
    assert plan.tile_stats()["busy"] == 0
    got = host(img)
    assert np.array_equal(got, np.ones_like(got))
    img = plan.grid_image(uvw, vis, wt)
    assert_close(host(img), o.image(o.Params.of(wl), wl.uvw, wl.vis, wl.weight),
                 False, "store after an empty call")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("chunk", [64, 333, 0])
def test_hot_bin_split_and_merge(precision, chunk):
    """Every visibility within a few cells of one point: tiles split into
    many work items whose partial tiles are merged."""
    rng = np.random.default_rng(12)
    n, m = 64, 6000
    fov = math.radians(2.0)
    xs = 32 + rng.normal(0, 1.5, m)
    ys = 32 + rng.normal(0, 1.5, m)
    uvw = np.stack([(xs - 32) / fov, (ys - 32) / fov,
                    rng.uniform(-10, 10, m)], 1)
    cdt = np.complex128 if precision == "fp64" else np.complex64
    vis = (rng.standard_normal(m) + 1j * rng.standard_normal(m)).astype(cdt)
    wl = synth.Workload(n, n, 2, fov, fov, -10.0, 10.0, 7, 0.0,
                        1 if precision == "fp64" else 0, uvw, vis, None)
    p = o.Params.of(wl)
    ref, _ = o.grid(p, uvw, vis, None)
    plan = plan_for(wl, chunk=chunk, tile=16)
    u, v, _ = dev(wl)
    plan.grid(u, v, None)
    assert_close(host(plan.planes), ref, precision == "fp64", "hot bin")
    img = plan.dirty_image(u, v, None)
    assert_close(host(img), o.image(p, uvw, vis, None),
                 precision == "fp64", "hot image")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_empty_and_invalid_inputs(precision):
    wl = _case(CASES[0], precision, seed=6)
    plan = plan_for(wl)
    d = torch.device("cuda")
    e = torch.empty((0, 3), dtype=torch.float64, device=d)
    ev = torch.empty(0, dtype=plan.cdtype, device=d)
    img = plan.dirty_image(e, ev)
    assert float(img.abs().max().item()) == 0.0
    out = plan.degrid(torch.ones((wl.nv, wl.nu), dtype=plan.rdtype, device=d),
                      e)
    assert out.numel() == 0
    # non-finite and far-off coordinates drop all their taps and touch nothing
    bad = np.array([[np.nan, 0, 0], [0, np.inf, 0], [0, 0, np.nan],
                    [1e30, 0, 0], [0.0, 0.0, 0.0]])
    vals = np.ones(5, dtype=np.complex128 if precision == "fp64"
                   else np.complex64)
    p = o.Params.of(wl)
    ref, ref_drop = o.grid(p, bad, vals, None)
    dropped = torch.zeros(1, dtype=torch.int64, device=d)
    plan.reset()
    plan.grid(torch.from_numpy(bad).to(d), torch.from_numpy(vals).to(d), None,
              dropped)
    assert int(dropped.item()) == ref_drop == 4 * 49
    assert_close(host(plan.planes), ref, precision == "fp64", "bad coords")
    # too many visibilities for the workspace is an error, not a fault
    with pytest.raises(ws.WStackError):
        big = torch.zeros((plan.max_vis + 1, 3), dtype=torch.float64, device=d)
        plan.grid(big, torch.zeros(plan.max_vis + 1, dtype=plan.cdtype,
                                   device=d))
    # gridding onto transformed planes is refused
    plan.reset()
    plan.grid(e, ev)
    plan.fft(+1)
    with pytest.raises(ws.WStackError):
        plan.grid(e, ev)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_config1_full_image(precision):
    wl = synth.config1(precision=1 if precision == "fp64" else 0)
    p = o.Params.of(wl)
    ref = o.image(p, wl.uvw, wl.vis, wl.weight)
    plan = plan_for(wl)
    uvw, vis, wt = dev(wl)
    img = host(plan.dirty_image(uvw, vis, wt))
    assert_close(img, ref, precision == "fp64", "config1")
    if precision == "fp32":
        print(f"config1 FP32 rel-L2 {rel_l2(img, ref):.3e}")


@pytest.mark.parametrize("tile", [16, 32, 64])
def test_tile_stats_cover_the_tiles_the_oracle_writes(tile):
    """Busy + idle tiles = every tile of the stack, and every tile that
    holds a nonzero cell of the oracle's gridded stack was counted busy."""
    wl = synth.random_case(23, n=256, nw=5, support=7, m=6000, law="core",
                           precision=1)
    plan = plan_for(wl, tile=tile)
    uvw, vis, wt = dev(wl)
    plan.reset()
    plan.grid(uvw, vis, wt)
    st = plan.tile_stats()
    assert st["tile"] == tile
    tu, tv = wl.nu // tile, wl.nv // tile
    assert st["busy"] + st["idle"] == wl.nw * tu * tv
    planes, _ = o.grid(o.Params.of(wl), wl.uvw, wl.vis, wl.weight)
    nz = np.abs(planes).reshape(wl.nw, tv, tile, tu, tile).max(axis=(2, 4))
    assert st["busy"] >= int((nz > 0).sum()) > 0
    assert 0 <= st["split"] <= st["busy"]
    # Exact counts: a visibility's record is read by its home tile (the
    # tile of its nearest cell) and by each neighbour whose edge strip of
    # width h it lies in (corner strips: three neighbours).
    h = (wl.support - 1) // 2
    _, _, i0, j0, k = o.coordinates(o.Params.of(wl), wl.uvw)
    reads, tiles = 0, set()
    for ii, jj, kk in zip(np.clip(i0, 0, wl.nu - 1), np.clip(j0, 0, wl.nv - 1),
                          k):
        tx, ty = ii // tile, jj // tile
        lx, ly = ii - tx * tile, jj - ty * tile
        dxs = [0] + ([-1] if lx < h and tx > 0 else []) + \
            ([1] if lx >= tile - h and tx + 1 < tu else [])
        dys = [0] + ([-1] if ly < h and ty > 0 else []) + \
            ([1] if ly >= tile - h and ty + 1 < tv else [])
        for a in dxs:
            for b in dys:
                tiles.add((int(kk), int(ty + b), int(tx + a)))
                reads += 1
    assert st["busy"] == len(tiles)
    assert st["record_reads"] == reads
    assert st["strips"] == len({(t[0], t[2]) for t in tiles})


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_grid_image_full_length_columns_edge_tile_rows(precision):
    """One-call path on 4096-row columns (64 tile rows of 64: every bit of
    the column transform's tile mask), with visibilities in the first and
    last tile rows and most tiles without records."""
    wl = synth.random_case(47, n=512, nv=4096, nw=2, support=7, m=3000,
                           law="gauss",
                           precision=1 if precision == "fp64" else 0)
    rng = np.random.default_rng(5)
    dv = 1.0 / wl.fov_m
    uvw = wl.uvw.copy()
    # Cells j = 4 .. 60 (tile row 0) and 4035 .. 4091 (tile row 63), the
    # kernel footprint still on the grid.
    lo = rng.integers(4, 61, 150) + rng.uniform(-0.4, 0.4, 150)
    hi = rng.integers(4035, 4092, 150) + rng.uniform(-0.4, 0.4, 150)
    uvw[:150, 1] = (lo - wl.nv / 2) * dv
    uvw[150:300, 1] = (hi - wl.nv / 2) * dv
    wl = synth.Workload(wl.nu, wl.nv, wl.nw, wl.fov_l, wl.fov_m, wl.w_min,
                        wl.w_max, wl.support, wl.sigma, wl.precision,
                        np.ascontiguousarray(uvw), wl.vis, wl.weight,
                        name="edge-rows")
    plan = plan_for(wl, tile=64)
    d_uvw, vis, wt = dev(wl)
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    plan.reset()
    img = plan.grid_image(d_uvw, vis, wt, dropped=dropped)
    st = plan.tile_stats()
    assert st["idle"] > st["busy"] > 0
    p = o.Params.of(wl)
    assert_close(host(img), o.image(p, wl.uvw, wl.vis, wl.weight),
                 precision == "fp64", "grid_image edge rows")
    assert int(dropped.item()) == o.grid(p, wl.uvw, wl.vis, wl.weight)[1]
