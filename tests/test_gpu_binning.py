"""Both binning modes (two-level partition and hashed counting sort)
against the oracle: planes, dropped taps, degridded values and the per-key
record offsets (exact), on ordinary, hot, empty, single and invalid
inputs.  The gridder reads the records by key ranges, so equal offsets
mean equal work items; the record order within a key may differ between
modes (ranks come from LDS atomics), which only reorders FP additions."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import wstack as o  # noqa: E402
import paper_2301_06061_amd as ws  # noqa: E402

pytestmark = pytest.mark.gpu

MODES = ["partition", "hashed"]


def _err(got, ref, fp64):
    got = np.asarray(got, np.complex128)
    ref = np.asarray(ref, np.complex128)
    if not np.any(ref):
        return float(np.abs(got).max())
    if fp64:
        return float(np.abs(got - ref).max() / np.abs(ref).max())
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def _dev(wl):
    d = torch.device("cuda", 0)
    wt = None if wl.weight is None else torch.from_numpy(wl.weight).to(d)
    return (torch.from_numpy(np.ascontiguousarray(wl.uvw)).to(d),
            torch.from_numpy(np.ascontiguousarray(wl.vis)).to(d), wt)


def _cases(precision):
    prec = 1 if precision == "fp64" else 0
    out = [synth.random_case(1, n=256, nw=5, support=7, m=30000, law="core",
                             precision=prec),
           synth.random_case(2, n=128, nv=64, nw=3, support=9, m=5000,
                             law="gauss", precision=prec),
           synth.edge_case(3, n=128, nw=4, support=7, m=3000, precision=prec)]
    # hot: every visibility within one cell of the centre, one plane
    hot = synth.random_case(4, n=64, nw=2, support=7, m=20000, law="core",
                            precision=prec)
    hot.uvw[:, :2] *= 1e-3
    out.append(hot)
    one = synth.random_case(5, n=64, nw=2, support=5, m=1, precision=prec)
    one.w_max = one.w_min + 1.0
    out.append(one)
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("mode", MODES)
def test_binning_modes_match_oracle(precision, mode):
    fp64 = precision == "fp64"
    for wl in _cases(precision):
        p = o.Params.of(wl)
        ref, drop_ref = o.grid(p, wl.uvw, wl.vis, wl.weight)
        uvw, vis, wt = _dev(wl)
        plan = ws.WStackPlan.from_workload(wl, binning=mode)
        dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
        plan.grid(uvw, vis, wt, dropped)
        torch.cuda.synchronize()
        assert _err(plan.planes.cpu().numpy(), ref, fp64) <= \
            (1e-12 if fp64 else 1e-5), wl.name
        assert int(dropped.item()) == drop_ref, wl.name
        img = plan.dirty_image(uvw, vis, wt)
        assert _err(img.cpu().numpy(), o.image(p, wl.uvw, wl.vis, wl.weight),
                    fp64) <= (1e-12 if fp64 else 1e-5), wl.name
        x = np.random.default_rng(0).standard_normal((wl.nv, wl.nu))
        v = plan.degrid(torch.from_numpy(x).to("cuda").to(plan.rdtype), uvw,
                        wt)
        torch.cuda.synchronize()
        assert _err(v.cpu().numpy(), o.degrid(p, x, wl.uvw, wl.weight),
                    fp64) <= (1e-12 if fp64 else 1e-5), wl.name
        plan.close()


def test_binning_modes_give_equal_work():
    """The two modes give the same per-key record counts, seen through the
    tile statistics they determine (tiles with and without records, split
    tiles, extra work items, marked column strips, total record reads),
    and the tiles with records are the oracle's: those some on-grid tap
    reaches."""
    wl = synth.random_case(6, n=256, nw=4, support=7, m=40000, law="core",
                           precision=0)
    uvw, vis, wt = _dev(wl)
    stats = {}
    for mode in MODES:
        plan = ws.WStackPlan.from_workload(wl, binning=mode)
        plan.grid(uvw, vis, wt)
        torch.cuda.synchronize()
        stats[mode] = plan.tile_stats()
        plan.close()
    assert stats["partition"] == stats["hashed"]
    p = o.Params.of(wl)
    x, y, i0, j0, k = o.coordinates(p, wl.uvw)
    T = stats["hashed"]["tile"]
    h = (p.support - 1) // 2
    tiles = set()
    for dj in range(-h, h + 1):
        for di in range(-h, h + 1):
            ii, jj = i0 + di, j0 + dj
            on = (ii >= 0) & (ii < p.nu) & (jj >= 0) & (jj < p.nv)
            t = (k[on] * (p.nv // T) + jj[on] // T) * (p.nu // T) + ii[on] // T
            tiles.update(np.unique(t).tolist())
    assert stats["hashed"]["busy"] == len(tiles)


def test_binning_partition_refused_where_it_does_not_fit():
    # 16384^2 with 16-cell tiles: 1024 tile rows per plane; even two rows a
    # bucket give 18432 keys per bucket, over the 16384 limit.
    p = ws.make_params(16384, 16384, 32, 0.1, 0.1, -1.0, 1.0, 7, 0.0, "fp32",
                       tile=16, binning="partition")
    with pytest.raises(ws.WStackError) as e:
        ws.workspace_bytes(p, 1000)
    assert e.value.status == -2
    p.binning = 0  # automatic: falls back to the hashed sort
    ws.workspace_bytes(p, 1000)
