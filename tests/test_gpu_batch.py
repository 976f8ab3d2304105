"""Batched channels: one persistent gridding launch over many plans, eager
and replayed from a HIP graph, against the oracle and the single-plan path."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import wstack as o  # noqa: E402
import paper_2301_06061_amd as ws  # noqa: E402
from paper_2301_06061_amd.batch import BatchedImager  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _channels(precision, seed=0):
    shapes = [(64, 2, 500), (128, 4, 3000), (256, 3, 8000), (64, 1, 0),
              (128, 2, 1)]
    wls = []
    for i, (n, nw, m) in enumerate(shapes):
        wl = synth.random_case(seed + i, n=n, nw=nw, support=7,
                               m=max(m, 1), law="core",
                               precision=1 if precision == "fp64" else 0)
        if m == 0:
            wl.uvw = wl.uvw[:0]
            wl.vis = wl.vis[:0]
            wl.weight = wl.weight[:0]
        if nw == 1:
            wl.w_max = wl.w_min
        elif m <= 1:
            # one visibility: the data give no w range of their own
            wl.w_max = wl.w_min + 1.0
        wls.append(wl)
    return wls


def _dev(wls):
    uvw = [torch.from_numpy(w.uvw.copy()).to(DEV) for w in wls]
    vis = [torch.from_numpy(w.vis.copy()).to(DEV) for w in wls]
    wt = [torch.from_numpy(w.weight.copy()).to(DEV) for w in wls]
    return uvw, vis, wt


def _err(got, ref, fp64):
    got = np.asarray(got, np.complex128)
    ref = np.asarray(ref, np.complex128)
    if fp64:
        return np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)
    return np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp64", 1e-12)])
def test_batch_matches_oracle(precision, tol):
    wls = _channels(precision)
    uvw, vis, wt = _dev(wls)
    b = BatchedImager(wls, uvw, vis, wt, precision=precision)
    imgs = [t.cpu().numpy() for t in b.run()]
    for i, wl in enumerate(wls):
        p = o.Params.of(wl)
        ref = o.image(p, wl.uvw, wl.vis, wl.weight)
        if not np.any(ref):
            assert not np.any(imgs[i])
            continue
        assert _err(imgs[i], ref, precision == "fp64") <= tol, i
    b.close()


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp64", 1e-12)])
def test_batch_graph_replays_match_oracle(precision, tol):
    """Every replay of the captured graph against the oracle's images of
    the visibilities it was given (new values between replays, with eager
    work in between)."""
    wls = _channels(precision, seed=10)
    uvw, vis, wt = _dev(wls)
    b = BatchedImager(wls, uvw, vis, wt, precision=precision)
    refs = [o.image(o.Params.of(w), w.uvw, w.vis, w.weight) for w in wls]
    b.run()
    b.capture()
    for rep in range(3):
        # eager work between replays: change the visibilities in place
        scale = float(rep + 1)
        for i in range(len(wls)):
            vis[i].copy_(torch.from_numpy(wls[i].vis).to(DEV) * scale)
        torch.cuda.synchronize()
        got = [t.cpu().numpy() for t in b.replay()]
        for i in range(len(wls)):
            if not np.any(refs[i]):
                assert not np.any(got[i]), (rep, i)
                continue
            assert _err(got[i], refs[i] * scale, precision == "fp64") <= tol, \
                (rep, i)
    b.close()


def test_batch_mixes_lazy_and_zeroed_plans():
    """Plans whose imaging reads by tile counts (tile edge 64, 512 columns
    or more: tiles without records stay unwritten) next to plans whose
    idle tiles must be zeroed (tile edge 32, or narrower grids), in one
    batch: every image against the oracle, on two runs in a row (the
    second run meets the first run's stack contents) and a graph replay."""
    shapes = [(512, 2, 2000, 64), (512, 2, 2000, 32), (256, 2, 1000, 0),
              (1024, 3, 3000, 64)]
    wls = [synth.random_case(40 + i, n=n, nw=nw, support=7, m=m, law="core",
                             precision=0)
           for i, (n, nw, m, _) in enumerate(shapes)]
    uvw, vis, wt = _dev(wls)
    b = BatchedImager(wls, uvw, vis, wt, precision="fp32",
                      params=[(t, 0) for (_, _, _, t) in shapes])
    refs = [o.image(o.Params.of(w), w.uvw, w.vis, w.weight) for w in wls]
    for run in range(2):
        got = [t.cpu().numpy() for t in b.run()]
        for i in range(len(wls)):
            assert _err(got[i], refs[i], False) <= 1e-5, (run, i)
    b.capture()
    got = [t.cpu().numpy() for t in b.replay()]
    for i in range(len(wls)):
        assert _err(got[i], refs[i], False) <= 1e-5, ("replay", i)
    b.close()


def test_autotuner_cache_round_trip_and_tuned_batch(tmp_path, monkeypatch):
    """tune() times the one-call step of every valid (tile, chunk) candidate
    on the caller's data, stores the winner per shape class, answers the second time from
    the cache without timing anything, and the batch built from the tuned
    parameters matches the oracle."""
    from paper_2301_06061_amd import autotune
    monkeypatch.setenv("WSTACK_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    wls = _channels("fp32", seed=40)[:3]
    for wl in wls:  # the kernel type is part of the shape class
        wl.kernel = "es"
    uvw, vis, wt = _dev(wls)
    picks = []
    for i, wl in enumerate(wls):
        t, c = autotune.tune(wl, uvw[i], vis[i], wt[i], "fp32", reps=2)
        assert t in autotune.TILES and c in autotune.CHUNKS, (t, c)
        assert t <= min(wl.nu, wl.nv)
        picks.append((t, c))
    import json
    db = json.load(open(tmp_path / "tune.json"))
    assert len(db) == 3
    for i, wl in enumerate(wls):
        key = autotune.shape_key(wl.nu, wl.nv, wl.nw, wl.support, "fp32",
                                 int(uvw[i].shape[0]), wl.kernel)
        e = db[key]
        assert (e["tile"], e["chunk"]) == picks[i]
        valid = [t for t in autotune.TILES if t <= min(wl.nu, wl.nv)]
        assert len(e["trials"]) == len(valid) * len(autotune.CHUNKS)
        assert e["ms"] == min(e["trials"].values())
    # second round: answered from the cache, nothing timed
    monkeypatch.setattr(autotune, "time_step",
                        lambda *a, **k: pytest.fail("timed despite cache"))
    for i, wl in enumerate(wls):
        assert autotune.tune(wl, uvw[i], vis[i], wt[i], "fp32") == picks[i]
    b = BatchedImager(wls, uvw, vis, wt, precision="fp32", tune=True)
    assert b.tuned == picks
    imgs = [t.cpu().numpy() for t in b.run()]
    for i, wl in enumerate(wls):
        ref = o.image(o.Params.of(wl), wl.uvw, wl.vis, wl.weight)
        assert _err(imgs[i], ref, False) <= 1e-5, i
    b.close()


def test_batch_rejects_mixed_precision():
    a = synth.random_case(1, n=64, nw=2, m=100, precision=0)
    c = synth.random_case(2, n=64, nw=2, m=100, precision=1)
    p1 = ws.WStackPlan.from_workload(a)
    p2 = ws.WStackPlan.from_workload(c)
    import ctypes as C
    from paper_2301_06061_amd import _abi
    wb = C.c_size_t(0)
    _abi.call("ws_batch_workspace_bytes", 2, C.byref(wb))
    work = torch.empty(wb.value, dtype=torch.uint8, device=DEV)
    h = C.c_void_p()
    st = _abi.lib().ws_batch_create(2, (C.c_void_p * 2)(p1._h, p2._h),
                                    C.c_void_p(work.data_ptr()), wb.value,
                                    C.byref(h))
    assert st == _abi.WS_INVALID_ARG and h.value is None


def test_config4_scaled_channels():
    """Config-4 recipe, 64 channels with counts scaled down 100x: every
    channel in one batch against its own single-plan image, three small
    channels against the oracle."""
    wls = synth.config4(m_scale=0.01)
    uvw, vis, wt = _dev(wls)
    b = BatchedImager(wls, uvw, vis, wt, precision="fp32")
    imgs = b.run()
    torch.cuda.synchronize()
    checked = 0
    for i, wl in enumerate(wls):
        plan = ws.WStackPlan.from_workload(wl)
        single = plan.dirty_image(uvw[i], vis[i], wt[i])
        err = float(torch.linalg.vector_norm(imgs[i] - single) /
                    torch.linalg.vector_norm(single))
        assert err <= 1e-6, (i, err)
        plan.close()
        if wl.nu == 1024 and checked < 3:
            ref = o.image(o.Params.of(wl), wl.uvw, wl.vis, wl.weight)
            assert _err(imgs[i].cpu().numpy(), ref, False) <= 1e-5, i
            checked += 1
    b.close()


def test_batch_graph_replays_lazy_channels():
    """Graph replays of a batch whose plans all leave tiles without records
    unwritten (tile edge 64, rows of 512 or more; the plan with 4096-row
    columns grids its tiles with records into the busy-tile store): each
    replay starts from the stacks the previous one left, with new
    visibility values."""
    wls = []
    for i, (n, nv, nw, m) in enumerate([(512, 512, 2, 4000),
                                        (1024, 512, 3, 6000),
                                        (512, 1024, 1, 2000),
                                        (512, 4096, 2, 3000)]):
        wl = synth.random_case(30 + i, n=n, nv=nv, nw=nw, support=7, m=m,
                               law="core", precision=0)
        if nw == 1:
            wl.w_max = wl.w_min
        wls.append(wl)
    uvw, vis, wt = _dev(wls)
    b = BatchedImager(wls, uvw, vis, wt, precision="fp32")
    eager = [t.clone() for t in b.run()]
    for i, wl in enumerate(wls):
        ref = o.image(o.Params.of(wl), wl.uvw, wl.vis, wl.weight)
        assert _err(eager[i].cpu().numpy(), ref, False) <= 1e-5, i
    refs = [o.image(o.Params.of(w), w.uvw, w.vis, w.weight) for w in wls]
    b.capture()
    for rep in range(3):
        scale = float(rep + 2)
        for i in range(len(wls)):
            vis[i].copy_(torch.from_numpy(wls[i].vis).to(DEV) * scale)
        torch.cuda.synchronize()
        got = b.replay()
        torch.cuda.synchronize()
        for i in range(len(wls)):
            assert _err(got[i].cpu().numpy(), refs[i] * scale, False) <= 1e-5, \
                (rep, i)
    b.close()
