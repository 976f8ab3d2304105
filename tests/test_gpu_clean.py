"""Imaging major cycle on the GPU (ws_dirty_beam, ws_residual_image,
ws_clean_minor and the MajorCycle driver) against the oracle.

Sec. 1 places CLEAN deconvolution (Hogbom's loop inside the major / minor
cycles of Clark and Schwab) after imaging; the oracle's readings are in
oracle/wstack.py.  Tolerances: FP64 rel-max 1e-12 for the beam and single
residual images; composite results (after minor cycles) relative to the
first residual image's peak, 1e-11.  FP32: rel-L2 1e-5.

Argmax decisions: the FP64 path must take exactly the oracle's pixels.  The
FP32 path searches its own FP32 residual, so on a near-tie it may take
another pixel than the FP64 oracle; each of its picks is therefore checked
to be a valid argmax (within the FP32 tolerance) of the oracle's residual
replayed with the GPU's earlier picks, and the final images are compared
with the oracle run on the GPU's pick sequence.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import wstack as o  # noqa: E402
import paper_2301_06061_amd as ws  # noqa: E402
from paper_2301_06061_amd.clean import MajorCycle  # noqa: E402

pytestmark = pytest.mark.gpu


def _sky_case(precision, n=128, nw=4, m=3000, seed=0, kernel="es"):
    """Hermitian-paired visibilities of a few point sources (Eq. 1, with
    w-terms) at pixel centres."""
    fp64 = precision == "fp64"
    wl = synth.random_case(seed, n=n, nw=nw, support=7, m=m, law="gauss",
                           precision=1)
    wl = synth.hermitian_pairs(wl)
    wl.kernel = kernel
    wl.correct = kernel == "es"
    p = o.Params.of(wl)
    srcs = [(n // 2 + 11, n // 2 - 7, 1.0), (n // 2 - 20, n // 2 + 15, 0.77),
            (n // 2 + 3, n // 2 + 30, -0.53), (n // 2 - 33, n // 2 - 25, 0.31)]
    vis = np.zeros(wl.uvw.shape[0], np.complex128)
    for (pp, q, s) in srcs:
        l0 = (pp - n / 2) * p.fov_l / n
        m0 = (q - n / 2) * p.fov_m / n
        nm1 = float(o.n_minus_one(l0, m0))
        ph = wl.uvw[:, 0] * l0 + wl.uvw[:, 1] * m0 + wl.uvw[:, 2] * nm1
        vis += s * np.exp(-2j * math.pi * ph)
    wl.vis = vis.astype(np.complex128 if fp64 else np.complex64)
    wl.precision = 1 if fp64 else 0
    return wl, p


def _dev(wl):
    d = torch.device("cuda", 0)
    return (torch.from_numpy(np.ascontiguousarray(wl.uvw)).to(d),
            torch.from_numpy(np.ascontiguousarray(wl.vis)).to(d),
            torch.from_numpy(np.ascontiguousarray(wl.weight)).to(d))


def _h(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def _relmax(got, ref, scale=None):
    s = np.abs(ref).max() if scale is None else scale
    return float(np.abs(got - ref).max() / s)


def _rell2(got, ref, scale=None):
    s = np.linalg.norm(ref) if scale is None else scale
    return float(np.linalg.norm(got - ref) / s)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("kernel", ["es", "gauss"])
def test_dirty_beam_and_residual_image(precision, kernel):
    wl, p = _sky_case(precision, kernel=kernel)
    fp64 = precision == "fp64"
    b_ref, beta_ref = o.dirty_beam(p, wl.uvw, wl.weight)
    plan = ws.WStackPlan.from_workload(wl)
    uvw, vis, wt = _dev(wl)
    mc = MajorCycle(plan, uvw, vis, wt)
    beam = _h(mc.beam)
    beta = float(mc.beta.item())
    if fp64:
        assert abs(beta - beta_ref) <= 1e-12 * abs(beta_ref)
        assert _relmax(beam, b_ref) <= 1e-12
    else:
        assert abs(beta - beta_ref) <= 1e-5 * abs(beta_ref)
        assert _rell2(beam, b_ref) <= 1e-5
    # residual image of a sparse model
    rng = np.random.default_rng(3)
    model = np.zeros((wl.nv, wl.nu))
    idx = rng.choice(wl.nu * wl.nv, 25, replace=False)
    model.flat[idx] = rng.standard_normal(25)
    mc.model.copy_(torch.from_numpy(model).to(mc.model.dtype))
    res = _h(mc.residual_image())
    ref = o.residual_image(p, wl.uvw, wl.vis, wl.weight, model, beta_ref)
    if fp64:
        assert _relmax(res, ref) <= 1e-12
    else:
        assert _rell2(res, ref) <= 1e-5


def _check_picks_valid(d0, beam, gpu_picks, gain, tol):
    """Each GPU pick is an argmax of the oracle's residual replayed with the
    GPU's earlier picks, within tol x the first peak."""
    peak0 = np.abs(d0).max()
    for t in range(len(gpu_picks)):
        _, dt, _ = o.hogbom(d0, beam, t, gain, picks=gpu_picks[:t])
        q, pp = gpu_picks[t]
        assert abs(dt[q, pp]) >= np.abs(dt).max() - tol * peak0, t


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_clean_minor_matches_oracle(precision):
    """The minor cycle alone on the oracle's residual image and beam."""
    wl, p = _sky_case(precision, seed=1)
    fp64 = precision == "fp64"
    b, beta = o.dirty_beam(p, wl.uvw, wl.weight)
    d0 = o.residual_image(p, wl.uvw, wl.vis, wl.weight,
                          np.zeros((wl.nv, wl.nu)), beta)
    plan = ws.WStackPlan.from_workload(wl)
    dt = plan.rdtype
    dev = torch.device("cuda", 0)
    res = torch.from_numpy(d0).to(dev).to(dt)
    beam = torch.from_numpy(b).to(dev).to(dt)
    model = torch.zeros_like(res)
    niter, gain = 60, 0.2
    picks = torch.full((niter,), -1, dtype=torch.int32, device=dev)
    n_done = torch.zeros(1, dtype=torch.int32, device=dev)
    from paper_2301_06061_amd import _abi
    from paper_2301_06061_amd.api import _ptr
    plan._bind()
    _abi.call("ws_clean_minor", plan._h, _ptr(res), _ptr(beam), _ptr(model),
              niter, gain, 0.0, _ptr(picks), _ptr(n_done))
    torch.cuda.synchronize()
    assert int(n_done.item()) == niter
    gp = [divmod(int(i), wl.nu) for i in picks.cpu().numpy()]
    m_ref, r_ref, comps = o.hogbom(d0, b, niter, gain)
    peak = np.abs(d0).max()
    if fp64:
        assert gp == [c[:2] for c in comps]
        assert _relmax(_h(model), m_ref, peak) <= 1e-12
        assert _relmax(_h(res), r_ref, peak) <= 1e-12
    else:
        _check_picks_valid(d0, b, gp, gain, 1e-5)
        m2, r2, _ = o.hogbom(d0, b, niter, gain, picks=gp)
        assert _rell2(_h(model), m2) <= 1e-5
        assert _rell2(_h(res), r2, np.linalg.norm(d0)) <= 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_clean_minor_unaligned_residual_matches_aligned(precision):
    """A residual that is not 16-byte aligned takes the one-pixel-per-load
    form of the minor step: the same picks and the same arithmetic per
    pixel as the aligned, vector-load form, so equal results."""
    wl, p = _sky_case(precision, seed=3, n=128, m=2000)
    b, beta = o.dirty_beam(p, wl.uvw, wl.weight)
    d0 = o.residual_image(p, wl.uvw, wl.vis, wl.weight,
                          np.zeros((wl.nv, wl.nu)), beta)
    plan = ws.WStackPlan.from_workload(wl)
    dt = plan.rdtype
    dev = torch.device("cuda", 0)
    from paper_2301_06061_amd import _abi
    from paper_2301_06061_amd.api import _ptr
    out = []
    for offset in (0, 1):
        store = torch.zeros(d0.size + 4, dtype=dt, device=dev)
        res = store[offset:offset + d0.size].view(wl.nv, wl.nu)
        res.copy_(torch.from_numpy(d0).to(dev).to(dt))
        assert (res.data_ptr() % 16 == 0) == (offset == 0)
        beam = torch.from_numpy(b).to(dev).to(dt)
        model = torch.zeros_like(beam)
        picks = torch.full((40,), -1, dtype=torch.int32, device=dev)
        n_done = torch.zeros(1, dtype=torch.int32, device=dev)
        plan._bind()
        _abi.call("ws_clean_minor", plan._h, _ptr(res), _ptr(beam),
                  _ptr(model), 40, 0.25, 0.0, _ptr(picks), _ptr(n_done))
        torch.cuda.synchronize()
        out.append((picks.cpu().numpy(), res.cpu().numpy(),
                    model.cpu().numpy(), int(n_done.item())))
    (p0, r0, m0, n0), (p1, r1, m1, n1) = out
    assert n0 == n1 == 40
    assert np.array_equal(p0, p1)
    assert np.array_equal(r0, r1) and np.array_equal(m0, m1)


def test_clean_minor_threshold_and_zero_iterations():
    wl, p = _sky_case("fp64", seed=2, n=64, m=1500)
    b, beta = o.dirty_beam(p, wl.uvw, wl.weight)
    d0 = o.residual_image(p, wl.uvw, wl.vis, wl.weight,
                          np.zeros((wl.nv, wl.nu)), beta)
    plan = ws.WStackPlan.from_workload(wl)
    dev = torch.device("cuda", 0)
    from paper_2301_06061_amd import _abi
    from paper_2301_06061_amd.api import _ptr
    thr = 0.5 * np.abs(d0).max()
    for niter, threshold in ((0, 0.0), (200, thr)):
        res = torch.from_numpy(d0).to(dev)
        beam = torch.from_numpy(b).to(dev)
        model = torch.zeros_like(res)
        picks = torch.full((max(niter, 1),), -1, dtype=torch.int32,
                           device=dev)
        n_done = torch.full((1,), -7, dtype=torch.int32, device=dev)
        plan._bind()
        _abi.call("ws_clean_minor", plan._h, _ptr(res), _ptr(beam),
                  _ptr(model), niter, 0.3, threshold, _ptr(picks),
                  _ptr(n_done))
        m_ref, r_ref, comps = o.hogbom(d0, b, niter, 0.3, threshold)
        n = int(n_done.item())
        assert n == len(comps)
        got = [divmod(int(i), wl.nu) for i in picks.cpu().numpy()[:n]]
        assert got == [c[:2] for c in comps]
        assert np.all(picks.cpu().numpy()[n:] == -1)
        assert _relmax(_h(res), r_ref, np.abs(d0).max()) <= 1e-12
        assert _relmax(_h(model), m_ref, np.abs(d0).max()) <= 1e-12
    # refused arguments
    with pytest.raises(ws.WStackError):
        _abi.call("ws_clean_minor", plan._h, _ptr(res), _ptr(beam),
                  _ptr(model), 5, 1.5, 0.0, None, None)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_major_cycle_matches_oracle(precision):
    wl, p = _sky_case(precision, seed=4)
    fp64 = precision == "fp64"
    n_major, n_minor, gain = 3, 25, 0.2
    plan = ws.WStackPlan.from_workload(wl)
    uvw, vis, wt = _dev(wl)
    mc = MajorCycle(plan, uvw, vis, wt)
    model = _h(mc.run(n_major, n_minor, gain))
    res = _h(mc.residual)
    gpicks = [[divmod(int(i), wl.nu) for i in pk.cpu().numpy()]
              for pk in mc.picks]
    vis64 = wl.vis.astype(np.complex128)
    if fp64:
        m_ref, r_ref, hist, b, beta = o.major_cycle(p, wl.uvw, vis64,
                                                    wl.weight, n_major,
                                                    n_minor, gain)
        assert gpicks == [[c[:2] for c in cyc] for cyc in hist]
    else:
        m_ref, r_ref, hist, b, beta = o.major_cycle(p, wl.uvw, vis64,
                                                    wl.weight, n_major,
                                                    n_minor, gain,
                                                    picks=gpicks)
        # each cycle's picks valid for the oracle's residual of that cycle
        model_j = np.zeros((wl.nv, wl.nu))
        for j in range(n_major):
            d0 = o.residual_image(p, wl.uvw, vis64, wl.weight, model_j, beta)
            _check_picks_valid(d0, b, gpicks[j], gain, 1e-5)
            dm, _, _ = o.hogbom(d0, b, n_minor, gain, picks=gpicks[j])
            model_j = model_j + dm
    d_first = o.residual_image(p, wl.uvw, vis64, wl.weight,
                               np.zeros((wl.nv, wl.nu)), beta)
    peak = np.abs(d_first).max()
    if fp64:
        assert _relmax(model, m_ref, peak) <= 1e-11
        assert _relmax(res, r_ref, peak) <= 1e-11
    else:
        assert _rell2(model, m_ref) <= 1e-5
        assert _rell2(res, r_ref, np.linalg.norm(d_first)) <= 1e-5
    # the sources are found: the brightest model pixels are theirs
    assert np.abs(res).max() < 0.5 * peak
