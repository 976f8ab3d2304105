"""Parity at the benchmark's full sizes, on sampled outputs the oracle can
compute one by one: grid cells summed visibility by visibility, and dirty-
image pixels from the definition (no FFT), in the launch configuration the
benchmark times (ws_grid_visibilities + ws_image_accumulate)."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import wstack as o  # noqa: E402
import paper_2301_06061_amd as ws  # noqa: E402

pytestmark = pytest.mark.gpu


def _sample_cells(wl, p, n_rand=12, seed=0):
    """Cells to check: the busiest cells of the busiest planes (dense core)
    plus random cells inside the visibility disk."""
    x, y, i0, j0, k = o.coordinates(p, wl.uvw[:2_000_000])
    rng = np.random.default_rng(seed)
    kk = np.bincount(k, minlength=p.nw).argsort()[-3:]
    cells = []
    for kq in kk:
        sel = k == kq
        flat = j0[sel] * p.nu + i0[sel]
        top = np.bincount(flat).argmax()
        cells.append((int(kq), int(top // p.nu), int(top % p.nu)))
        cells.append((int(kq), int(top // p.nu) + 2, int(top % p.nu) - 3))
    idx = rng.integers(0, len(i0), n_rand)
    for t in idx:
        cells.append((int(k[t]), int(j0[t]) + int(rng.integers(-3, 4)),
                      int(i0[t]) + int(rng.integers(-3, 4))))
    return cells


def _run(wl, pixels, cells, precision):
    dev = torch.device("cuda", 0)
    plan = ws.WStackPlan.from_workload(wl, precision=precision)
    uvw = torch.from_numpy(wl.uvw).to(dev)
    vis = torch.from_numpy(wl.vis).to(dev)
    if precision == "fp64":
        vis = vis.to(torch.complex128)
    wt = torch.from_numpy(wl.weight).to(dev)
    dropped = torch.zeros(1, dtype=torch.int64, device=dev)
    plan.reset()
    plan.grid(uvw, vis, wt, dropped)
    torch.cuda.synchronize()
    got_cells = np.array([plan.planes[c].item() for c in cells])
    img = plan.new_image()
    plan.image_accumulate(img)
    torch.cuda.synchronize()
    got_pix = np.array([img[q, pp].item() for q, pp in pixels])
    rms = float(img.abs().pow(2).mean().sqrt())
    nd = int(dropped.item())
    del plan
    torch.cuda.empty_cache()
    return got_cells, got_pix, rms, nd


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_config2_full_size_sampled(precision):
    wl = synth.config2(precision=0)
    p = o.Params.of(wl)
    cells = _sample_cells(wl, p)
    pixels = [(2048, 2048), (1000, 3000), (4000, 17)]
    got_cells, got_pix, rms, nd = _run(wl, pixels, cells, precision)
    assert nd == 0
    ref_cells = o.grid_cells_direct(p, wl.uvw, wl.vis, wl.weight, cells)
    ref_pix = o.image_pixels_direct(p, wl.uvw, wl.vis, wl.weight, pixels)
    if precision == "fp64":
        scale = np.abs(ref_cells).max()
        assert np.abs(got_cells - ref_cells).max() <= 1e-12 * scale
        assert np.abs(got_pix - ref_pix).max() <= 1e-11 * rms
    else:
        assert np.all(np.abs(got_cells - ref_cells) <=
                      2e-6 * np.abs(ref_cells) + 1e-6 * np.abs(ref_cells).max())
        assert np.abs(got_pix - ref_pix).max() <= 1e-5 * rms


@pytest.fixture(scope="module")
def config3_data():
    wl = synth.config3(precision=0)
    p = o.Params.of(wl)
    cells = _sample_cells(wl, p, n_rand=1)[:3]
    pixels = [(8192, 8192)]
    ref_cells = o.grid_cells_direct(p, wl.uvw, wl.vis, wl.weight, cells)
    ref_pix = o.image_pixels_direct(p, wl.uvw, wl.vis, wl.weight, pixels)
    return wl, cells, pixels, ref_cells, ref_pix


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_config3_full_size_sampled(config3_data, precision):
    """16384^2 x 32 planes, K = 9, 1e8 visibilities: four-step columns,
    and on the FP64 path rows split in two LDS halves."""
    wl, cells, pixels, ref_cells, ref_pix = config3_data
    got_cells, got_pix, rms, nd = _run(wl, pixels, cells, precision)
    assert nd == 0
    if precision == "fp64":
        scale = np.abs(ref_cells).max()
        assert np.abs(got_cells - ref_cells).max() <= 1e-12 * scale
        assert np.abs(got_pix - ref_pix).max() <= 1e-11 * rms
    else:
        assert np.all(np.abs(got_cells - ref_cells) <=
                      2e-6 * np.abs(ref_cells) +
                      1e-6 * np.abs(ref_cells).max())
        assert np.abs(got_pix - ref_pix).max() <= 1e-5 * rms


def _golden_pixels():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "config2_pixels.txt")
    px, val = [], []
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            q, p, re, im = line.split()
            px.append((int(q), int(p)))
            val.append(complex(float(re), float(im)))
    return px, np.array(val)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_config2_timed_path_pixels(precision):
    """The call the benchmark times (ws_grid_image on the dense-core 1e7
    visibility workload, default plan) against 64 pixels of the oracle's
    per-pixel definition (written by tests/golden/make_config2_pixels.py):
    corners, edges, the centre and random pixels.  FP32: the sampled
    pixels' rel-L2 <= 1e-5 and every pixel within 1e-5 of the image rms;
    FP64: within 1e-11 of the rms."""
    px, ref = _golden_pixels()
    assert len(px) == 64
    wl = synth.config2(precision=0)
    dev = torch.device("cuda", 0)
    plan = ws.WStackPlan.from_workload(wl, precision=precision)
    uvw = torch.from_numpy(wl.uvw).to(dev)
    vis = torch.from_numpy(wl.vis).to(dev)
    if precision == "fp64":
        vis = vis.to(torch.complex128)
    wt = torch.from_numpy(wl.weight).to(dev)
    img = plan.new_image()
    plan.reset()
    plan.grid_image(uvw, vis, wt, image=img)
    torch.cuda.synchronize()
    qi = torch.tensor([q for q, _ in px], device=dev)
    pi = torch.tensor([p for _, p in px], device=dev)
    got = img[qi, pi].cpu().numpy().astype(np.complex128)
    rms = float(img.abs().pow(2).mean().sqrt())
    err = np.abs(got - ref)
    if precision == "fp64":
        assert err.max() <= 1e-11 * rms, err.max() / rms
    else:
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-5
        assert err.max() <= 1e-5 * rms, err.max() / rms
    del plan
    torch.cuda.empty_cache()
