"""Benchmark of the w-stacking imaging path on one MI355X.

One step = the whole hot path on one batch of synthetic visibilities held in
HBM, in one call (ws_grid_image): binning + gridding onto N_w w-planes, then
the per-plane 2-D FFT, w-screen and plane sum into the dirty image.  Default
workload: 1e7 visibilities with a dense core (r = R U^2, w = wmax r/R +
N(0, 0.1 wmax)), 4096^2 grid, 32 w-planes, 7x7 Gaussian kernel, 5 deg field,
FP32 path; the FP64 path is timed on the same inputs for comparison.

Further legs (on by default, each skippable): the large single image
(1e8 visibilities, 16384^2 x 32, K = 9, FP32 and FP64), 64 batched channels
(autotuned, replayed from a HIP graph), the differentiable operator
(degrid forward + grid backward, 1e7 visibilities, 4096^2 x 32), the
headline grid fed baseline-major rows (8 channels x 4 correlations ->
Stokes I), an imaging major cycle on the config-5 sky, and the headline
step with its host-to-device input copies (pinned memory) and the image
copy back inside the timing.

Prints one JSON line (the last line on stdout).  value = visibilities imaged
per second (Mvis/s) over the timed steps of the headline workload.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def record_bytes(elem):
    """Bytes of one binned record (FP32 path: elem 8; FP64: 16)."""
    return 24 if elem == 8 else 40


def algorithmic_bytes(name, wl, elem, m, st=None):
    """Bytes a kernel must move per launch (reads + writes).

    Without tile statistics ``st``, the definition of the step on a full
    stack: the 2-D transform reads and writes the stack once, the screen
    pass reads it once and the image twice, gridding writes every cell once
    and reads every record once.  With ``st`` (ws_tile_stats of the timed
    one-call path), the bytes that path has to move given the work the
    binning found: only tiles that received records are written by the
    gridder and read by the column transform, only marked column strips
    (tile-wide columns of one plane) are written by the column transform
    and read by the row pass, and every record is read once per tile its
    footprint reaches.
      fft_cols:       busy tiles read + marked strips written;
      row_screen_sum: marked strips read + image read and written;
      grid (step):    busy tiles written + records read + split-tile
                      partials written and read back by the merge;
      bin_count:      uvw read (24 B) + key/rank written (8 B) per vis;
      bin_scatter:    uvw, vis, weight, key/rank and the key offset read,
                      one record written per visibility;
      part_count1:    uvw read + key/rank written per vis (as bin_count);
      part_scatter1:  key/rank, uvw, vis, weight read, one record and its
                      4-byte key written per visibility;
      part_count2:    key read + rank written (4 + 4 B) per vis;
      part_scatter2:  record, key and rank read, record written per vis.
    """
    cells = wl.nu * wl.nv * wl.nw
    img = wl.nu * wl.nv
    rec = record_bytes(elem)
    if st is None:
        full = {
            "fft_cols": 2 * cells * elem,
            "row_screen_sum": cells * elem + 2 * img * elem,
            "grid": cells * elem + m * rec,
        }
    else:
        tile_b = st["tile"] ** 2 * elem
        strip_b = wl.nv * st["tile"] * elem
        parts = st["split"] + st["extra_items"]
        full = {
            "fft_cols": st["busy"] * tile_b + st["strips"] * strip_b,
            "row_screen_sum": st["strips"] * strip_b + 2 * img * elem,
            "grid": (st["busy"] * tile_b + st["record_reads"] * rec +
                     2 * parts * tile_b),
        }
    full["bin_count"] = m * (24 + 8)
    full["bin_scatter"] = m * (24 + elem + 4 + 8 + 4 + rec)
    full["part_count1"] = m * (24 + 8)
    full["part_scatter1"] = m * (8 + 24 + elem + 4 + rec + 4)
    full["part_count2"] = m * (4 + 4)
    full["part_scatter2"] = m * (rec + 4 + 4 + rec)
    return full.get(name)


# Headers every kernel source includes: a change there changes the kernels.
_KERNEL_HEADERS = ("ws_common.h", "ws_kernels.h")


def source_digest(path):
    """Digest of a kernel's source file together with the shared kernel
    headers (record layout, geometry, launch declarations)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2301_06061_amd", "csrc")
    for p in (path,) + tuple(os.path.join(csrc, n) for n in _KERNEL_HEADERS):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def pmc_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/<kernel>_config2_fp32_pmc.txt), or None when there is none or
    the kernel's source has changed since the counters were taken.  The
    summary holds FETCH_SIZE and WRITE_SIZE (KiB per dispatch) and the
    factors that scale them to bytes, measured on an elementwise kernel of
    known size."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_config2_fp32_pmc.txt")
    try:
        kv = {}
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        src = os.path.join(ROOT, kv["source"])
        if source_digest(src) != kv["source_sha256_16"]:
            return None
        return (float(kv["fetch_kib_per_launch"]) * 1024 *
                float(kv["fetch_scale"]) +
                float(kv["write_kib_per_launch"]) * 1024 *
                float(kv["write_scale"]))
    except (OSError, KeyError, ValueError):
        return None


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on the host cores (run before any GPU use)
# ---------------------------------------------------------------------------

_CPU = {}


def _plane_job(k):
    """Oracle steps for plane k of the workload held in _CPU (inherited by
    the forked workers): grid its visibilities, transform, screen + sum."""
    from oracle import wstack as o
    wl, kall = _CPU["wl"], _CPU["k"]
    p = o.Params.of(wl)
    dw = o.plane_spacing(p)
    sel = kall == k
    ps = o.Params(p.nu, p.nv, 1, p.fov_l, p.fov_m, p.w_min + k * dw,
                  p.w_min + (k + 1) * dw, p.support, p.sigma)
    t0 = time.perf_counter()
    planes, _ = o.grid(ps, wl.uvw[sel], wl.vis[sel].astype(np.complex128),
                       wl.weight[sel])
    t1 = time.perf_counter()
    f = o.fft_planes(ps, planes, +1)
    t2 = time.perf_counter()
    o.wcorrect(ps, f)
    t3 = time.perf_counter()
    return t1 - t0, t2 - t1, t3 - t2, int(sel.sum())


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, max_procs=16):
    """The FP64 oracle on the whole headline workload, plane-parallel over
    the host cores: one process per core (at most ``max_procs``), each
    taking whole w-planes (grid that plane's visibilities, transform it,
    apply its screen into an image).  value = visibilities / wall time.
    The final sum of the per-process images is not included."""
    from oracle import wstack as o
    p = o.Params.of(wl)
    _CPU["wl"] = wl
    _CPU["k"] = o.plane_index(p, wl.uvw[:, 2])
    procs = max(1, min(max_procs, len(os.sched_getaffinity(0))))
    order = list(range(wl.nw))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        res = pool.map(_plane_job, order, chunksize=1)
    wall = time.perf_counter() - t0
    _CPU.clear()
    tg = sum(r[0] for r in res)
    tf = sum(r[1] for r in res)
    ts = sum(r[2] for r in res)
    nvis = sum(r[3] for r in res)
    return {
        "value": wl.m / wall / 1e6, "unit": "Mvis/s", "cores": procs,
        "kind": "oracle",
        "sample": (f"whole workload ({nvis} visibilities, {wl.nw} planes) "
                   f"through the FP64 NumPy oracle, one process per core "
                   f"taking whole planes; {wall:.1f} s wall; summed stage "
                   f"times grid {tg:.1f} s, FFT {tf:.1f} s, screen + sum "
                   f"{ts:.1f} s"),
        "nproc": os.cpu_count(),
        "cpu_model": cpu_model(),
        "wall_s": wall,
        "stage_cpu_s": {"grid": tg, "fft": tf, "screen": ts},
    }


# ---------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------

def time_path(plan, uvw, vis, wt, img, steps, warmup, torch):
    def step():
        plan.reset()
        img.zero_()
        plan.grid_image(uvw, vis, wt, image=img)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    plan.kernel_times(reset=True)
    plan.set_profiling(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    kt = plan.kernel_times(reset=True)
    plan.set_profiling(False)
    # A second timed pass without per-kernel events for the headline time.
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    return (t3 - t2) / steps, kt


def kernel_table(kt, wl, elem, m, st, steps):
    """Per kernel: average launch time, the bytes the launch has to move
    (see algorithmic_bytes), that rate against the HBM peak, and the
    counter-measured bytes where a current summary exists."""
    out = {}
    for k, (tot, cnt) in kt.items():
        avg = tot / max(cnt, 1)
        e = {"avg_ms": avg, "launches": cnt}
        ab = algorithmic_bytes(k, wl, elem, m, st)
        if ab is not None and avg > 0:
            e["bytes"] = ab
            e["gbs"] = ab / (avg / 1e3) / 1e9
            e["frac"] = e["gbs"] / HBM_PEAK_GBS
            tr = pmc_traffic(k) if elem == 8 else None
            if tr is not None:
                e["counter_bytes"] = tr
                e["counter_gbs"] = tr / (avg / 1e3) / 1e9
        out[k] = e
    g = [k for k in ("grid_tiles", "grid_merge") if k in kt]
    if g:
        ms = sum(kt[k][0] for k in g) / steps
        ab = algorithmic_bytes("grid", wl, elem, m, st)
        out["grid_step"] = {"kernels": g, "avg_ms": ms, "bytes": ab,
                            "gbs": ab / (ms / 1e3) / 1e9,
                            "frac": ab / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}
    return out


def grid_ms(kt, steps):
    """Gridding step time: everything but the two transform passes."""
    return sum(v[0] for k, v in kt.items()
               if k not in ("fft_cols", "row_screen_sum", "fft_cols4",
                            "fft_rows", "wcorrect")) / steps


def bench_large(args, torch, ws, synth):
    """Large single image: 1e8 visibilities, 16384^2 x 32 planes, K = 9,
    8 deg; FP32 and FP64 paths, a few steps each."""
    dev = torch.device("cuda", 0)
    t = time.perf_counter()
    wl = synth.config3(m=args.m3, precision=0)
    log(f"config3: {wl.m} vis drawn in {time.perf_counter() - t:.1f} s")
    uvw = torch.from_numpy(wl.uvw).to(dev)
    vis32 = torch.from_numpy(wl.vis).to(dev)
    wt = torch.from_numpy(wl.weight).to(dev)
    del wl.uvw, wl.vis, wl.weight
    out = {"workload": "dense-core 1e8 vis, 16384^2 x 32 w-planes, K=9 "
                       "Gaussian, 8 deg", "m": int(uvw.shape[0])}
    steps = max(1, min(args.steps, 3))
    imgs = {}
    for prec in ("fp32", "fp64"):
        vis = vis32 if prec == "fp32" else vis32.to(torch.complex128)
        plan = ws.WStackPlan(16384, 16384, 32, wl.fov_l, wl.fov_m, wl.w_min,
                             wl.w_max, 9, 0.0, prec,
                             max_vis=int(uvw.shape[0]))
        img = plan.new_image()
        sec, kt = time_path(plan, uvw, vis, wt, img, steps, 1, torch)
        g = grid_ms(kt, steps)
        out[prec] = {"ms_per_step": sec * 1e3,
                     "mvis_per_s": out["m"] / sec / 1e6,
                     "grid_ms": g, "grid_mvis_per_s": out["m"] / g / 1e3,
                     "kernels": {k: v[0] / max(v[1], 1)
                                 for k, v in kt.items()}}
        log(f"config3 {prec}: {sec * 1e3:.2f} ms/step, grid {g:.2f} ms")
        imgs[prec] = img
        del plan, vis
        torch.cuda.empty_cache()
    a = imgs["fp32"].to(torch.complex128)
    out["rel_l2_fp32_vs_fp64"] = float(
        torch.linalg.vector_norm(a - imgs["fp64"]) /
        torch.linalg.vector_norm(imgs["fp64"]))
    out["fp32_speedup"] = (out["fp64"]["ms_per_step"] /
                           out["fp32"]["ms_per_step"])
    del imgs, a, uvw, vis32, wt
    torch.cuda.empty_cache()
    return out


def bench_degrid(args, torch, ws, synth):
    """Config 5: A x (degrid) and A^H (A x - V) (grid) for a sparse 4096^2
    sky and 1e7 visibilities, FP32; one step = forward + backward."""
    from paper_2301_06061_amd.autograd import imaging_op
    dev = torch.device("cuda", 0)
    wl, x = synth.config5(m=args.m)
    plan = ws.WStackPlan.from_workload(wl)
    uvw = torch.from_numpy(wl.uvw).to(dev)
    vis = torch.from_numpy(wl.vis).to(dev)
    wt = torch.from_numpy(wl.weight).to(dev)
    xt = torch.from_numpy(x).to(dev).requires_grad_(True)

    def step():
        xt.grad = None
        loss = (imaging_op(xt, plan, uvw, wt) - vis).abs().pow(2).sum()
        loss.backward()

    steps = max(1, min(args.steps, 10))
    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    plan.set_profiling(True)
    plan.kernel_times(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    kt = plan.kernel_times(reset=True)
    plan.set_profiling(False)
    deg = sum(v[0] for k, v in kt.items()
              if k in ("screen_row_bcast", "degrid_tiles")) / steps
    log(f"config5 forward+backward: {sec * 1e3:.3f} ms/step")
    del plan, uvw, vis, wt, xt
    torch.cuda.empty_cache()
    return {"ms_per_step": sec * 1e3, "mvis_per_s": wl.m / sec / 1e6,
            "degrid_kernels_ms": deg,
            "kernels": {k: v[0] / max(v[1], 1) for k, v in kt.items()},
            "note": "degrid forward + grid/FFT/screen backward (two binning "
                    "passes, one per direction)"}


def bench_batch(args, torch, ws, synth):
    """Config 4: 64 channels (1e5-5e6 visibilities each, 1024^2-4096^2
    grids, 16-32 planes) imaged as one batch replayed from a HIP graph, with
    the (tile, chunk) of each shape class chosen by the autotuner."""
    from paper_2301_06061_amd.batch import BatchedImager
    dev = torch.device("cuda", 0)
    os.environ.setdefault("WSTACK_AUTOTUNE_CACHE",
                          os.path.join("/tmp", f"wstack_autotune_{os.getpid()}"
                                       ".json"))
    wls = synth.config4()
    uvw = [torch.from_numpy(w.uvw).to(dev) for w in wls]
    vis = [torch.from_numpy(w.vis).to(dev) for w in wls]
    wt = [torch.from_numpy(w.weight).to(dev) for w in wls]
    t = time.perf_counter()
    b = BatchedImager(wls, uvw, vis, wt, precision="fp32", tune=True)
    tune_s = time.perf_counter() - t
    for _ in range(max(1, args.warmup)):
        b.run()
    b.capture()
    b.replay()
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 10))
    t0 = time.perf_counter()
    for _ in range(steps):
        b.replay()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    m = sum(w.m for w in wls)
    choice = {}
    for tc in b.tuned:
        key = f"T{tc[0]}_C{tc[1]}"
        choice[key] = choice.get(key, 0) + 1
    log(f"config4 batch of {len(wls)}: {sec * 1e3:.3f} ms/step "
        f"(tuning {tune_s:.1f} s: {choice})")
    b.close()
    del uvw, vis, wt
    torch.cuda.empty_cache()
    return {"ms_per_step": sec * 1e3, "mvis_per_s": m / sec / 1e6,
            "channels": len(wls), "visibilities": m,
            "autotune_s": tune_s, "tuned_tile_chunk": choice}


def bench_rows(args, torch, ws, synth):
    """Baseline-major input: the headline grid and field as m / 8 rows
    (baseline, time) x 8 channels (100-200 MHz) x 4 correlations combined
    into Stokes I, through ws_grid_image_rows (FP32)."""
    dev = torch.device("cuda", 0)
    nrows = args.m // 8
    t = time.perf_counter()
    rw = synth.rows_case(0, n=4096, nw=32, support=7, nrows=nrows, nchan=8,
                         npol=4, fov_deg=5.0, precision=0, law="core")
    log(f"rows: {nrows} x 8 x 4 drawn in {time.perf_counter() - t:.1f} s")
    plan = ws.WStackPlan.from_workload(rw.geo, max_vis=nrows * 8)
    du = torch.from_numpy(rw.uvw_m).to(dev)
    df = torch.from_numpy(rw.freq_hz).to(dev)
    dv = torch.from_numpy(rw.vis).to(dev)
    dw = torch.from_numpy(rw.weight).to(dev)
    img = plan.new_image()
    coef = [0.5, 0.0, 0.0, 0.5]  # Stokes I from linear feeds: (XX + YY) / 2

    def step():
        plan.reset()
        img.zero_()
        plan.grid_image_rows(du, df, dv, dw, coef, image=img)

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 10))
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    m = nrows * 8
    log(f"rows (baseline-major) fp32: {sec * 1e3:.3f} ms/step")
    in_bytes = int(rw.uvw_m.nbytes + rw.freq_hz.nbytes + rw.vis.nbytes +
                   rw.weight.nbytes)
    del plan, du, df, dv, dw, img
    torch.cuda.empty_cache()
    return {"workload": "4096^2 x 32 w-planes, K=7 Gaussian, 5 deg: "
                        f"{nrows} rows x 8 channels x 4 correlations -> "
                        "Stokes I, dense core",
            "visibilities": m, "ms_per_step": sec * 1e3,
            "mvis_per_s": m / sec / 1e6,
            "input_bytes_per_vis": in_bytes / m}


def bench_clean(args, torch, ws, synth):
    """Imaging major cycle on the config-5 workload: the 1000-source sky's
    visibilities (predicted by the degridder), dirty beam, then major
    cycles of (residual image, Hogbom minor cycle), FP32."""
    from paper_2301_06061_amd.clean import MajorCycle
    dev = torch.device("cuda", 0)
    wl, x = synth.config5(m=args.m)
    plan = ws.WStackPlan.from_workload(wl)
    uvw = torch.from_numpy(wl.uvw).to(dev)
    wt = torch.from_numpy(wl.weight).to(dev)
    vis = plan.degrid(torch.from_numpy(x).to(dev), uvw, None)
    n_major, n_minor, gain = 2, 200, 0.1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mc = MajorCycle(plan, uvw, vis, wt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.set_profiling(True)
    plan.kernel_times(reset=True)
    mc.run(n_major, n_minor, gain)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    kt = plan.kernel_times(reset=True)
    plan.set_profiling(False)
    minor_ms = kt.get("clean_minor", (0.0, 1))[0] / n_major
    npix = wl.nu * wl.nv
    step_bytes = 3 * npix * 4  # read residual and beam, write residual
    per_it = minor_ms / n_minor
    found = int((mc.model.abs() > 0).sum().item())
    log(f"clean: beam {1e3 * (t1 - t0):.1f} ms, {n_major} major cycles "
        f"{1e3 * (t2 - t1):.1f} ms, minor {per_it * 1e3:.1f} us/iteration")
    out = {"workload": "config-5 sky (1000 sources, 4096^2, 32 w-planes, "
                       "K=7), 1e7 visibilities predicted by the degridder",
           "beam_ms": 1e3 * (t1 - t0),
           "major_cycles": n_major, "minor_per_cycle": n_minor,
           "gain": gain,
           "ms_total": 1e3 * (t2 - t1),
           "ms_per_major_cycle": 1e3 * (t2 - t1) / n_major,
           "minor_cycle_ms": minor_ms,
           "minor_iteration_us": per_it * 1e3,
           "minor_step_roofline": {
               "bound": "hbm", "bytes_per_iteration": step_bytes,
               "achieved": step_bytes / (per_it / 1e3) / 1e9,
               "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": step_bytes / (per_it / 1e3) / 1e9 / HBM_PEAK_GBS},
           "model_pixels": found,
           "kernels": {k: v[0] / max(v[1], 1) for k, v in kt.items()}}
    del mc, plan, uvw, wt, vis
    torch.cuda.empty_cache()
    return out


def bench_with_copies(args, torch, plan, wl, img):
    """The headline FP32 step with its input copies from pinned host memory
    (uvw, vis, weight) and the image copy back inside the timing, as the
    paper's GPU timings include host-device transfers."""
    dev = torch.device("cuda", 0)
    h_uvw = torch.from_numpy(wl.uvw).pin_memory()
    h_vis = torch.from_numpy(wl.vis).pin_memory()
    h_wt = torch.from_numpy(wl.weight).pin_memory()
    h_img = torch.empty(img.shape, dtype=img.dtype).pin_memory()
    d_uvw = torch.empty(h_uvw.shape, dtype=h_uvw.dtype, device=dev)
    d_vis = torch.empty(h_vis.shape, dtype=h_vis.dtype, device=dev)
    d_wt = torch.empty(h_wt.shape, dtype=h_wt.dtype, device=dev)

    def step():
        d_uvw.copy_(h_uvw, non_blocking=True)
        d_vis.copy_(h_vis, non_blocking=True)
        d_wt.copy_(h_wt, non_blocking=True)
        plan.reset()
        img.zero_()
        plan.grid_image(d_uvw, d_vis, d_wt, image=img)
        h_img.copy_(img, non_blocking=True)

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 10))
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    log(f"fp32 with pinned H2D inputs + D2H image: {sec * 1e3:.3f} ms/step")
    return {"ms_per_step": sec * 1e3, "mvis_per_s": wl.m / sec / 1e6,
            "h2d_bytes": int(h_uvw.nbytes + h_vis.nbytes + h_wt.nbytes),
            "d2h_bytes": int(h_img.nbytes)}


def fft_references(planes: int = 32, n: int = 4096) -> dict:
    """Reference rates for the two transform passes on the headline stack
    (planes x n x n complex64, dense).  First the access-pattern probe (a
    separate program; its source states the patterns): the HBM rate of
    moving column blocks with 64- or 128-byte row segments, strided or
    contiguous on each side, and of the row pass's reads.  Then torch.fft
    (the vendor FFT library) along columns and along rows, and plain copies
    whose reads are row segments of 32, 64 or 128 bytes at a stride of one
    row, written contiguously.  Rates are bytes read + written per
    second."""
    import subprocess
    exe = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                       "paper_2301_06061_amd", "probes", "access_patterns")
    probe = {"error": "not built (run __graft_entry__.build())"}
    if os.path.exists(exe):
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
        try:
            probe = json.loads(r.stdout.strip().splitlines()[-1])
        except (ValueError, IndexError):
            probe = {"error": f"rc {r.returncode}: {r.stderr[-300:]}"}
    import torch
    dev = torch.device("cuda", 0)
    x = torch.randn(planes, n, n, dtype=torch.complex64, device=dev)
    gb = 2.0 * x.numel() * 8 / 1e9

    def t(f, reps=5):
        f()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            f()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / reps

    out = {"stack": f"{planes} x {n} x {n} complex64 ({gb / 2:.2f} GB)",
           "access_patterns": probe}
    for name, f in [("torch_fft_columns", lambda: torch.fft.fft(x, dim=1)),
                    ("torch_fft_rows", lambda: torch.fft.fft(x, dim=2)),
                    ("torch_fft2", lambda: torch.fft.fft2(x)),
                    ("copy_contiguous", lambda: x.clone())]:
        ms = t(f)
        out[name] = {"ms": round(ms, 3), "tb_s": round(gb / ms, 2)}
    y = torch.empty_like(x)
    for w in (4, 8, 16):
        src = x.view(planes, n, n // w, w).permute(0, 2, 1, 3)
        dst = y.view(planes, n // w, n, w)
        ms = t(lambda: dst.copy_(src))
        out[f"copy_{w * 8}B_row_segments"] = {"ms": round(ms, 3),
                                               "tb_s": round(gb / ms, 2)}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--m", type=int, default=10_000_000)
    ap.add_argument("--m3", type=int, default=100_000_000,
                    help="visibilities of the large-image leg")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 16384^2 x 32, 1e8-visibility leg")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64 batched channels")
    ap.add_argument("--no-degrid", action="store_true",
                    help="skip the differentiable operator")
    ap.add_argument("--no-copies", action="store_true",
                    help="skip the copy-inclusive headline step")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the baseline-major input leg")
    ap.add_argument("--no-clean", action="store_true",
                    help="skip the imaging major cycle leg")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline workload (no further legs, no "
                         "CPU baseline)")
    ap.add_argument("--fft-references", action="store_true",
                    help="only time references for the transform passes on "
                         "the headline stack shape and print them: the "
                         "access-pattern probe (paper_2301_06061_amd/probes,"
                         " built by build()) and torch.fft along columns "
                         "and rows")
    ap.add_argument("--probe-copy", action="store_true",
                    help="also run one plain elementwise kernel that reads "
                         "1 GiB and writes 1 GiB (a reference for HBM byte "
                         "counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only "
                          "(the imaging path has no multi-GPU mode); "
                          "--gpus must be 1"}))
        return 2
    if args.fft_references:
        print(json.dumps(fft_references()))
        return 0
    if args.headline_only:
        args.no_cpu_baseline = args.no_large = args.no_batch = True
        args.no_degrid = args.no_copies = True
        args.no_rows = args.no_clean = True

    import synth
    t = time.perf_counter()
    wl = synth.config2(m=args.m, precision=0)
    log(f"workload: {wl.m} vis, {wl.nu}^2 x {wl.nw} planes, K={wl.support} "
        f"({time.perf_counter() - t:.1f} s to draw)")
    cpu = None
    if not args.no_cpu_baseline:
        # Before any GPU use: the worker processes are forked from here.
        cpu = cpu_baseline(wl)
        log(f"cpu baseline: {cpu['value']:.3f} Mvis/s on {cpu['cores']} "
            f"cores ({cpu['wall_s']:.1f} s)")

    import torch
    import paper_2301_06061_amd as ws

    dev = torch.device("cuda", 0)
    if args.probe_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.mul(a, 2.0, out=b)  # one elementwise kernel: 1 GiB in, 1 GiB out
        torch.cuda.synchronize()
        del a, b
    uvw = torch.from_numpy(wl.uvw).to(dev)
    vis32 = torch.from_numpy(wl.vis).to(dev)
    wt = torch.from_numpy(wl.weight).to(dev)

    plan32 = ws.WStackPlan.from_workload(wl, precision="fp32")
    img32 = plan32.new_image()
    sec32, kt32 = time_path(plan32, uvw, vis32, wt, img32, args.steps,
                            args.warmup, torch)
    stats32 = plan32.tile_stats()
    log(f"fp32: {sec32 * 1e3:.3f} ms/step; tiles {stats32}")
    for n_, (ms_, c_) in sorted(kt32.items(), key=lambda x: -x[1][0]):
        log(f"  {n_:18s} {ms_ / max(c_, 1):8.3f} ms x {c_}")
    grid32 = grid_ms(kt32, args.steps)

    res = {}
    if not args.no_fp64:
        plan64 = ws.WStackPlan.from_workload(wl, precision="fp64")
        vis64 = vis32.to(torch.complex128)
        img64 = plan64.new_image()
        sec64, kt64 = time_path(plan64, uvw, vis64, wt, img64, args.steps,
                                args.warmup, torch)
        stats64 = plan64.tile_stats()
        log(f"fp64: {sec64 * 1e3:.3f} ms/step")
        for n_, (ms_, c_) in sorted(kt64.items(), key=lambda x: -x[1][0]):
            log(f"  {n_:18s} {ms_ / max(c_, 1):8.3f} ms x {c_}")
        a = img32.to(torch.complex128)
        rel = float(torch.linalg.vector_norm(a - img64) /
                    torch.linalg.vector_norm(img64))
        grid64 = grid_ms(kt64, args.steps)
        res["fp64"] = {
            "ms_per_step": sec64 * 1e3,
            "mvis_per_s": wl.m / sec64 / 1e6,
            "grid_mvis_per_s": wl.m / (grid64 / 1e3) / 1e6,
            "fp32_speedup": sec64 / sec32,
            "fp32_grid_speedup": grid64 / grid32,
            "kernels": kernel_table(kt64, wl, 16, wl.m, stats64, args.steps),
        }
        res["rel_l2_fp32_vs_fp64"] = rel
        del plan64, img64, vis64, a
        torch.cuda.empty_cache()

    # Roofline of the dominant kernel (largest share of the step): the
    # bytes this launch has to move, over its average launch time from HIP
    # events on the plan's stream.
    table = kernel_table(kt32, wl, 8, wl.m, stats32, args.steps)
    name, (tot, cnt) = max(kt32.items(), key=lambda x: x[1][0])
    e = table[name]
    roof = None
    if "bytes" in e:
        roof = {"kernel": name, "bound": "hbm", "achieved": e["gbs"],
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": e["frac"],
                "traffic": e.get("counter_bytes"), "avg_ms": e["avg_ms"],
                "algorithmic_bytes": e["bytes"],
                "full_stack_bytes": algorithmic_bytes(name, wl, 8, wl.m),
                "full_stack_effective_gbs": algorithmic_bytes(
                    name, wl, 8, wl.m) / (e["avg_ms"] / 1e3) / 1e9}

    extra = {}
    if not args.no_copies:
        extra["fp32_with_copies"] = bench_with_copies(args, torch, plan32, wl,
                                                      img32)
    del plan32, img32, uvw, vis32, wt
    torch.cuda.empty_cache()
    if not args.no_degrid:
        extra["degrid_config5"] = bench_degrid(args, torch, ws, synth)
    if not args.no_rows:
        extra["rows_config2"] = bench_rows(args, torch, ws, synth)
    if not args.no_clean:
        extra["clean_config5"] = bench_clean(args, torch, ws, synth)
    if not args.no_batch:
        extra["batch_config4"] = bench_batch(args, torch, ws, synth)
    if not args.no_large:
        extra["large_config3"] = bench_large(args, torch, ws, synth)

    out = {
        "metric": "Mvis/s gridded + image s, 1 GPU; FP32 vs FP64 path at "
                  "stated rel-L2 err",
        "value": wl.m / sec32 / 1e6,
        "unit": "Mvis/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "dense-core 1e7 vis, 4096^2 x 32 w-planes, "
                               "K=7 Gaussian, 5 deg, FP32 path",
                   "m": wl.m, "n": wl.nu, "nw": wl.nw, "support": wl.support,
                   "precision": "fp32"},
        "image_s": sec32,
        "grid_mvis_per_s": wl.m / (grid32 / 1e3) / 1e6,
        "ggpas": wl.m * wl.support ** 2 / (grid32 / 1e3) / 1e9,
        "roofline": roof,
        "tile_stats": stats32,
        "kernels_fp32": table,
        "cpu_baseline": cpu,
    }
    out.update(res)
    out.update(extra)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
