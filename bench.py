"""Benchmark of the w-stacking imaging path on one MI355X.

One step = the whole hot path on one batch of synthetic visibilities held in
HBM, in one call (ws_grid_image): binning + gridding onto N_w w-planes, then
the per-plane 2-D FFT, w-screen and plane sum into the dirty image.  Default workload: 1e7 visibilities with a dense core
(r = R U^2, w = wmax r/R + N(0, 0.1 wmax)), 4096^2 grid, 32 w-planes, 7x7
Gaussian kernel, 5 deg field, FP32 path; the FP64 path is timed on the same
inputs for comparison.

Prints one JSON line (the last line on stdout).  value = visibilities imaged
per second (Mvis/s) over the timed steps.
"""
from __future__ import annotations

import argparse
import json
import math
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


def algorithmic_bytes(name, wl, elem, m):
    """Bytes a kernel must move per launch (reads + writes), by definition
    of the step it performs (not what the kernel happens to skip).

    fft_cols:       the 2-D transform of the stack: read + write the stack
                    once (the row half is fused into row_screen_sum);
    row_screen_sum: read the stack once + read/write the image once;
    grid (step):    write every stack cell once + read each binned record
                    once (zero_idle + grid_tiles + grid_merge together; the
                    one-call path writes only the tiles with records);
    bin_count:      read uvw (24 B) + write key/rank (8 B) per visibility;
    bin_scatter:    read uvw, vis, weight, key/rank + write a record.
    """
    cells = wl.nu * wl.nv * wl.nw
    img = wl.nu * wl.nv
    rec = 32 if elem == 8 else 48
    vis_b = elem
    return {
        "fft_cols": 2 * cells * elem,
        "row_screen_sum": cells * elem + 2 * img * elem,
        "grid": cells * elem + m * rec,
        "bin_count": m * (24 + 8),
        "bin_scatter": m * (24 + vis_b + 4 + 8 + rec),
    }.get(name)


def source_digest(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


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
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = plan.kernel_times(reset=True)
    plan.set_profiling(False)
    # A second timed pass without per-kernel events for the headline time.
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    return (t3 - t2) / steps, (t1 - t0) / steps, kt


def cpu_baseline(wl, budget_s=12.0):
    """The FP64 oracle on a bounded sample of the same workload.

    Sample: w-planes taken one at a time from the middle outwards, each with
    the visibilities that fall on it, gridded and then transformed and
    screened, until about ``budget_s`` seconds of oracle time are spent; the
    time is scaled to the whole job (gridding by visibility count, FFT and
    screen by plane count).  NumPy runs these steps on one core.
    """
    from oracle import wstack as o
    p = o.Params.of(wl)
    kall = o.plane_index(p, wl.uvw[:, 2])
    dw = o.plane_spacing(p)
    order = sorted(range(wl.nw), key=lambda k: abs(k - (wl.nw - 1) / 2))
    t_grid = t_fft = 0.0
    nvis = nplanes = 0
    for k in order:
        sel = kall == k
        ps = o.Params(p.nu, p.nv, 1, p.fov_l, p.fov_m, p.w_min + k * dw,
                      p.w_min + (k + 1) * dw, p.support, p.sigma)
        t0 = time.perf_counter()
        planes, _ = o.grid(ps, wl.uvw[sel], wl.vis[sel].astype(np.complex128),
                           wl.weight[sel])
        t1 = time.perf_counter()
        o.wcorrect(ps, o.fft_planes(ps, planes, +1))
        t2 = time.perf_counter()
        t_grid += t1 - t0
        t_fft += t2 - t1
        nvis += int(sel.sum())
        nplanes += 1
        if t_grid + t_fft >= budget_s:
            break
    est = t_grid * wl.m / max(nvis, 1) + t_fft * wl.nw / nplanes
    return {
        "value": wl.m / est / 1e6, "unit": "Mvis/s", "cores": 1,
        "kind": "oracle",
        "sample": (f"FP64 NumPy oracle on {nplanes} of {wl.nw} w-planes: "
                   f"{nvis} visibilities gridded in {t_grid:.1f} s, FFT + "
                   f"screen of those planes in {t_fft:.1f} s; scaled to "
                   f"{wl.m} visibilities and {wl.nw} planes = {est:.0f} s "
                   f"per image"),
    }


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

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.set_profiling(True)
    plan.kernel_times(reset=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    kt = plan.kernel_times(reset=True)
    plan.set_profiling(False)
    deg = sum(v[0] for k, v in kt.items()
              if k in ("screen_row_bcast", "degrid_tiles", "bin_count",
                       "bin_scatter", "scan_keys", "tile_work",
                       "zero_counts")) / args.steps
    log(f"config5 forward+backward: {sec * 1e3:.3f} ms/step")
    return {"ms_per_step": sec * 1e3, "mvis_per_s": wl.m / sec / 1e6,
            "kernels": {k: v[0] / max(v[1], 1) for k, v in kt.items()},
            "note": "degrid forward + grid/FFT/screen backward; kernel "
                    "times include both directions' shared binning"}


def bench_batch(args, torch, ws, synth):
    """Config 4: 64 channels (1e5-5e6 visibilities each, 1024^2-4096^2
    grids, 16-32 planes) imaged as one batch replayed from a HIP graph."""
    from paper_2301_06061_amd.batch import BatchedImager
    dev = torch.device("cuda", 0)
    wls = synth.config4()
    uvw = [torch.from_numpy(w.uvw).to(dev) for w in wls]
    vis = [torch.from_numpy(w.vis).to(dev) for w in wls]
    wt = [torch.from_numpy(w.weight).to(dev) for w in wls]
    b = BatchedImager(wls, uvw, vis, wt, precision="fp32")
    for _ in range(args.warmup):
        b.run()
    b.capture()
    b.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.replay()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    m = sum(w.m for w in wls)
    log(f"config4 batch of {len(wls)}: {sec * 1e3:.3f} ms/step")
    b.close()
    return {"ms_per_step": sec * 1e3, "mvis_per_s": m / sec / 1e6,
            "channels": len(wls), "visibilities": m}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--m", type=int, default=10_000_000)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe-copy", action="store_true",
                    help="also run one plain elementwise kernel that reads "
                         "1 GiB and writes 1 GiB (a reference for HBM byte "
                         "counters)")
    ap.add_argument("--degrid", action="store_true",
                    help="also time the differentiable operator on the "
                         "config-5 workload (degrid forward + grid backward)")
    ap.add_argument("--batch", action="store_true",
                    help="also time 64 batched channels (config-4 workload)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; "
                          "--gpus must be 1"}))
        return 2

    import torch
    import paper_2301_06061_amd as ws
    import synth

    dev = torch.device("cuda", 0)
    if args.probe_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.mul(a, 2.0, out=b)  # one elementwise kernel: 1 GiB in, 1 GiB out
        torch.cuda.synchronize()
        del a, b
    t = time.perf_counter()
    wl = synth.config2(m=args.m, precision=0)
    log(f"workload: {wl.m} vis, {wl.nu}^2 x {wl.nw} planes, K={wl.support} "
        f"({time.perf_counter() - t:.1f} s to draw)")
    uvw = torch.from_numpy(wl.uvw).to(dev)
    vis32 = torch.from_numpy(wl.vis).to(dev)
    wt = torch.from_numpy(wl.weight).to(dev)

    plan32 = ws.WStackPlan.from_workload(wl, precision="fp32")
    img32 = plan32.new_image()
    sec32, sec32_prof, kt32 = time_path(plan32, uvw, vis32, wt, img32,
                                        args.steps, args.warmup, torch)
    stats32 = plan32.tile_stats()
    log(f"fp32: {sec32 * 1e3:.3f} ms/step; tiles {stats32}")
    for n_, (ms_, c_) in sorted(kt32.items(), key=lambda x: -x[1][0]):
        log(f"  {n_:18s} {ms_ / max(c_, 1):8.3f} ms x {c_}")

    res = {}
    if not args.no_fp64:
        plan64 = ws.WStackPlan.from_workload(wl, precision="fp64")
        vis64 = vis32.to(torch.complex128)
        img64 = plan64.new_image()
        sec64, _, kt64 = time_path(plan64, uvw, vis64, wt, img64, args.steps,
                                   args.warmup, torch)
        log(f"fp64: {sec64 * 1e3:.3f} ms/step")
        for n_, (ms_, c_) in sorted(kt64.items(), key=lambda x: -x[1][0]):
            log(f"  {n_:18s} {ms_ / max(c_, 1):8.3f} ms x {c_}")
        a = img32.to(torch.complex128)
        rel = float(torch.linalg.vector_norm(a - img64) /
                    torch.linalg.vector_norm(img64))
        grid64 = sum(kt64[k][0] for k in kt64 if k not in (
            "fft_cols", "row_screen_sum")) / args.steps
        res["fp64"] = {
            "ms_per_step": sec64 * 1e3,
            "mvis_per_s": wl.m / sec64 / 1e6,
            "grid_mvis_per_s": wl.m / (grid64 / 1e3) / 1e6,
            "fp32_speedup": sec64 / sec32,
            "fp32_grid_speedup": None,
        }
        res["rel_l2_fp32_vs_fp64"] = rel
        del plan64, img64, vis64
    grid32 = sum(kt32[k][0] for k in kt32 if k not in (
        "fft_cols", "row_screen_sum")) / args.steps
    if "fp64" in res:
        res["fp64"]["fp32_grid_speedup"] = (res["fp64"]["grid_mvis_per_s"] and
                                            (wl.m / (grid32 / 1e3) / 1e6) /
                                            res["fp64"]["grid_mvis_per_s"])

    # Roofline of the dominant kernel (largest share of the step), from its
    # average launch time measured with HIP events on the plan's stream.
    name, (tot, cnt) = max(kt32.items(), key=lambda x: x[1][0])
    avg_ms = tot / max(cnt, 1)
    ab = algorithmic_bytes(name, wl, 8, wl.m)
    roof = None
    if ab is not None:
        ach = ab / (avg_ms / 1e3) / 1e9
        tr = pmc_traffic(name)
        roof = {"kernel": name, "bound": "hbm", "achieved": ach,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": tr,
                "avg_ms": avg_ms, "algorithmic_bytes": ab}
    kernels = {k: {"avg_ms": v[0] / max(v[1], 1), "launches": v[1]}
               for k, v in kt32.items()}
    # The gridding step as a whole (its kernels write the stack together).
    # Without zero_idle (the one-call path) only the tiles that received
    # records are written: the step moves those cells plus the records.
    gk = [k for k in ("zero_idle", "grid_tiles", "grid_merge") if k in kt32]
    gb = None
    if gk:
        g_ms = sum(kt32[k][0] for k in gk) / args.steps
        gab = algorithmic_bytes("grid", wl, 8, wl.m)
        if "zero_idle" not in kt32:
            gab = (wl.m * 32 +
                   stats32["busy"] * stats32["tile"] ** 2 * 8)
        gb = {"kernels": gk, "ms": g_ms, "bytes": gab,
              "tiles_written": stats32["busy"],
              "achieved_gbs": gab / (g_ms / 1e3) / 1e9,
              "frac": gab / (g_ms / 1e3) / 1e9 / HBM_PEAK_GBS}

    extra = {}
    if args.degrid:
        extra["degrid_config5"] = bench_degrid(args, torch, ws, synth)
    if args.batch:
        extra["batch_config4"] = bench_batch(args, torch, ws, synth)

    cpu = None
    if not args.no_cpu_baseline:
        t = time.perf_counter()
        cpu = cpu_baseline(wl)
        log(f"cpu baseline: {cpu['value']:.3f} Mvis/s "
            f"({time.perf_counter() - t:.1f} s)")

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
        "grid_step_roofline": gb,
        "kernels_fp32": kernels,
        "cpu_baseline": cpu,
    }
    out.update(res)
    out.update(extra)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
