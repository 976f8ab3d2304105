"""Autotuner for the gridder's launch parameters.

For a shape class - grid size, plane count, kernel support and type,
precision and the visibility count rounded to a half decade - it times the
one-call imaging step a batch runs per channel (binning, tile accumulation,
merge, column FFT and fused rows + screen + plane sum, ws_grid_image) on
the caller's own data for every candidate (tile edge T, records per work
item C) and keeps the fastest.  The whole step, not the gridding alone:
the tile edge also decides whether the imaging may leave tiles without
records unwritten and skip them (64-cell tiles), which a gridding-only
timing does not see.
Results are cached in a JSON file keyed by GPU architecture and shape
class ($WSTACK_AUTOTUNE_CACHE, default ~/.cache/wstack/autotune.json).
The kernel support and type are not tuned: they change the result, so
each (K, kernel type) has its own compiled kernel and its own cache
entries.

Not among the candidates, and why:
* lanes per visibility: the gridder's lane mapping (one kernel row per
  lane, floor(64 / K) records per group) is a compile-time structure per
  K, chosen by measurement against one tap per lane (K^2 lanes per record:
  1.19 -> 1.06 ms FP32, 2.04 -> 1.32 ms FP64 on 1e7 visibilities); it is
  not a launch parameter;
* plane batch: every plan keeps its whole plane stack resident (288 GB of
  HBM holds the largest workloads here: 137 GB for 16384^2 x 32 FP64), so
  all planes of a channel are gridded in one launch and transformed in one
  launch; there is no plane batch to choose.
"""
from __future__ import annotations

import json
import math
import os
from typing import Optional, Sequence, Tuple

import torch

from .api import WStackPlan

TILES = (32, 64)
CHUNKS = (1024, 2048, 4096, 8192)


def cache_path() -> str:
    return os.environ.get(
        "WSTACK_AUTOTUNE_CACHE",
        os.path.join(os.path.expanduser("~"), ".cache", "wstack",
                     "autotune.json"))


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def shape_key(nu, nv, nw, support, precision, m, kernel="gauss") -> str:
    bucket = 0 if m <= 0 else round(2 * math.log10(m)) / 2
    return (f"{_arch()}|{nu}x{nv}x{nw}|K{support}{kernel}|{precision}|"
            f"m1e{bucket:g}")


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db: dict) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(key: str) -> Optional[Tuple[int, int]]:
    e = _load().get(key)
    return None if e is None else (int(e["tile"]), int(e["chunk"]))


def _valid_tile(t, wl) -> bool:
    return t <= min(wl.nu, wl.nv) and t > wl.support - 1


def time_step(plan: WStackPlan, uvw, vis, weight, reps: int = 3) -> float:
    """Median milliseconds of one one-call grid-and-image step into a zeroed
    image (after one warm-up)."""
    img = plan.new_image()

    def step():
        plan.reset()
        img.zero_()
        plan.grid_image(uvw, vis, weight, image=img)

    step()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        step()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    plan.reset()
    return sorted(times)[len(times) // 2]


def tune(wl, uvw, vis, weight=None, precision: str = "fp32",
         tiles: Sequence[int] = TILES, chunks: Sequence[int] = CHUNKS,
         reps: int = 3, use_cache: bool = True) -> Tuple[int, int]:
    """Best (tile, chunk) for this workload's shape class.

    ``wl`` carries the geometry (nu, nv, nw, fov, w range, support, sigma);
    uvw, vis, weight are the device tensors that will be gridded.
    """
    m = int(uvw.shape[0])
    kernel = getattr(wl, "kernel", "gauss")
    key = shape_key(wl.nu, wl.nv, wl.nw, wl.support, precision, m, kernel)
    if use_cache:
        hit = lookup(key)
        if hit is not None:
            return hit
    best = None
    trials = {}
    for t in tiles:
        if not _valid_tile(t, wl):
            continue
        for c in chunks:
            plan = WStackPlan(wl.nu, wl.nv, wl.nw, wl.fov_l, wl.fov_m,
                              wl.w_min, wl.w_max, wl.support, wl.sigma,
                              precision, max_vis=max(1, m), tile=t, chunk=c,
                              kernel=kernel, beta=getattr(wl, "beta", 0.0))
            ms = time_step(plan, uvw, vis, weight, reps)
            plan.close()
            del plan
            trials[f"T{t}_C{c}"] = ms
            if best is None or ms < best[2]:
                best = (t, c, ms)
    if best is None:
        return (0, 0)
    if use_cache:
        db = _load()
        db[key] = {"tile": best[0], "chunk": best[1], "ms": best[2],
                   "trials": trials}
        _store(db)
    return best[0], best[1]
