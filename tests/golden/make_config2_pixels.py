"""Write config2_pixels.txt: dirty-image pixels of the dense-core 1e7
visibility workload (4096^2 x 32 planes, K = 7, 5 deg; seed 0, complex64
visibilities) computed by the oracle's per-pixel definition
(``oracle.wstack.image_pixels_direct``: each visibility's screen times the
DFT of its own on-grid taps, no FFT and no plane stack).

Only the oracle and the seeded input generator run here.  Usage:
    python tests/golden/make_config2_pixels.py [--procs 8]
"""
import argparse
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "config2_pixels.txt")
N = 4096


def pixels():
    fixed = [(0, 0), (0, N - 1), (N - 1, 0), (N - 1, N - 1), (N // 2, N // 2),
             (N // 2, 0), (0, N // 2), (N - 1, N // 2), (N // 2, N - 1),
             (N // 2 - 1, N // 2 + 1), (1, 1), (N // 2 + 7, N // 2 - 3)]
    rng = np.random.default_rng(2024)
    rand = [(int(q), int(p)) for q, p in rng.integers(0, N, (64 - len(fixed),
                                                             2))]
    return fixed + rand


def _work(chunk):
    import synth
    from oracle import wstack as o
    wl = synth.config2(precision=0)
    p = o.Params.of(wl)
    return o.image_pixels_direct(p, wl.uvw, wl.vis, wl.weight, chunk)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    a = ap.parse_args()
    px = pixels()
    chunks = [px[i::a.procs] for i in range(a.procs)]
    with mp.get_context("spawn").Pool(a.procs) as pool:
        res = pool.map(_work, chunks)
    val = {}
    for ch, r in zip(chunks, res):
        for pq, v in zip(ch, r):
            val[pq] = v
    with open(OUT, "w") as f:
        f.write("# Dirty-image pixels I[q][p] of the dense-core workload "
                "(1e7 visibilities, seed 0,\n# complex64 values, 4096^2 x 32 "
                "planes, K = 7, 5 deg field) from the oracle's per-pixel\n"
                "# definition (Eqs. 2-3, no FFT), written by "
                "make_config2_pixels.py.\n# q p re im\n")
        for q, p in px:
            v = val[(q, p)]
            f.write(f"{q} {p} {float(v.real)!r} {float(v.imag)!r}\n")
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
