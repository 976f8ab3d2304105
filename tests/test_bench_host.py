"""Host logic of bench.py: algorithmic bytes per kernel and the rule that
measured HBM traffic is reported only while the kernel's source is the one
the counters were taken on."""
import os

import bench


class _W:
    nu = nv = 4096
    nw = 32


def test_algorithmic_bytes_of_the_column_pass_and_gridding():
    cells = 4096 * 4096 * 32
    assert bench.algorithmic_bytes("fft_cols", _W, 8, 10**7) == 2 * cells * 8
    assert bench.algorithmic_bytes("fft_cols", _W, 16, 10**7) == 2 * cells * 16
    # read the stack once, read and write the image once
    assert bench.algorithmic_bytes("row_screen_sum", _W, 8, 10**7) == (
        cells * 8 + 2 * 4096 * 4096 * 8)
    # every cell written once plus one 24-byte record (40 for FP64) read
    assert bench.algorithmic_bytes("grid", _W, 8, 10**7) == cells * 8 + 24e7
    assert bench.algorithmic_bytes("grid", _W, 16, 10**7) == (
        cells * 16 + 40e7)
    assert bench.algorithmic_bytes("no_such_kernel", _W, 8, 1) is None


def test_traffic_needs_the_recorded_source(tmp_path, monkeypatch):
    root = tmp_path
    (root / "profiles").mkdir()
    src_dir = root / "src"
    src_dir.mkdir()
    src = src_dir / "k.hip"
    src.write_text("kernel source\n")
    csrc = root / "paper_2301_06061_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in ("ws_common.h", "ws_kernels.h"):
        (csrc / name).write_text(f"// {name}\n")
    monkeypatch.setattr(bench, "ROOT", str(root))
    digest = bench.source_digest(str(src))
    (root / "profiles" / "k_config2_fp32_pmc.txt").write_text(
        "# header line: not a value\n"
        "source: src/k.hip\n"
        f"source_sha256_16: {digest}\n"
        "fetch_kib_per_launch: 100.0\n"
        "write_kib_per_launch: 50.0\n"
        "fetch_scale: 2.0\n"
        "write_scale: 1.0\n")
    assert bench.pmc_traffic("k") == 100.0 * 1024 * 2.0 + 50.0 * 1024 * 1.0
    # a change to a shared kernel header changes the kernels too
    (csrc / "ws_common.h").write_text("// record layout changed\n")
    assert bench.pmc_traffic("k") is None
    (csrc / "ws_common.h").write_text("// ws_common.h\n")
    assert bench.pmc_traffic("k") is not None
    src.write_text("kernel source, changed\n")
    assert bench.pmc_traffic("k") is None
    assert bench.pmc_traffic("missing") is None


def test_committed_column_pass_counters_match_their_source():
    """The committed counter summary of the column pass names a source file
    of this tree; while that file is unchanged the traffic is a positive
    byte count below the algorithmic bytes (skipped strips and rows)."""
    root = os.path.dirname(os.path.abspath(bench.__file__))
    path = os.path.join(root, "profiles", "fft_cols_config2_fp32_pmc.txt")
    assert os.path.exists(path)
    t = bench.pmc_traffic("fft_cols")
    if t is not None:
        assert 0 < t < bench.algorithmic_bytes("fft_cols", _W, 8, 10**7)


def test_algorithmic_bytes_from_tile_statistics():
    """With the binning's tile counts, each pass is charged only for what
    the one-call path has to touch: busy tiles, marked strips, record reads
    and split-tile partials."""
    st = {"tile": 64, "busy": 100, "idle": 5, "split": 3, "extra_items": 7,
          "strips": 10, "record_reads": 12345}
    tile_b = 64 * 64 * 8
    strip_b = 4096 * 64 * 8
    assert bench.algorithmic_bytes("fft_cols", _W, 8, 10**7, st) == (
        100 * tile_b + 10 * strip_b)
    assert bench.algorithmic_bytes("row_screen_sum", _W, 8, 10**7, st) == (
        10 * strip_b + 2 * 4096 * 4096 * 8)
    assert bench.algorithmic_bytes("grid", _W, 8, 10**7, st) == (
        100 * tile_b + 12345 * 24 + 2 * 10 * tile_b)
    # binning is charged per visibility either way
    assert bench.algorithmic_bytes("bin_count", _W, 8, 10, st) == 10 * 32
    assert bench.algorithmic_bytes("bin_scatter", _W, 8, 10, st) == (
        10 * (24 + 8 + 4 + 8 + 4 + 24))


def test_gpu_count_other_than_one_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().out
