"""bench.py's host-side contract: it runs on one GPU only and says so (without touching a GPU)
when asked for more."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    for n in (2, 8):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n), "--steps", "1"],
                           capture_output=True, text=True, timeout=120, cwd=ROOT)
        assert r.returncode == 2
        assert "one GPU only" in r.stderr and r.stdout == ""


def test_bench_help_lists_the_legs():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--gpus", "--no-cpu", "--tile-w", "--no-mirror"):
        assert flag in r.stdout


def test_compare_unfolded_checks_the_computed_rows_and_the_mirror_rows():
    """bench.compare_unfolded on CPU tensors: the top tile rows must match bit for bit, the
    bottom rows must be their mirror copies, and the rest is reported as differences."""
    import dataclasses

    import pytest
    import torch

    sys.path.insert(0, ROOT)
    import bench
    import workloads as W

    wl = W.small(1, width=32, height=24, center=(16.0, 12.0))
    wl = dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, tile_w=8, mirror=3))  # 8x8 tiles: 3 rows
    g = torch.Generator().manual_seed(0)
    full = torch.rand(24, 32, generator=g) + 1.0
    full = 0.5 * (full + torch.flip(full, [0]))          # up-down symmetric
    full = 0.5 * (full + torch.flip(full, [1]))          # and left-right
    folded = full.clone()
    unfolded = full.clone()
    unfolded[16:] *= 1.0 + 1e-7                            # rows 16.. come from mirror copies
    r = bench.compare_unfolded(wl, folded, unfolded)
    assert r["computed_rows_bit_identical"] and not r["image_bit_identical"]
    assert 0 < r["rel_l2"] < 1e-6 and r["max_rel_pixel"] < 2e-7
    bad = folded.clone()
    bad[0, 0] += 1.0                                       # a computed pixel that differs
    with pytest.raises(AssertionError):
        bench.compare_unfolded(wl, bad, unfolded)
    bad = folded.clone()
    bad[23, 5] += 1.0                                      # a mirror row that is not a copy
    with pytest.raises(AssertionError):
        bench.compare_unfolded(wl, bad, unfolded)
