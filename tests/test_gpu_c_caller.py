"""A caller of the C ABI without Python or torch: the example program
paper_2608_23245_amd/examples/fdtbx_pattern.cpp (built next to the library) reads a model and
its atoms from a file, runs the reflection list (with the extinction cull), the structure
factors and the one-call pattern on buffers it allocates with hipMalloc, and writes the image
and the list.  The list must equal the oracle's enumeration bit for bit and the image the
oracle's pattern to the pattern tolerances.  A malformed input file is rejected before any
HIP call, which the CPU case checks."""
import dataclasses
import importlib
import math
import os
import subprocess
import sys

import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

DEG = math.pi / 180
EXE = importlib.import_module("paper_2608_23245_amd.build").EXAMPLE


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def need_exe():
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is missing: build the library first (python -m paper_2608_23245_amd.build)")


def write_input(path, wl):
    from paper_2608_23245_amd import binding as B
    a = wl.atoms
    n = int(np.asarray(a.x).size)
    ff = np.ascontiguousarray(a.ff, dtype=np.float32)
    with open(path, "wb") as f:
        f.write(bytes(B.make_model(wl)))
        f.write(np.array([n, ff.shape[0]], dtype=np.int64).tobytes())
        for v in (a.x, a.y, a.z, a.B, a.occ):
            f.write(np.ascontiguousarray(v, dtype=np.float32).tobytes())
        f.write(np.ascontiguousarray(a.type, dtype=np.int32).tobytes())
        f.write(ff.tobytes())


def read_output(path, wl):
    raw = open(path, "rb").read()
    npix = wl.geom.width * wl.geom.height
    img = np.frombuffer(raw, dtype=np.float32, count=npix).reshape(wl.geom.height, wl.geom.width)
    n_hkl = int(np.frombuffer(raw, dtype=np.int64, count=1, offset=4 * npix)[0])
    hkl = np.frombuffer(raw, dtype=np.int32, offset=4 * npix + 8).reshape(-1, 3)
    assert hkl.shape[0] == n_hkl
    return img, hkl


CASES = {
    "laue_tilted": dict(seed=311, width=40, height=30, center=(17.3, 12.6), tilt=12 * DEG,
                        sigma_theta=3 * DEG, gamma_theta=1 * DEG, g=(0.02, 0.01, 0.03)),
    "gaussian_folded": dict(seed=312, width=48, height=26, center=(24.0, 13.4), sigma_theta=2 * DEG, lineshape=1,
                            tile_w=16, mirror=1),
    "hosemann_ragged": dict(seed=313, width=37, height=23, center=(-3.0, 8.5), sigma_theta=2 * DEG,
                            gamma_theta=2 * DEG, g=(0.03, 0.02, 0.01), lineshape=2, tile_w=4),
}


def make_case(name):
    kw = dict(CASES[name])
    tw, mirror = kw.pop("tile_w", 0), kw.pop("mirror", 0)
    wl = W.small(**kw)
    return dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, tile_w=tw, mirror=mirror))


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(CASES))
def test_c_caller_pattern_vs_oracle(name, tmp_path):
    need_exe()
    wl = make_case(name)
    g = wl.geom
    say(f"C caller {name}: {g.width}x{g.height}, tile {g.tile_w}, mirror {g.mirror}, lineshape {wl.dis.lineshape}")
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    write_input(inp, wl)
    r = subprocess.run([EXE, str(inp), str(out)], capture_output=True, text=True, timeout=120)
    say(f"  exit {r.returncode}: {r.stdout.strip()} {r.stderr.strip()}")
    assert r.returncode == 0, r.stderr
    img, hkl = read_output(out, wl)
    ref_hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    ref_hkl = ref_hkl[~O.extinct_mask(ref_hkl, wl.dis, wl.quad.extinction)]
    assert hkl.shape[0] > 0 and np.array_equal(hkl, ref_hkl)
    ref = O.pattern(wl, O.prepare(wl, hkl=np.ascontiguousarray(ref_hkl)))
    got = img.astype(np.float64)
    assert ref.max() > 0
    rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    big = ref > 1e-3 * ref.max()
    px = float(np.max(np.abs(got[big] - ref[big]) / ref[big]))
    say(f"  rel-L2 {rel:.2e}, per-pixel {px:.2e}")
    assert rel <= 1e-4 and px <= 1e-3


def test_c_caller_rejects_a_truncated_input(tmp_path):
    need_exe()
    wl = make_case("laue_tilted")
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    write_input(inp, wl)
    data = inp.read_bytes()
    inp.write_bytes(data[: len(data) - 5])
    r = subprocess.run([EXE, str(inp), str(out)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "malformed input" in r.stderr
    assert not out.exists()
    r = subprocess.run([EXE, str(inp)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "usage" in r.stderr
