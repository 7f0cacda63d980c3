"""The oracle's C loops (oracle/oracle_c.c) built with AddressSanitizer and UndefinedBehavior-
Sanitizer, run on small workloads in a child process, and compared bit for bit with the
ordinary build.

Every C entry point is driven: structure factors, the pattern, the exact skip (reach and the
skipped profile table), single-point profiles, the gradient sums, the deterministic splat and
the cylindrical average, over the Laue, Gaussian and Hosemann lineshapes, a Lorentzian and a
Voigt angular shape, a tilted fibre, a one-pixel-wide detector and nonzero g.  Any invalid
access or undefined operation aborts the child (-fno-sanitize-recover); both builds keep
-ffp-contract=off, so the arithmetic, and every output, is the same bit for bit."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "oracle_c.c")

CHILD = r"""
import ctypes, math, sys
import numpy as np
sys.path[:0] = [sys.argv[1], sys.argv[2]]
import workloads as W
from oracle import oracle as O

DEG = math.pi / 180.0
CASES = [
    W.small(seed=41, width=13, height=11),
    W.with_disorder(W.small(seed=42, width=9, height=14, g=(0.04, 0.02, 0.01)), lineshape=1),
    W.with_disorder(W.small(seed=43, width=10, height=10, sigma_theta=0.0, gamma_theta=2.5 * DEG), lineshape=2,
                    B_axis=(3.0, 0.0, 1.0)),
    W.small(seed=44, width=1, height=7, sigma_theta=2 * DEG, gamma_theta=1 * DEG, tilt=20 * DEG),
]


def run(path):
    O._lib = ctypes.CDLL(path)
    O.set_threads(2)
    out = []
    for k, wl in enumerate(CASES):
        hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
        F = O.structure_factors_c(hkl, wl.cell, wl.atoms)
        P = O.prepare(wl, hkl=hkl, F=F, cull_extinct=False)
        R, Z = O.pixel_rz(wl.geom)
        R, Z = R.ravel(), Z.ravel()
        rng = np.random.default_rng(k)
        G = rng.standard_normal(R.size)
        g = O.gradients(wl, P, G, R, Z)
        pts = rng.uniform(-0.3, 0.3, (16, 3))
        ridx = rng.integers(0, hkl.shape[0], 16)
        img, n_ev = O.splat(wl, P, 3, 4, count=True)
        out += [F.real, F.imag, O.pattern_at(P, R, Z), O.pattern_at(P, R, Z, use_skip=False),
                O.reachable(wl, hkl, R, Z).astype(np.float64), O.profile_table(P, R, Z, use_skip=True).ravel(),
                O.profile_points(P, ridx, pts), img.ravel(), np.array([float(n_ev)]),
                O.cyl_at(P, R, Z, 0.02)]
        out += [np.ravel(np.asarray(v, dtype=np.float64)) for v in g["atoms"].values()]
        out += [np.ravel(np.asarray(g[n], dtype=np.float64)) for n in ("sigma_theta", "gamma_theta", "N_base", "g", "B_axis")]
    return np.concatenate(out)


a = run(sys.argv[3])
b = run(sys.argv[4])
assert a.shape == b.shape and np.all(np.isfinite(a)), (a.shape, b.shape)
assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), int(np.sum(a != b))
print("sanitized oracle: %d values, bit-identical to the ordinary build" % a.size)
"""


def _gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.slow
def test_oracle_c_under_address_and_undefined_sanitizers(tmp_path):
    asan = _gcc_runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    plain = str(tmp_path / "oracle_plain.so")
    checked = str(tmp_path / "oracle_sanitized.so")
    common = ["-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC"]
    subprocess.check_call(["gcc", "-O2", *common, "-o", plain, SRC, "-lm"])
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", *common, "-o", checked, SRC, "-lm"])
    env = dict(os.environ)
    # the sanitizer runtime has to come first in the process; whatever is preloaded already stays
    env["LD_PRELOAD"] = " ".join(p for p in (asan, env.get("LD_PRELOAD", "")) if p)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "2"
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, HERE, checked, plain], env=env, capture_output=True,
                       text=True, timeout=600)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "bit-identical" in r.stdout
