"""Parity of the forward splat (fdtbx_splat, through the C ABI) with the FP64 oracle's splat
on the same deterministic sampling: images to the pattern tolerances (relative L2 <= 1e-4,
per-pixel <= 1e-3 over pixels above 1e-3 of the maximum), and the number of (sample, node)
pairs inside the support equal up to float32 boundary decisions."""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2608_23245_amd import binding as B  # noqa: E402

DEG = math.pi / 180


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_splat(wl, hkl, n_r, n_s):
    model = B.make_model(wl)
    h = torch.from_numpy(np.ascontiguousarray(hkl, dtype=np.int32)).cuda()
    F = O.structure_factors_c(hkl, wl.cell, wl.atoms)
    F2 = torch.as_tensor((F.real ** 2 + F.imag ** 2).astype(np.float32)).cuda()
    refl, _ = B.reflection_prep(model, h, F2)
    nodes = B.node_table(model)
    img = B.splat(model, h, refl, nodes, n_r, n_s).cpu().numpy().astype(np.float64)
    cnt = B.splat(model, h, refl, nodes, n_r, n_s, count=True)
    return img, cnt, F


def check(img, ref, tag):
    assert ref.max() > 0, f"{tag}: empty reference"
    r = float(np.linalg.norm(img - ref) / np.linalg.norm(ref))
    big = ref > 1e-3 * ref.max()
    px = float(np.max(np.abs(img[big] - ref[big]) / ref[big]))
    say(f"{tag}: rel-L2 {r:.2e}, per-pixel {px:.2e} over {int(big.sum())} px")
    assert r <= 1e-4 and px <= 1e-3, (tag, r, px)


CASES = {
    "config0": (None, 4, 16),
    "voigt_tilted": (dict(seed=71, width=40, height=36, sigma_theta=2 * DEG, gamma_theta=1 * DEG, g=(0.02, 0.02, 0.0),
                          tilt=22 * DEG, center=(19.4, 15.2)), 4, 24),
    "gaussian_lineshape": (dict(seed=72, width=32, height=30, sigma_theta=3 * DEG, lineshape=1, B_axis=(4.0, 9.0, 2.5)), 3, 20),
    "hosemann_lineshape": (dict(seed=73, width=30, height=34, sigma_theta=2 * DEG, gamma_theta=0.5 * DEG, lineshape=2,
                                g=(0.03, 0.02, 0.01)), 3, 20),
    "ragged_samples": (dict(seed=74, width=25, height=27, sigma_theta=4 * DEG, n_nodes=10), 5, 13),
    "detector_tilted": (dict(seed=75, width=34, height=30, sigma_theta=2 * DEG, gamma_theta=1 * DEG, tilt=10 * DEG,
                             det_tilt=25 * DEG, center=(16.2, 13.9)), 4, 20),
}


@pytest.mark.parametrize("name", list(CASES))
def test_splat_vs_oracle(name):
    kw, n_r, n_s = CASES[name]
    wl = W.config0() if kw is None else W.small(**kw)
    say(f"splat {name}: n_r {n_r}, n_s {n_s}")
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    hkl = np.ascontiguousarray(hkl[~O.extinct_mask(hkl, wl.dis, wl.quad.extinction)])
    img, cnt, F = gpu_splat(wl, hkl, n_r, n_s)
    P = O.prepare(wl, hkl=hkl, F=F, cull_extinct=False)
    ref, n_ref = O.splat(wl, P, n_r, n_s, count=True)
    check(img, ref, name)
    say(f"  evaluations: GPU {cnt}, oracle {n_ref}")
    assert abs(cnt - n_ref) <= 1e-5 * n_ref + 2


def test_splat_medium_reflection_subset():
    """The medium workload at full detector size for 150 of its reflections (seeded pick)."""
    wl = W.config1()
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    hkl = hkl[~O.extinct_mask(hkl, wl.dis, wl.quad.extinction)]
    pick = np.sort(np.random.default_rng(5).choice(hkl.shape[0], 150, replace=False))
    hkl = np.ascontiguousarray(hkl[pick])
    say("splat medium, 150 reflections, n_r 3, n_s 16")
    img, cnt, F = gpu_splat(wl, hkl, 3, 16)
    P = O.prepare(wl, hkl=hkl, F=F, cull_extinct=False)
    ref, n_ref = O.splat(wl, P, 3, 16, count=True)
    check(img, ref, "medium subset")
    assert abs(cnt - n_ref) <= 1e-5 * n_ref + 2


def test_splat_argument_checks():
    wl = W.config0()
    model = B.make_model(wl)
    h = torch.zeros((1, 3), dtype=torch.int32, device="cuda")
    r = torch.zeros((1, B.REFL_FLOATS), dtype=torch.float32, device="cuda")
    with pytest.raises(B.FdtbxError):
        B.splat(model, h, r, r, 0, 16)
    with pytest.raises(B.FdtbxError):
        B.splat(model, h, r, r, 4, 5000)
