"""Degenerate inputs through the C ABI: an empty resolution shell, a reflection list that the
extinction cull empties, a model without atoms, and the smallest and largest node grids.
Empty inputs are valid calls: images come out zero, culling lists empty, gradients zero."""
import dataclasses
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

from paper_2608_23245_amd import Pipeline  # noqa: E402
from paper_2608_23245_amd import binding as B  # noqa: E402

DEG = math.pi / 180


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _zero_everything(wl):
    """Forward, culling, splat, cylindrical average and backward of a workload whose
    reflection list is empty."""
    pipe = Pipeline(wl)
    assert pipe.n_hkl == 0
    img = pipe.pattern()
    torch.cuda.synchronize()
    assert img.shape == (wl.geom.height, wl.geom.width)
    assert torch.count_nonzero(img).item() == 0
    model = pipe.model
    F, F2 = B.structure_factors(pipe.cell, pipe.atoms, pipe.hkl)
    assert F.shape == (0, 2) and F2.shape == (0,)
    refl, cull = B.reflection_prep(model, pipe.hkl, F2)
    nodes = B.node_table(model)
    pix, tile = B.pixel_map(model.geom)
    off, idx = B.cull(model.geom, tile, cull)
    assert idx.shape[0] == 0 and torch.count_nonzero(off).item() == 0
    assert torch.count_nonzero(B.splat(model, pipe.hkl, refl, nodes, 2, 8)).item() == 0
    cyl = B.cyl_records(model, pipe.hkl)
    off_c, idx_c = B.cull(model.geom, tile, cyl)
    assert idx_c.shape[0] == 0 and torch.count_nonzero(off_c).item() == 0
    # the per-tile kernels read no record and no list entry when every list is empty
    # (one-element stand-ins give them valid pointers; torch's empty tensors have none)
    refl1 = torch.zeros((1, B.REFL_FLOATS), dtype=torch.float32, device="cuda")
    idx1 = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert torch.count_nonzero(B.profile(model, refl1, nodes, pix, tile, off, idx1)).item() == 0
    assert B.profile(model, refl1, nodes, pix, tile, off, idx1, count=True) == 0
    assert torch.count_nonzero(B.profile_cyl(model, refl1, nodes, pix, off_c, idx1, 2e-3)).item() == 0
    G = torch.ones_like(img)
    out, glob, dF2 = B.pattern_backward(pipe.plan, pipe.hkl, F, G, pipe.atoms)
    torch.cuda.synchronize()
    assert dF2.shape == (0,)
    assert np.all(glob.cpu().numpy() == 0.0)
    for k, v in out.items():
        assert v.shape == (wl.atoms.x.shape[0],) and torch.count_nonzero(v).item() == 0, k


def test_empty_resolution_shell():
    """d_min above the longest cell edge: no reflection lies in the shell."""
    wl = W.small(61, width=13, height=11, d_min=14.0)
    say("empty shell")
    assert O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max).shape[0] == 0
    _zero_everything(wl)


def test_empty_resolution_shell_folded_16x4():
    """The same with the mirror fold and 16 x 4 tiles of 4 waves."""
    wl = W.small(61, width=32, height=11, d_min=14.0, center=(16.0, 5.5))
    wl = dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, tile_w=16, mirror=1, tile_waves=4))
    say("empty shell, folded")
    _zero_everything(wl)


def test_every_reflection_extinct():
    """Disorder so strong that the extinction cull removes every reflection of a
    high-resolution shell (2.5 to 3 A)."""
    wl = W.small(62, width=10, height=12, g=(0.99, 0.99, 0.99), d_min=2.5)
    wl = dataclasses.replace(wl, quad=dataclasses.replace(wl.quad, d_max=3.0))
    say("all extinct")
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    assert hkl.shape[0] > 0 and np.all(O.extinct_mask(hkl, wl.dis, wl.quad.extinction))
    _zero_everything(wl)


def test_model_without_atoms():
    """No atoms: F = 0, so the pattern is zero although the reflections and their supports
    are all there."""
    wl = W.small(63, width=12, height=9)
    say("no atoms")
    pipe = Pipeline(wl)
    assert pipe.n_hkl > 0
    empty = {k: v[:0].contiguous() for k, v in pipe.atoms.items() if k != "ff"}
    empty["ff"] = pipe.atoms["ff"]
    F, F2 = B.structure_factors(pipe.cell, empty, pipe.hkl)
    torch.cuda.synchronize()
    assert torch.count_nonzero(F).item() == 0 and torch.count_nonzero(F2).item() == 0
    img = pipe.pattern(F2)
    torch.cuda.synchronize()
    assert torch.count_nonzero(img).item() == 0


@pytest.mark.parametrize("n_nodes", [1, 2, 256])
def test_node_grid_extremes_vs_oracle(n_nodes):
    """One node (the shell quadrature degenerates to the node at D), two, and the largest
    grid the library accepts."""
    wl = W.small(64 + n_nodes, width=17, height=14, sigma_theta=3 * DEG, gamma_theta=1 * DEG, n_nodes=n_nodes,
                 d_min=5.5, g=(0.02, 0.02, 0.0))
    say(f"node grid {n_nodes}")
    pipe = Pipeline(wl)
    img = pipe.pattern().cpu().numpy().astype(np.float64)
    ref = O.pattern(wl, O.prepare(wl, hkl=pipe.hkl.cpu().numpy()))
    assert ref.max() > 0
    r = float(np.linalg.norm(img - ref) / np.linalg.norm(ref))
    big = ref > 1e-3 * ref.max()
    px = float(np.max(np.abs(img[big] - ref[big]) / ref[big]))
    say(f"  rel-L2 {r:.2e}, per-pixel {px:.2e} over {int(big.sum())} px")
    assert r <= 1e-4 and px <= 1e-3


def test_negative_sizes_are_rejected():
    wl = W.config0()
    model = B.make_model(wl)
    z = torch.zeros(16, dtype=torch.float32, device="cuda")
    L = B.lib()
    rc = L.fdtbx_reflection_prep(B.ctypes.byref(model), B._ptr(z), -1, B._ptr(z), B._ptr(z), B._ptr(z), None)
    assert rc == -1
    assert L.fdtbx_pattern_workspace(B.ctypes.byref(model), -1, 0) == 0
