"""A seeded sweep of launch configurations through the C ABI: random small workloads (detector
sizes, beam centres, cells, tilts, lineshapes, node grids) crossed with random tile shapes,
waves per tile and, where the beam is centred, the mirror folds (left-right; up-down for a
third of the cases, which are then made untilted and centred on the rows).  Every pattern is
compared with the oracle at the pattern tolerances, and every folded pattern with its unfolded
twin (same waves per tile): bit for bit under the left-right fold alone, the computed rows bit
for bit and the rest to float32 rounding under the up-down one.  Eight more cases compare the
atom gradients of the hand-written adjoint with the oracle's."""
import dataclasses
import math
import sys

import numpy as np
import pytest

import gradcheck as GC
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


def random_case(seed):
    rng = np.random.default_rng(1000 + seed)
    tw = int(rng.choice([2, 4, 8, 16, 32]))
    waves = int(rng.choice([0, 1, 2, 4]))
    fold = bool(rng.integers(0, 2))
    width = int(rng.integers(9, 50))
    if fold:
        width = max(tw, (width // tw) * tw)
    height = int(rng.integers(7, 40))
    cx = width / 2.0 if fold else float(rng.uniform(-5.0, width + 5.0))
    cy = float(rng.uniform(0.2, 0.8)) * height
    ls = int(rng.integers(0, 3))
    st, gt = [(3 * DEG, 0.0), (0.0, 2 * DEG), (2 * DEG, 1.5 * DEG)][int(rng.integers(0, 3))]
    edges = rng.uniform(8.0, 13.0, 3)
    angles = rng.uniform(85.0, 100.0, 3) * DEG
    wl = W.small(seed, n_atoms=int(rng.integers(5, 30)), width=width, height=height, center=(cx, cy),
                 cell=W.Cell(*edges, *angles), sigma_theta=st, gamma_theta=gt,
                 g=tuple(float(v) for v in rng.uniform(0.0, 0.04, 3)), n_nodes=int(rng.integers(6, 20)),
                 d_min=float(rng.uniform(4.0, 6.0)), tilt=float(rng.uniform(-30.0, 30.0)) * DEG, lineshape=ls)
    geom = dataclasses.replace(wl.geom, tile_w=tw, tile_waves=waves)
    # drawn last, so that the earlier draws of every seed stay as they were
    updown = bool(rng.integers(0, 3) == 0)
    if updown:
        th = 64 // tw
        h = max(th, (height // th) * th)
        geom = dataclasses.replace(geom, height=h, center_y=h / 2.0, tilt=0.0)
    return dataclasses.replace(wl, geom=geom), int(fold) | (2 if updown else 0)


# seed 7660: an 8x8 detector that none of the 18 reflections reaches (the oracle's image is 0);
# seed 39077: an 8x16 detector under both folds whose mirrored rows differ from the unfolded
# launch's by 3e-6 relative L2 (float32 rounding over 64 pixels)
@pytest.mark.parametrize("seed", list(range(40)) + [7660, 39077])
def test_random_launch_vs_oracle(seed):
    wl, fold = random_case(seed)
    g = wl.geom
    say(f"seed {seed}: {g.width}x{g.height}, centre ({g.center_x:.1f}, {g.center_y:.1f}), tile {g.tile_w} wide, "
        f"waves {g.tile_waves}, mirror bits {fold}, tilt {g.tilt / DEG:.0f} deg, lineshape {wl.dis.lineshape}")
    pipe = Pipeline(wl)
    if pipe.n_hkl == 0:
        pytest.skip("empty reflection list")
    img = pipe.pattern()
    ref = O.pattern(wl, O.prepare(wl, hkl=pipe.hkl.cpu().numpy()))
    got = img.cpu().numpy().astype(np.float64)
    if ref.max() == 0.0:
        say("  no reflection reaches the detector: the image must be 0")
        assert np.all(got == 0.0)
    else:
        r = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        big = ref > 1e-3 * ref.max()
        px = float(np.max(np.abs(got[big] - ref[big]) / ref[big]))
        say(f"  rel-L2 {r:.2e}, per-pixel {px:.2e}")
        assert r <= 1e-4 and px <= 1e-3
    if fold:
        # at the unfolded launch's waves per tile (the library's choice depends on the tile count)
        fg = dataclasses.replace(g, mirror=fold, tile_waves=B.launch_waves(pipe.model.geom))
        folded = Pipeline(dataclasses.replace(wl, geom=fg)).pattern()
        torch.cuda.synchronize()
        if fold & 2:
            th = 64 // g.tile_w
            top = ((g.height // th + 1) // 2) * th
            d = (folded[:top] - img[:top]).abs().max().item()
            assert torch.equal(folded[:top], img[:top]), ("computed rows", top, d)
            low = g.height - top
            assert torch.equal(folded[g.height - low:], torch.flip(folded[:low], [0])), ("mirrored rows", low)
            # the mirrored rows hold the Friedel mates' sums, which round differently from the
            # unfolded launch's: float32 rounding, relative L2 up to a few 1e-6 on small images
            a, b = folded.double().cpu().numpy(), img.double().cpu().numpy()
            assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b), ("folded image", np.linalg.norm(a - b))
        else:
            assert torch.equal(folded, img), ("left-right fold", (folded - img).abs().max().item())


@pytest.mark.parametrize("seed", range(100, 108))
def test_random_launch_gradients_vs_oracle(seed):
    from paper_2608_23245_amd import autograd as AG
    from paper_2608_23245_amd import binding as B
    wl, fold = random_case(seed)
    if fold:
        wl = dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, mirror=fold))
    g = wl.geom
    say(f"gradients seed {seed}: {g.width}x{g.height}, tile {g.tile_w} wide, waves {g.tile_waves}, "
        f"fold {fold}, lineshape {wl.dis.lineshape}")
    eng = AG.PatternEngine(wl)
    if eng.n_hkl == 0:
        pytest.skip("empty reflection list")
    G = np.random.default_rng(seed).normal(size=(g.height, g.width))
    a = wl.atoms
    atoms = eng.atoms(*(torch.as_tensor(v) for v in (a.x, a.y, a.z, a.B, a.occ)))
    F, F2 = B.structure_factors(eng.cell, atoms, eng.hkl)
    eng.plan.run(eng.hkl, F2)
    out, glob, _ = B.pattern_backward(eng.plan, eng.hkl, F, torch.as_tensor(G, dtype=torch.float32).cuda(), atoms)
    ref = O.gradients(wl, O.prepare(wl, hkl=eng.hkl.cpu().numpy(), cull_extinct=False), G)
    for k in ("x", "y", "z", "B", "occ"):
        got = out[k].cpu().numpy().astype(np.float64)
        r = np.asarray(ref["atoms"][k], np.float64)
        rel_l2, elem = GC.errors(got, r, GC.RANDOM_FLOOR)  # a random cotangent G
        assert rel_l2 <= 1e-3 and elem <= 1e-3, (k, rel_l2, elem)
    say("  atom gradients within 1e-3")
