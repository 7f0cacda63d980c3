"""The up-down (Friedel) fold, bit 1 of fdtbx_geometry.mirror, through the C ABI.  With the fibre
normal to the beam and the beam centre at height/2 the folded launches compute the top tile rows
bit for bit as the unfolded ones do and copy them to the mirror rows; the image agrees with the
unfolded one to float32 rounding and with the oracle to the pattern tolerances (pattern and
cylindrical average, every lineshape, an odd number of tile rows, with and without the
left-right fold); gradients agree with the unfolded ones to rounding; a batch of folded models
agrees with its unfolded single runs; and the culling lists cover the launched tiles only."""
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
from paper_2608_23245_amd import autograd as AG  # noqa: E402
from paper_2608_23245_amd import binding as B  # noqa: E402
from paper_2608_23245_amd.batch import BatchEngine  # noqa: E402

DEG = math.pi / 180


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def with_geom(wl, **kw):
    return dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, **kw))


# beams centred on the rows (center_y = height / 2), fibre normal to the beam; heights multiples
# of the tile height; (workload keywords, tile width, mirror bits)
CASES = {
    "voigt_both": (dict(seed=171, width=48, height=32, sigma_theta=3 * DEG, gamma_theta=1 * DEG,
                        g=(0.02, 0.02, 0.0)), 8, 3),
    "voigt_updown_offcentre_x": (dict(seed=172, width=41, height=40, cx=17.3, sigma_theta=2 * DEG,
                                      gamma_theta=2 * DEG), 8, 2),
    "odd_rows_16x4": (dict(seed=173, width=64, height=36, sigma_theta=2 * DEG, gamma_theta=1 * DEG), 16, 3),
    "gaussian_4x16": (dict(seed=174, width=44, height=48, sigma_theta=3 * DEG, lineshape=1,
                           B_axis=(4.0, 9.0, 2.5)), 4, 3),
    "hosemann_odd_rows": (dict(seed=175, width=56, height=24, sigma_theta=3 * DEG, g=(0.03, 0.02, 0.01),
                               lineshape=2), 8, 2),
}


def case(name, mirror=None):
    kw, tw, m = CASES[name]
    kw = dict(kw)
    cx = kw.pop("cx", kw["width"] / 2.0)
    kw["center"] = (cx, kw["height"] / 2.0)
    wl = with_geom(W.small(**kw), tile_w=tw)
    return with_geom(wl, mirror=m if mirror is None else mirror)


def top_rows(wl):
    th = 64 // (wl.geom.tile_w or 8)
    ty = -(-wl.geom.height // th)
    return ((ty + 1) // 2) * th


def check_fold(wl, img_fold, img_full):
    """Computed rows bit-identical, mirror rows copied, the rest to rounding."""
    H = wl.geom.height
    top = top_rows(wl)
    assert torch.equal(img_fold[:top], img_full[:top])
    low = H - top
    assert torch.equal(img_fold[H - low:], torch.flip(img_fold[:low], [0]))
    a, b = img_fold.double().cpu().numpy(), img_full.double().cpu().numpy()
    r = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    big = b > 1e-3 * b.max()
    px = float(np.max(np.abs(a[big] - b[big]) / b[big]))
    say(f"  folded vs unfolded: rel-L2 {r:.2e}, per-pixel {px:.2e}")
    assert b.max() > 0 and r <= 2e-6 and px <= 2e-5


@pytest.mark.parametrize("name", list(CASES))
def test_updown_folded_pattern(name):
    wl = case(name)
    g = wl.geom
    say(f"up-down fold, pattern {name}: {g.width}x{g.height}, tile {g.tile_w}, mirror {g.mirror}")
    fold = Pipeline(wl)
    waves = B.launch_waves(fold.model.geom)
    full = Pipeline(with_geom(wl, mirror=0, tile_waves=waves))
    img_fold, img_full = fold.pattern(), full.pattern()
    torch.cuda.synchronize()
    check_fold(wl, img_fold, img_full)
    ref = O.pattern(wl, O.prepare(wl, hkl=fold.hkl.cpu().numpy()))
    got = img_fold.cpu().numpy().astype(np.float64)
    r = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    big = ref > 1e-3 * ref.max()
    px = float(np.max(np.abs(got[big] - ref[big]) / ref[big]))
    say(f"  folded vs oracle: rel-L2 {r:.2e}, per-pixel {px:.2e}")
    assert r <= 1e-4 and px <= 1e-3

    # the folded launch evaluates the top tile rows (and, with bit 0, the left columns) only
    def count(p):
        _, F2 = p.structure_factors()
        refl, cull = B.reflection_prep(p.model, p.hkl, F2)
        pix, tile = B.pixel_map(p.model.geom)
        off, idx = B.cull(p.model.geom, tile, cull)
        return B.profile(p.model, refl, B.node_table(p.model), pix, tile, off, idx, count=True,
                         order=B.tile_order(p.model.geom, off))
    n_full, n_fold = count(full), count(fold)
    say(f"  evaluations {n_full} unfolded, {n_fold} folded")
    tx, ty = B.tile_grid(fold.model.geom)
    assert 0.2 * n_full < n_fold < n_full
    if ty % 2 == 0 and (tx % 2 == 0 or not g.mirror & 1):
        # no middle row or column: a half (or a quarter) of the tiles, mirror tiles evaluating
        # the same support tests up to rounding
        share = 0.5 if not g.mirror & 1 else 0.25
        assert abs(n_fold - share * n_full) <= 1e-3 * n_full


def cyl_image(wl):
    model = B.make_model(wl)
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    h = torch.from_numpy(np.ascontiguousarray(hkl[~O.extinct_mask(hkl, wl.dis, wl.quad.extinction)])).cuda()
    refl, _ = B.reflection_prep(model, h, torch.ones(h.shape[0], dtype=torch.float32, device="cuda"))
    cull = B.cyl_records(model, h)
    pix, tile = B.pixel_map(model.geom)
    off, idx = B.cull(model.geom, tile, cull)
    return B.profile_cyl(model, refl, B.node_table(model), pix, off, idx, 2e-3, order=B.tile_order(model.geom, off))


@pytest.mark.parametrize("name", ["voigt_both", "odd_rows_16x4"])
def test_updown_folded_cyl(name):
    wl = case(name)
    say(f"up-down fold, cylindrical average {name}")
    waves = B.launch_waves(B.make_model(wl).geom)
    img_fold = cyl_image(wl)
    img_full = cyl_image(with_geom(wl, mirror=0, tile_waves=waves))
    torch.cuda.synchronize()
    check_fold(wl, img_fold, img_full)


@pytest.mark.parametrize("name", ["voigt_both", "odd_rows_16x4", "hosemann_odd_rows"])
def test_updown_folded_gradients(name):
    wl = case(name)
    say(f"up-down fold, gradients {name}")
    G = np.random.default_rng(11).normal(size=(wl.geom.height, wl.geom.width))
    res = []
    for m in (0, wl.geom.mirror):
        eng = AG.PatternEngine(with_geom(wl, mirror=m))
        a = wl.atoms
        atoms = eng.atoms(*(torch.as_tensor(v) for v in (a.x, a.y, a.z, a.B, a.occ)))
        F, F2 = B.structure_factors(eng.cell, atoms, eng.hkl)
        eng.plan.run(eng.hkl, F2)
        out, glob, dF2 = B.pattern_backward(eng.plan, eng.hkl, F, torch.as_tensor(G, dtype=torch.float32).cuda(), atoms)
        res.append(({k: v.cpu().numpy().astype(np.float64) for k, v in out.items()},
                    glob.cpu().numpy().astype(np.float64), dF2.cpu().numpy().astype(np.float64)))
    (o0, g0, f0), (o1, g1, f1) = res
    for k in o0:
        err = np.abs(o1[k] - o0[k]).max() / np.abs(o0[k]).max()
        say(f"  {k}: folded vs unfolded {err:.1e} of the largest")
        assert err <= 1e-4, k
    # per reflection: the mirror rows' weight goes to the Friedel mate, so dL/d|F|^2 of every
    # reflection (not only of each Friedel pair) is the unfolded one
    err = np.abs(f1 - f0).max() / np.abs(f0).max()
    pair = np.abs((f1 + f1[::-1]) - (f0 + f0[::-1])).max() / np.abs(f0).max()
    say(f"  dF2: folded vs unfolded {err:.1e} of the largest (Friedel-pair sums {pair:.1e})")
    assert err <= 1e-4
    # both against the oracle's gradients (relative 1e-3, floor 1e-3 of the group's largest)
    ref = O.gradients(wl, O.prepare(wl, hkl=eng.hkl.cpu().numpy(), cull_extinct=False), G)
    refg = np.asarray([ref["sigma_theta"], ref["gamma_theta"], *ref["N_base"], *ref["g"], *ref["B_axis"]], np.float64)
    groups = [(np.asarray(ref["atoms"][k], np.float64), o0[k], o1[k]) for k in ("x", "y", "z", "B", "occ")]
    for r, a0, a1 in groups + [(refg, g0, g1)]:
        for got in (a0, a1):
            rel_l2, elem = GC.errors(got, r, GC.RANDOM_FLOOR)  # a random cotangent G
            assert rel_l2 <= 1e-3 and elem <= 1e-3, (rel_l2, elem)


def test_updown_folded_batch_matches_unfolded_single_runs():
    wls = [case("voigt_both"), case("odd_rows_16x4"), case("hosemann_odd_rows"), case("gaussian_4x16", mirror=0)]
    be = BatchEngine(wls)
    be.forward()
    torch.cuda.synchronize()
    for m, wl in enumerate(wls):
        ref = Pipeline(with_geom(wl, mirror=0)).pattern().cpu().numpy().astype(np.float64)
        got = be.image_of(m).cpu().numpy().astype(np.float64)
        r = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        say(f"  model {m} (mirror {wl.geom.mirror}): rel-L2 vs unfolded single run {r:.2e}")
        assert r <= 1e-5


@pytest.mark.parametrize("mirror", [2, 3])
def test_updown_culling_lists_cover_the_launched_tiles(mirror):
    wl = case("odd_rows_16x4")
    lists = []
    for m in (0, mirror):
        w = with_geom(wl, mirror=m)
        model = B.make_model(w)
        hkl = O.enumerate_hkl(w.cell, w.quad.d_min, w.quad.d_max)
        h = torch.from_numpy(np.ascontiguousarray(hkl)).cuda()
        _, cull = B.reflection_prep(model, h, torch.ones(h.shape[0], dtype=torch.float32, device="cuda"))
        pix, tile = B.pixel_map(model.geom)
        off, idx = B.cull(model.geom, tile, cull)
        lists.append((off.cpu().numpy(), idx.cpu().numpy()))
    (o0, i0), (o1, i1) = lists
    tx, ty = B.tile_grid(B.make_model(wl).geom)
    lcols = (tx + 1) // 2 if mirror & 1 else tx
    lrows = (ty + 1) // 2
    for t in range(tx * ty):
        got = i1[o1[t]:o1[t + 1]]
        if t % tx < lcols and t // tx < lrows:
            assert np.array_equal(got, i0[o0[t]:o0[t + 1]]), t
        else:
            assert got.size == 0, t
