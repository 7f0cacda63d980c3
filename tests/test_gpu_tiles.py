"""Pixel-tile shapes other than 8 x 8 (fdtbx_geometry.tile_w) and the tile-shape tuner,
through the C ABI: pixel map, tile boxes and culling lists bit-exact against the oracle's
tiles of the same shape; patterns, cylindrical averages and gradients to the parity
tolerances against the oracle; batches whose models run in different shapes equal to
their single runs; the tuner picks one of its candidates by timing their launches and
caches the choice, and the batch tuner keeps the batch engine of the fastest shape."""
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
from paper_2608_23245_amd.autotune import TileTuner  # noqa: E402
from paper_2608_23245_amd.batch import BatchEngine  # noqa: E402

DEG = math.pi / 180
SHAPES = [2, 4, 16, 32]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def shaped(wl, tw):
    return dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, tile_w=tw))


def check_pattern(img, ref, tag):
    img = np.asarray(img, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert ref.max() > 0, f"{tag}: the reference image is empty"
    r = float(np.linalg.norm(img - ref) / np.linalg.norm(ref))
    big = ref > 1e-3 * ref.max()
    px = float(np.max(np.abs(img[big] - ref[big]) / ref[big]))
    say(f"{tag}: rel-L2 {r:.2e}, max per-pixel rel {px:.2e} over {int(big.sum())} px")
    assert r <= 1e-4 and px <= 1e-3, (tag, r, px)


CASES = {
    "ragged": dict(seed=121, width=37, height=23, center=(17.7, 10.2), sigma_theta=3 * DEG, gamma_theta=1 * DEG,
                   g=(0.02, 0.02, 0.0)),
    "tilted": dict(seed=122, width=26, height=35, center=(13.0, 19.4), tilt=22 * DEG, sigma_theta=2 * DEG,
                   gamma_theta=1 * DEG),
    "hosemann": dict(seed=123, width=29, height=21, sigma_theta=3 * DEG, g=(0.03, 0.02, 0.01), lineshape=2),
}


def _hkl(wl):
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    return np.ascontiguousarray(hkl[~O.extinct_mask(hkl, wl.dis, wl.quad.extinction)])


@pytest.mark.parametrize("tw", SHAPES)
@pytest.mark.parametrize("name", ["ragged", "tilted"])
def test_pixel_map_tiles_and_lists_bit_exact(name, tw):
    wl = shaped(W.small(**CASES[name]), tw)
    th = 64 // tw
    say(f"tiles {tw}x{th} {name}")
    model = B.make_model(wl)
    tx, ty = B.tile_grid(model.geom)
    assert (tx, ty) == (-(-wl.geom.width // tw), -(-wl.geom.height // th))
    pix, tile = B.pixel_map(model.geom)
    R, Z = O.pixel_rz(wl.geom)
    p = pix.cpu().numpy()
    assert np.array_equal(p[..., 0], R) and np.array_equal(p[..., 1], Z)
    assert np.array_equal(tile.cpu().numpy()[:, :6], O.tile_boxes(wl.geom, tw, th).reshape(-1, 6))
    hkl = _hkl(wl)
    _, cull = B.reflection_prep(model, torch.from_numpy(hkl).cuda(),
                                torch.ones(hkl.shape[0], dtype=torch.float32, device="cuda"))
    off, idx = B.cull(model.geom, tile, cull)
    off, idx = off.cpu().numpy(), idx.cpu().numpy()
    ref = O.culling_lists(wl, hkl, tw, th)
    assert len(ref) == tx * ty
    for t, lst in enumerate(ref):
        assert np.array_equal(idx[off[t]:off[t + 1]], lst), t
    o = B.tile_order(model.geom, torch.from_numpy(off).cuda()).cpu().numpy()
    assert np.array_equal(np.sort(o[o >= 0]), np.arange(tx * ty))


@pytest.mark.parametrize("tw", SHAPES)
@pytest.mark.parametrize("name", list(CASES))
def test_pattern_vs_oracle(name, tw):
    wl = shaped(W.small(**CASES[name]), tw)
    pipe = Pipeline(wl)
    img = pipe.pattern().cpu().numpy()
    ref = O.pattern(wl, O.prepare(wl, hkl=pipe.hkl.cpu().numpy()))
    check_pattern(img, ref, f"pattern {name}, tiles {tw}x{64 // tw}")


@pytest.mark.parametrize("tw,waves", [(4, 0), (16, 0), (8, 1), (8, 2)])
def test_cyl_vs_oracle(tw, waves):
    wl = shaped(W.small(**CASES["ragged"]), tw)
    wl = dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, tile_waves=waves))
    arc = 2e-3
    hkl = _hkl(wl)
    model = B.make_model(wl)
    h = torch.from_numpy(hkl).cuda()
    F = O.structure_factors_c(hkl, wl.cell, wl.atoms)
    F2 = torch.as_tensor((F.real ** 2 + F.imag ** 2).astype(np.float32)).cuda()
    refl, _ = B.reflection_prep(model, h, F2)
    cull = B.cyl_records(model, h)
    nodes = B.node_table(model)
    pix, tile = B.pixel_map(model.geom)
    off, idx = B.cull(model.geom, tile, cull)
    lists = O.culling_lists(wl, hkl, tw, 64 // tw, boxes=O.cyl_boxes(wl, hkl))
    o, ix = off.cpu().numpy(), idx.cpu().numpy()
    for t, lst in enumerate(lists):
        assert np.array_equal(ix[o[t]:o[t + 1]], lst), t
    order = B.tile_order(model.geom, off)
    img = B.profile_cyl(model, refl, nodes, pix, off, idx, arc, order=order).cpu().numpy()
    P = O.prepare(wl, hkl=hkl, F=F, cull_extinct=False)
    R, Z = O.pixel_rz(wl.geom)
    check_pattern(img, O.cyl_at(P, R, Z, arc).reshape(img.shape), f"cylindrical average, tiles {tw}x{64 // tw}, waves {waves}")


@pytest.mark.parametrize("tw", [4, 32])
def test_adjoint_vs_oracle(tw):
    wl = shaped(W.small(126, n_atoms=30, width=19, height=22, sigma_theta=3 * DEG, gamma_theta=1 * DEG,
                        g=(0.03, 0.02, 0.01)), tw)
    say(f"adjoint, tiles {tw}x{64 // tw}")
    G = np.random.default_rng(8).normal(size=(wl.geom.height, wl.geom.width))
    eng = AG.PatternEngine(wl)
    a = wl.atoms
    atoms = eng.atoms(*(torch.as_tensor(v) for v in (a.x, a.y, a.z, a.B, a.occ)))
    F, F2 = B.structure_factors(eng.cell, atoms, eng.hkl)
    eng.plan.run(eng.hkl, F2)
    out, glob, _ = B.pattern_backward(eng.plan, eng.hkl, F, torch.as_tensor(G, dtype=torch.float32).cuda(), atoms)
    P = O.prepare(wl, hkl=eng.hkl.cpu().numpy(), cull_extinct=False)
    ref = O.gradients(wl, P, G)
    for k in ("x", "y", "z", "B", "occ"):
        got = out[k].cpu().numpy().astype(np.float64)
        r = np.asarray(ref["atoms"][k], np.float64)
        err = np.abs(got - r) / np.maximum(np.abs(r), GC.RANDOM_FLOOR * np.abs(r).max())
        say(f"  {k}: max rel err {err.max():.2e}")
        assert err.max() <= 1e-3, (k, err.max())


def test_batch_with_mixed_shapes_matches_single_runs():
    wls = [shaped(W.small(131, n_atoms=20, width=24, height=20, sigma_theta=3 * DEG, gamma_theta=1 * DEG), 4),
           shaped(W.small(132, n_atoms=25, width=17, height=29, sigma_theta=2 * DEG, lineshape=1), 16),
           shaped(W.small(133, n_atoms=15, width=33, height=12, sigma_theta=4 * DEG, g=(0.03, 0.0, 0.0),
                          lineshape=2), 32),
           W.small(134, n_atoms=10, width=20, height=20, sigma_theta=2 * DEG, gamma_theta=2 * DEG)]
    be = BatchEngine(wls)
    assert be.tile_w == [4, 16, 32, 8]
    be.forward()
    torch.cuda.synchronize()
    for m, wl in enumerate(wls):
        ref = Pipeline(shaped(wl, 0)).pattern().cpu().numpy().astype(np.float64)
        got = be.image_of(m).cpu().numpy().astype(np.float64)
        r = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        say(f"  model {m} ({be.tile_w[m]} wide tiles): rel-L2 vs single 8x8 run {r:.2e}")
        assert r <= 1e-5


def test_tuner_choice_and_cache():
    wl = W.config0()
    pipe = Pipeline(wl)
    _, F2 = pipe.structure_factors()
    model = pipe.model
    refl, cull = B.reflection_prep(model, pipe.hkl, F2)
    nodes = B.node_table(model)
    tuner = TileTuner(candidates=(4, 8, 16))
    tw = tuner.choose(model, refl, nodes, cull)
    best, times = tuner.cached(model, refl.shape[0])
    say(f"tuner: {times} -> {tw}")
    assert tw == best and tw in (4, 8, 16) and set(times) == {4, 8, 16}
    assert all(t > 0 for t in times.values())
    # an equal model with another tile width is the same cache entry
    other = B.Model.from_buffer_copy(model)
    other.geom.tile_w = 16
    assert tuner.cached(other, refl.shape[0]) == (best, times)
    # the default shape wins unless another beats it by the margin
    if tw != 8:
        assert times[tw] <= (1 - tuner.margin) * times[8]
    assert TileTuner(min_tiles=10 ** 6).choose(model, refl, nodes, cull) == 8


def test_tune_batch_keeps_the_fastest_engine():
    from paper_2608_23245_amd.autotune import tune_batch
    wls = [W.small(151, n_atoms=20, width=64, height=48, sigma_theta=3 * DEG, gamma_theta=1 * DEG),
           W.small(152, n_atoms=25, width=40, height=72, sigma_theta=2 * DEG, lineshape=1),
           W.small(153, n_atoms=15, width=56, height=56, sigma_theta=4 * DEG, g=(0.03, 0.0, 0.0))]
    be, times = tune_batch(wls, candidates=(16, 8, 4), reps=2)
    say(f"batch tile tuning: {times} -> {be.tile_w}")
    assert set(times) == {4, 8, 16} and all(t > 0 for t in times.values())
    tw = be.tile_w[0]
    assert be.tile_w == [tw] * len(wls)
    if tw != 8:
        assert times[tw] < 0.98 * times[8] and times[tw] == min(times.values())
    else:
        assert min(times[4], times[16]) >= 0.98 * times[8]
    be.forward()
    torch.cuda.synchronize()
    for m, wl in enumerate(wls):
        ref = Pipeline(wl).pattern().cpu().numpy().astype(np.float64)
        got = be.image_of(m).cpu().numpy().astype(np.float64)
        assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref), m


@pytest.mark.parametrize("waves", [1, 2, 4])
@pytest.mark.parametrize("name", ["ragged", "hosemann"])
def test_tile_waves_pattern_and_counts(name, waves):
    """Waves per tile (fdtbx_geometry.tile_waves): the same image to float32 summation order
    and the same number of support-passing evaluations for 1, 2 and 4 waves."""
    base = W.small(**CASES[name])
    wl = dataclasses.replace(base, geom=dataclasses.replace(base.geom, tile_waves=waves))
    pipe = Pipeline(wl)
    img = pipe.pattern().cpu().numpy()
    ref = O.pattern(wl, O.prepare(wl, hkl=pipe.hkl.cpu().numpy()))
    check_pattern(img, ref, f"pattern {name}, {waves} waves per tile")
    counts = []
    for w in (1, waves):
        m = B.make_model(dataclasses.replace(base, geom=dataclasses.replace(base.geom, tile_waves=w)))
        _, F2 = pipe.structure_factors()
        refl, cull = B.reflection_prep(m, pipe.hkl, F2)
        pix, tile = B.pixel_map(m.geom)
        off, idx = B.cull(m.geom, tile, cull)
        counts.append(B.profile(m, refl, B.node_table(m), pix, tile, off, idx, count=True))
    assert counts[0] == counts[1] > 0


@pytest.mark.parametrize("waves", [1, 2, 4])
def test_tile_waves_adjoint_vs_oracle(waves):
    wl = W.small(127, n_atoms=30, width=23, height=18, sigma_theta=3 * DEG, gamma_theta=1 * DEG, g=(0.03, 0.02, 0.01))
    wl = dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, tile_waves=waves))
    say(f"adjoint, {waves} waves per tile")
    G = np.random.default_rng(10).normal(size=(wl.geom.height, wl.geom.width))
    eng = AG.PatternEngine(wl)
    a = wl.atoms
    atoms = eng.atoms(*(torch.as_tensor(v) for v in (a.x, a.y, a.z, a.B, a.occ)))
    F, F2 = B.structure_factors(eng.cell, atoms, eng.hkl)
    eng.plan.run(eng.hkl, F2)
    out, glob, _ = B.pattern_backward(eng.plan, eng.hkl, F, torch.as_tensor(G, dtype=torch.float32).cuda(), atoms)
    P = O.prepare(wl, hkl=eng.hkl.cpu().numpy(), cull_extinct=False)
    ref = O.gradients(wl, P, G)
    for k in ("x", "y", "z", "B", "occ"):
        got = out[k].cpu().numpy().astype(np.float64)
        r = np.asarray(ref["atoms"][k], np.float64)
        err = np.abs(got - r) / np.maximum(np.abs(r), GC.RANDOM_FLOOR * np.abs(r).max())
        assert err.max() <= 1e-3, (k, err.max())
    rg = np.array([ref["sigma_theta"], ref["gamma_theta"], *ref["N_base"], *ref["g"], *ref["B_axis"]], np.float64)
    gg = glob.cpu().numpy()[:rg.size]
    err = np.abs(gg - rg) / np.maximum(np.abs(rg), GC.RANDOM_FLOOR * np.abs(rg).max())
    say(f"  globals: max rel err {err.max():.2e}")
    assert err.max() <= 1e-3


def test_library_choice_of_waves():
    """tile_waves = 0: 4 waves when the launched tiles fit in eight rounds of one-wave
    workgroups (32 per compute unit), else 2."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for width, height, mirror in [(64, 64, 0), (1024, 1024, 0), (2048, 2048, 1), (2048, 2048, 0), (4096, 4096, 0)]:
        g = B.Geometry(1.0, 100.0, 0.1, width, height, width / 2.0, height / 2.0, 0.0, 8, mirror, 0)
        tx, ty = B.tile_grid(g)
        n = ((tx + 1) // 2 if mirror else tx) * ty
        want = 4 if n <= 8 * 32 * cus else 2
        assert B.launch_waves(g) == want, (width, mirror, n)
