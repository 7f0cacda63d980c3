"""The balanced forward launch (fdtbx_profile_balanced): the same image as the per-tile launch
to float32 rounding and as the oracle to the pattern tolerances, for every lineshape, skewed
cells, tilted fibres, ragged and tiny detectors and unit sizes from 1 pair to more than a
tile's list; the same bits on every run, with or without a launch order; computed rows of a
folded launch bit-identical to the unfolded launch's at the same unit size; and the host
checks of its workspace and arguments."""
import ctypes
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

from paper_2608_23245_amd import atoms_to_device  # noqa: E402
from paper_2608_23245_amd import binding as B  # noqa: E402

DEG = math.pi / 180

CASES = {
    "ragged": dict(seed=41, width=21, height=19, center=(9.7, 10.2)),
    "skew_voigt": dict(seed=42, width=24, height=24, cell=W.Cell(9.5, 12.0, 14.0, 80 * DEG, 100 * DEG, 110 * DEG),
                       sigma_theta=2 * DEG, gamma_theta=1.5 * DEG),
    "lorentz_tall": dict(seed=43, width=17, height=33, sigma_theta=0.0, gamma_theta=2.5 * DEG),
    "tiny_det": dict(seed=44, width=1, height=3, center=(-8.0, 1.5)),
    "tilted": dict(seed=45, width=26, height=22, center=(13.0, 9.4), tilt=22 * DEG, sigma_theta=2 * DEG,
                   gamma_theta=1 * DEG),
    "gaussian": dict(seed=46, width=22, height=20, sigma_theta=2 * DEG, gamma_theta=1 * DEG, g=(0.03, 0.02, 0.01),
                     lineshape=1, B_axis=(4.0, 9.0, 2.5)),
    "hosemann": dict(seed=47, width=23, height=21, sigma_theta=3 * DEG, g=(0.03, 0.02, 0.01), lineshape=2),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def with_geom(wl, **kw):
    return dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, **kw))


def inputs(wl):
    """Reflection records, node table, pixel map, culling lists and launch order of wl."""
    model = B.make_model(wl)
    ext = (wl.dis.g[0], wl.dis.g[1], wl.dis.g[2], wl.quad.extinction)
    hkl = B.enumerate_hkl(model.cell, wl.quad.d_min, wl.quad.d_max, extinction=ext)
    _, F2 = B.structure_factors(model.cell, atoms_to_device(wl.atoms), hkl, want_F=False)
    refl, cull = B.reflection_prep(model, hkl, F2)
    nodes = B.node_table(model)
    pix, tile = B.pixel_map(model.geom)
    off, idx = B.cull(model.geom, tile, cull)
    order = B.tile_order(model.geom, off)
    return model, hkl, F2, refl, nodes, pix, tile, off, idx, order


def oracle_image(wl, hkl, F2):
    F = np.sqrt(F2.cpu().numpy().astype(np.float64)).astype(complex)
    P = O.prepare(wl, hkl=hkl.cpu().numpy(), F=F, cull_extinct=False)
    return O.pattern(wl, P)


def check(img, ref, tag, rel=1e-4, px_tol=1e-3):
    img = np.asarray(img, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert ref.max() > 0
    r = float(np.linalg.norm(img - ref) / np.linalg.norm(ref))
    big = ref > 1e-3 * ref.max()
    px = float(np.max(np.abs(img[big] - ref[big]) / ref[big]))
    say(f"  {tag}: rel-L2 {r:.2e}, per-pixel {px:.2e}")
    assert r <= rel and px <= px_tol, (tag, r, px)


@pytest.mark.parametrize("name", list(CASES))
def test_balanced_matches_per_tile_and_oracle(name):
    wl = W.small(**CASES[name])
    say(f"balanced launch, {name} ({wl.geom.width}x{wl.geom.height})")
    model, hkl, F2, refl, nodes, pix, tile, off, idx, order = inputs(wl)
    if hkl.shape[0] == 0 or idx.numel() == 0:
        pytest.skip("no reflection reaches the detector")
    lens = (off[1:] - off[:-1]).cpu().numpy()
    per_tile = B.profile(model, refl, nodes, pix, tile, off, idx, order=order).cpu().numpy()
    ref = oracle_image(wl, hkl, F2)
    check(per_tile, ref, "per-tile launch vs oracle")
    for u in (0, 1, 5, 64, int(lens.max()) + 7):
        m = B.make_model(with_geom(wl, unit_pairs=u))
        img = B.profile_balanced(m, refl, nodes, pix, tile, off, idx, order=order).cpu().numpy()
        check(img, ref, f"balanced, {u or B.unit_pairs(idx.numel())} pairs per unit, vs oracle")
        # the per-tile launch sums the same terms, grouped by wave chunk instead of by unit
        scale = np.abs(per_tile).max()
        assert np.max(np.abs(img - per_tile)) <= 2e-6 * scale, (u, float(np.max(np.abs(img - per_tile)) / scale))
        # a tile without pairs comes out zero
        tx, ty = B.tile_grid(model.geom)
        tw = model.geom.tile_w or 8
        for t in np.nonzero(lens == 0)[0][:8]:
            i0, j0 = (t % tx) * tw, (t // tx) * (64 // tw)
            assert np.all(img[j0:j0 + 64 // tw, i0:i0 + tw] == 0.0)


def medium_crop(mirror=0, tile_w=16):
    wl = W.config1()
    return with_geom(wl, width=128, height=128, center_x=64.0, center_y=64.0, tile_w=tile_w, mirror=mirror)


def test_balanced_repeats_and_ignores_the_launch_order():
    """The medium model on a 128x128 crop, 3 units' sizes: three runs give the same bits, and
    the launch without an order (tiles in index order, other queues) gives the same bits too:
    a tile's units and the order of their sum do not depend on which wave ran them."""
    wl = medium_crop()
    model, hkl, F2, refl, nodes, pix, tile, off, idx, order = inputs(wl)
    say(f"balanced launch, medium 128x128 crop: {idx.numel()} pairs")
    for u in (0, 17, 300):
        m = B.make_model(with_geom(wl, unit_pairs=u))
        runs = [B.profile_balanced(m, refl, nodes, pix, tile, off, idx, order=order) for _ in range(3)]
        runs.append(B.profile_balanced(m, refl, nodes, pix, tile, off, idx, order=None))
        torch.cuda.synchronize()
        for r in runs[1:]:
            assert torch.equal(r, runs[0]), u
        assert runs[0].max().item() > 0


@pytest.mark.parametrize("mirror", [1, 2, 3])
def test_balanced_folded_rows_match_unfolded(mirror):
    """Folded and unfolded launches of the crop at the same pairs per unit: the computed rows
    (all of them under the left-right fold) are bit-identical."""
    wl = medium_crop()
    full = inputs(wl)
    u = B.unit_pairs(full[8].numel())
    fw = with_geom(wl, mirror=mirror, unit_pairs=u)
    fold = inputs(fw)
    say(f"balanced launch, fold {mirror}: {fold[8].numel()} of {full[8].numel()} pairs, {u} per unit")
    m0 = B.make_model(with_geom(wl, unit_pairs=u))
    img0 = B.profile_balanced(m0, *full[3:9], order=full[9])
    img1 = B.profile_balanced(fold[0], *fold[3:9], order=fold[9])
    torch.cuda.synchronize()
    top = 64 if mirror & 2 else 128
    assert torch.equal(img1[:top], img0[:top])
    if mirror & 2:
        assert torch.equal(img1[64:], torch.flip(img1[:64], [0]))
        a, b = img1.double().cpu().numpy(), img0.double().cpu().numpy()
        assert np.linalg.norm(a - b) <= 2e-6 * np.linalg.norm(b)


def test_balanced_host_checks():
    """Workspace below the size query, negative capacity or unit size, null pointers: refused
    on the host, before any launch."""
    wl = W.small(48, width=12, height=10)
    model, hkl, F2, refl, nodes, pix, tile, off, idx, order = inputs(wl)
    L = B.lib()
    cap = int(idx.numel())
    wsb = L.fdtbx_profile_balanced_workspace(ctypes.byref(model), cap)
    assert wsb > 0
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    img = torch.full((wl.geom.height, wl.geom.width), 7.0, device="cuda")
    args = [B._ptr(refl), B._ptr(nodes), B._ptr(pix), B._ptr(tile), B._ptr(off), B._ptr(idx), B._ptr(order), cap,
            B._ptr(img)]
    assert L.fdtbx_profile_balanced(ctypes.byref(model), *args, B._ptr(ws), wsb - 1, B._stream()) == -3
    bad = list(args)
    bad[7] = -1
    assert L.fdtbx_profile_balanced(ctypes.byref(model), *bad, B._ptr(ws), wsb, B._stream()) == -1
    assert L.fdtbx_profile_balanced(ctypes.byref(model), *args, None, wsb, B._stream()) == -1
    m = B.make_model(with_geom(wl, unit_pairs=-2))
    assert L.fdtbx_profile_balanced_workspace(ctypes.byref(m), cap) == 0
    assert L.fdtbx_profile_balanced(ctypes.byref(m), *args, B._ptr(ws), wsb, B._stream()) == -1
    torch.cuda.synchronize()
    assert torch.all(img == 7.0)  # nothing was launched
    assert B.unit_pairs(0) == 32 and B.unit_pairs(-1) == 0 and B.unit_pairs((1 << 19) * 100 + 1) == 101


@pytest.mark.parametrize("name,mirror", [("skew_voigt", 0), ("hosemann", 0), ("medium_crop", 3)])
def test_balanced_adjoint_matches_per_tile(name, mirror):
    """fdtbx_profile_adjoint_balanced over the units of a balanced forward: every pair's sums
    are computed as in the per-tile adjoint, so the per-reflection binary64 sums agree to the
    rounding of their (atomic) addition order."""
    wl = medium_crop(mirror=mirror) if name == "medium_crop" else W.small(**CASES[name])
    model, hkl, F2, refl, nodes, pix, tile, off, idx, order = inputs(wl)
    G = torch.as_tensor(np.random.default_rng(9).normal(size=(wl.geom.height, wl.geom.width)),
                        dtype=torch.float32).cuda().contiguous()
    say(f"balanced adjoint, {name}: {idx.numel()} pairs")
    ref = B.profile_adjoint(model, refl, nodes, pix, tile, off, idx, G, order=order)
    for u in (0, 7):
        m = B.make_model(with_geom(wl, unit_pairs=u))
        ws = B.balanced_workspace(m, int(idx.numel()))
        B.profile_balanced(m, refl, nodes, pix, tile, off, idx, order=order, ws=ws)
        got = B.profile_adjoint_balanced(m, refl, nodes, pix, tile, off, idx, G, ws, order=order)
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        scale = np.abs(r).max(axis=0)
        assert np.all(scale > 0)
        err = float(np.max(np.abs(g - r) / scale))
        say(f"  {u or 'default'} pairs per unit: max difference {err:.1e} of each sum's largest")
        assert err <= 1e-10, (u, err)
