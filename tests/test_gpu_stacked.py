"""Stacked tiles of the batched forward (fdtbx_stacked_boxes, fdtbx_stacked_cull,
fdtbx_batch_profile_stacked): the stacked boxes are the unions of their two tiles' boxes, every
launched stacked list contains the lists of both its tiles (ascending, the other lists empty),
and a batch walked on stacked tiles gives the images of the per-tile walk to float32 rounding,
with and without the mirror folds, for odd and even numbers of launched tile rows, one tile
row, every lineshape and tile shapes from 4x16 to 32x2; and a batch of sixteen random small
models of the launch sweep against the per-tile walk and the oracle."""
import ctypes
import dataclasses
import math
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2608_23245_amd import atoms_to_device  # noqa: E402
from paper_2608_23245_amd import binding as B  # noqa: E402
from paper_2608_23245_amd.batch import BatchEngine  # noqa: E402

DEG = math.pi / 180


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def geom(wl, **kw):
    return dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, **kw))


def cases():
    base = [
        W.small(71, n_atoms=30, width=24, height=20, sigma_theta=3 * DEG, gamma_theta=1 * DEG, g=(0.02, 0.02, 0.0)),
        W.small(72, n_atoms=15, width=17, height=29, sigma_theta=0.0, gamma_theta=2 * DEG, n_nodes=20,
                cell=W.Cell(8.0, 12.0, 10.0, 90 * DEG, 104 * DEG, 90 * DEG), center=(5.2, 14.7)),
        W.small(73, n_atoms=40, width=32, height=36, sigma_theta=4 * DEG, gamma_theta=0.0, g=(0.03, 0.0, 0.01),
                n_nodes=16, d_min=4.0, lineshape=1, B_axis=(3.0, 5.0, 1.0)),
        W.small(74, n_atoms=25, width=9, height=3, sigma_theta=2 * DEG, gamma_theta=2 * DEG, center=(-6.0, 1.0)),
        W.small(75, n_atoms=33, width=27, height=11, sigma_theta=5 * DEG, gamma_theta=0.5 * DEG, n_nodes=10,
                cell=W.Cell(11.0, 9.5, 12.5, 95 * DEG, 90 * DEG, 100 * DEG), lineshape=2, g=(0.02, 0.01, 0.0),
                tilt=15 * DEG),
    ]
    out = {}
    for i, wl in enumerate(base):
        out[f"m{i}"] = wl
    # centred detectors under the folds: 14 tile rows of each shape, 7 of them launched under
    # the up-down fold (an odd number: the last stacked row holds one tile row)
    def centred(tw, width=64, rows=14):
        h = rows * (64 // tw)
        return geom(W.small(76, n_atoms=30, width=width, height=h, center=(width / 2, h / 2), sigma_theta=3 * DEG,
                            gamma_theta=1 * DEG), tile_w=tw)
    for tw in (4, 8, 16, 32):
        out[f"fold3_tw{tw}"] = geom(centred(tw), mirror=3)
    out["fold1_tw16"] = geom(centred(16, rows=13), mirror=1)
    out["fold2_tw8"] = geom(centred(8, width=40, rows=12), mirror=2)
    return out


CASES = cases()


def lists(model, wl):
    ext = (wl.dis.g[0], wl.dis.g[1], wl.dis.g[2], wl.quad.extinction) if wl.quad.extinction > 0 else None
    hkl = B.enumerate_hkl(model.cell, wl.quad.d_min, wl.quad.d_max, extinction=ext)
    _, F2 = B.structure_factors(model.cell, atoms_to_device(wl.atoms), hkl, want_F=False)
    _, cull = B.reflection_prep(model, hkl, F2)
    _, tile = B.pixel_map(model.geom)
    off, idx = B.cull(model.geom, tile, cull)
    return tile, cull, off, idx


@pytest.mark.parametrize("name", list(CASES))
def test_stacked_boxes_and_lists(name):
    wl = CASES[name]
    model = B.make_model(wl)
    tile, cull, off, idx = lists(model, wl)
    sbox, soff, sidx = B.stacked_cull(model.geom, tile, cull)
    tx, ty = B.tile_grid(model.geom)
    g = model.geom
    lcols = (tx + 1) // 2 if g.mirror & 1 else tx
    lrows = (ty + 1) // 2 if g.mirror & 2 else ty
    nrows = (lrows + 1) // 2
    say(f"stacked tiles, {name}: {tx}x{ty} tiles, {lrows} launched rows -> {nrows} stacked rows, "
        f"{sidx.numel()} stacked pairs against {idx.numel()}")
    assert B.lib().fdtbx_stacked_rows(ctypes.byref(g)) == nrows
    assert tuple(sbox.shape) == (tx * nrows, 8)
    tb = tile.cpu().numpy().reshape(ty, tx, 8)
    sb = sbox.cpu().numpy().reshape(nrows, tx, 8)
    o, ix = off.cpu().numpy(), idx.cpu().numpy()
    so, six = soff.cpu().numpy(), sidx.cpu().numpy()
    for sy in range(nrows):
        r0 = 2 * sy
        r1 = r0 + 1 if r0 + 1 < lrows else r0
        lo = np.minimum(tb[r0, :, 0:6:2], tb[r1, :, 0:6:2])
        hi = np.maximum(tb[r0, :, 1:6:2], tb[r1, :, 1:6:2])
        assert np.array_equal(sb[sy, :, 0:6:2], lo) and np.array_equal(sb[sy, :, 1:6:2], hi)
        assert np.all(sb[sy, :, 6:] == 0.0)
        for sx in range(tx):
            s = sy * tx + sx
            got = six[so[s]:so[s + 1]]
            if sx >= lcols:
                assert got.size == 0
                continue
            assert np.all(np.diff(got) > 0)
            for r in (r0, r1):
                t = r * tx + sx
                assert np.all(np.isin(ix[o[t]:o[t + 1]], got)), (sy, sx, r)


def compare(wls, tag):
    a = BatchEngine(wls, stacked=True)
    b = BatchEngine(wls, stacked=False)
    a.forward()
    b.forward()
    torch.cuda.synchronize()
    assert a.totals["stacked_pair"] < a.totals["pair"] or a.totals["pair"] == 0
    for m in range(len(wls)):
        x = a.image_of(m).double().cpu().numpy()
        y = b.image_of(m).double().cpu().numpy()
        scale = float(np.abs(y).max())
        err = float(np.abs(x - y).max())
        say(f"  {tag} model {m} {x.shape}: largest difference {err / max(scale, 1e-300):.1e} of the largest pixel")
        assert scale > 0 and err <= 2e-6 * scale
    return a


def test_stacked_forward_matches_per_tile_walk():
    wls = [CASES[k] for k in CASES]
    say(f"stacked against per-tile batched forward, {len(wls)} models")
    a = compare(wls, "cases")
    say(f"  pairs: stacked {a.totals['stacked_pair']}, per tile {a.totals['pair']}")


def test_stacked_forward_benchmark_models():
    wls = W.config4(n_models=3)[:2]
    say("stacked against per-tile batched forward, two models of the benchmark batch")
    compare([geom(w, tile_w=16) for w in wls], "config4")


def test_stacked_host_checks():
    """Invalid geometry and null pointers: refused on the host, before any launch."""
    L = B.lib()
    g = B.make_model(CASES["m0"]).geom
    bad = type(g).from_buffer_copy(g)
    bad.width = 0
    assert L.fdtbx_stacked_rows(ctypes.byref(bad)) == 0
    assert L.fdtbx_stacked_cull_workspace(ctypes.byref(bad), 10) == 0
    assert L.fdtbx_stacked_boxes(ctypes.byref(g), None, None, B._stream()) == -1
    one = torch.zeros(1, dtype=torch.int64, device="cuda")
    assert L.fdtbx_batch_profile_stacked(None, 1, B._ptr(one), B._ptr(one), 1, *([B._ptr(one)] * 9),
                                         B._stream()) == -1


def test_stacked_random_batch_vs_oracle():
    """Sixteen seeded random small models of the launch sweep (detector sizes, beam centres,
    cells, fibre tilts, lineshapes, tile shapes from 2x32 to 32x2, the mirror folds where the
    beam is centred) in one batch: stacked against per-tile walk, and each image against the
    oracle at the pattern tolerances."""
    from oracle import oracle as O
    from test_gpu_launch_sweep import random_case
    wls = []
    for seed in range(16):
        wl, fold = random_case(seed)
        wl = geom(wl, mirror=fold)
        m = B.make_model(wl)
        ext = (wl.dis.g[0], wl.dis.g[1], wl.dis.g[2], wl.quad.extinction) if wl.quad.extinction > 0 else None
        if B.enumerate_hkl(m.cell, wl.quad.d_min, wl.quad.d_max, extinction=ext).shape[0] > 0:
            wls.append(wl)
    say(f"random batch: {len(wls)} models, tile widths {[w.geom.tile_w for w in wls]}, "
        f"mirror bits {[w.geom.mirror for w in wls]}")
    a = compare(wls, "random")
    for m, wl in enumerate(wls):
        hkl = a.hkl[a.hkl_off[m]:a.hkl_off[m + 1]].cpu().numpy()
        ref = O.pattern(wl, O.prepare(wl, hkl=hkl))
        got = a.image_of(m).cpu().numpy().astype(np.float64)
        r = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        big = ref > 1e-3 * ref.max()
        px = float(np.max(np.abs(got[big] - ref[big]) / ref[big]))
        say(f"  model {m}: rel-L2 {r:.2e}, per-pixel {px:.2e} against the oracle")
        assert r <= 1e-4 and px <= 1e-3, (m, r, px)
