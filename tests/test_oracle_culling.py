"""The culling contract against the oracle's own exact skip at the medium workload's full size,
and the stored oracle values of the large workload against a fresh oracle run (slow CPU tests).

Conservativeness: at 512 stratified pixels of the medium detector (tests/strata.py), every
reflection whose oracle profile is nonzero at a pixel (over the whole reflection list, the
exact skip ruling out only reflections whose support provably misses the pixel) is listed for
the pixel's tile, in the 8x8 tiles and in the benchmark's 16x4 tiles.

Stored values: four of the 1024 pixels of golden/large_pixels.json (two strong, two in a
corner) recomputed from scratch, which ties the file to the current oracle and inputs."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import oracle as O
from strata import stratified_pixels

pytestmark = pytest.mark.slow

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large_pixels.json")


def _full_list(wl):
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    return np.ascontiguousarray(hkl[~O.extinct_mask(hkl, wl.dis, wl.quad.extinction)])


def test_culling_lists_are_conservative_at_medium_size():
    wl = W.config1()
    hkl = _full_list(wl)
    P = O.prepare(wl, hkl=hkl, F=O.structure_factors_c(hkl, wl.cell, wl.atoms), cull_extinct=False)
    pix = stratified_pixels(wl, P, {"strong": 192, "meridian": 64, "equator": 64, "corners": 32, "uniform": 160},
                            seed=17)
    q = np.array([p for p, _ in pix], dtype=np.int64)
    assert q.size == 512
    R, Z = O.pixel_rz(wl.geom)
    table = O.profile_table(P, R.ravel()[q], Z.ravel()[q], use_skip=True)     # [pixel][reflection]
    hit = table > 0.0
    print(f"  {int(hit.sum())} (pixel, reflection) pairs with a nonzero profile at {q.size} pixels", flush=True)
    assert hit.sum() > 10 * q.size
    W_ = wl.geom.width
    for tw in (8, 16):
        th = 64 // tw
        tx_n = -(-W_ // tw)
        tiles = (q // W_) // th * tx_n + (q % W_) // tw
        uniq = np.unique(tiles)
        lists = dict(zip(uniq.tolist(), O.culling_lists(wl, hkl, tile_w=tw, tile_h=th, tiles=uniq)))
        for k in range(q.size):
            need = np.nonzero(hit[k])[0]
            assert np.all(np.isin(need, lists[int(tiles[k])])), (tw, int(q[k]))
        print(f"  {tw}x{th} tiles: every contributing reflection of the {q.size} pixels is listed", flush=True)


def test_stored_large_values_match_a_fresh_oracle_run():
    doc = json.load(open(GOLDEN))
    wl = W.config2()
    assert doc["width"] == wl.geom.width and doc["height"] == wl.geom.height
    strong = [p for p in doc["pixels"] if p["stratum"] == "strong"][:2]
    corner = [p for p in doc["pixels"] if p["stratum"] == "corners"][:2]
    pick = strong + corner
    q = np.array([p["q"] for p in pick], dtype=np.int64)
    R, Z = O.pixel_rz(wl.geom)
    vals, sub = O.pattern_sampled(wl, R.ravel()[q], Z.ravel()[q])
    assert O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max).shape[0] >= doc["n_hkl"]
    stored = np.array([float(p["value"]) for p in pick])
    print(f"  {q.size} pixels over {sub.size} reachable reflections: {vals} vs stored {stored}", flush=True)
    np.testing.assert_allclose(vals, stored, rtol=1e-12, atol=0)
