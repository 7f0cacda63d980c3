"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Integer and index results (reflection lists, culling lists, pixel map and the
binary64 culling records) must be bit-identical.  Floating-point results meet
the tolerances of the method's statement: patterns relative L2 <= 1e-4 and
per-pixel relative error <= 1e-3 over pixels above 1e-3 of the maximum; the
structure factors feed the patterns linearly through |F|^2 and are held to a
relative L2 of 2e-5 on |F|^2.  At the full benchmark sizes the oracle computes
sampled pixels and reflections one by one.
"""
import dataclasses
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import oracle as O
from strata import stratified_pixels

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2608_23245_amd import Pipeline, atoms_to_device  # noqa: E402
from paper_2608_23245_amd import binding as B  # noqa: E402

DEG = math.pi / 180


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def check_pattern(img, ref, tag):
    img = np.asarray(img, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert ref.max() > 0, f"{tag}: the reference image is empty"
    r = rel_l2(img, ref)
    big = ref > 1e-3 * ref.max()
    px = float(np.max(np.abs(img[big] - ref[big]) / ref[big]))
    say(f"{tag}: rel-L2 {r:.2e}, max per-pixel rel {px:.2e} over {int(big.sum())} px")
    assert r <= 1e-4 and px <= 1e-3, (tag, r, px)


SMALL = {
    "ragged": dict(seed=21, width=21, height=19, center=(9.7, 10.2)),
    "offcentre_g": dict(seed=22, width=30, height=26, center=(6.3, 20.9), g=(0.04, 0.02, 0.01)),
    "skew_voigt": dict(seed=23, width=24, height=24, cell=W.Cell(9.5, 12.0, 14.0, 80 * DEG, 100 * DEG, 110 * DEG),
                       sigma_theta=2 * DEG, gamma_theta=1.5 * DEG),
    "lorentz": dict(seed=24, width=17, height=33, sigma_theta=0.0, gamma_theta=2.5 * DEG),
    "tiny_det": dict(seed=25, width=1, height=3, center=(-8.0, 1.5)),
    "wide_nodes": dict(seed=26, width=16, height=16, n_nodes=40, d_min=4.0),
    "tilted": dict(seed=27, width=26, height=22, center=(13.0, 9.4), tilt=22 * DEG, sigma_theta=2 * DEG,
                   gamma_theta=1 * DEG),
    "tilted_back": dict(seed=28, width=19, height=25, tilt=-40 * DEG, g=(0.03, 0.03, 0.0)),
    "gaussian_damped": dict(seed=29, width=22, height=20, sigma_theta=2 * DEG, gamma_theta=1 * DEG,
                            g=(0.03, 0.02, 0.01), lineshape=1, B_axis=(4.0, 9.0, 2.5)),
    "hosemann": dict(seed=30, width=23, height=21, sigma_theta=3 * DEG, g=(0.03, 0.02, 0.01), lineshape=2),
    "hosemann_small_n": dict(seed=31, width=18, height=18, sigma_theta=2 * DEG, gamma_theta=2 * DEG,
                             g=(0.1, 0.02, 0.0), lineshape=2, size_A=(12.0, 60.0, 50.0), B_axis=(2.0, 2.0, 8.0)),
    "no_intensity_model": dict(seed=32, width=20, height=17, g=(0.04, 0.04, 0.0), intensity_model=0),
    "detector_tilted": dict(seed=33, width=24, height=22, center=(11.6, 10.3), det_tilt=25 * DEG, sigma_theta=2 * DEG,
                            gamma_theta=1 * DEG),
    "detector_and_fibre_tilted": dict(seed=34, width=20, height=26, det_tilt=-20 * DEG, tilt=15 * DEG,
                                      g=(0.02, 0.02, 0.0)),
}


@pytest.mark.parametrize("cfg", [0, 1, 2])
def test_enumeration_bit_exact(cfg):
    wl = W.config(cfg)
    say(f"enumeration config {cfg}")
    ext = (wl.dis.g[0], wl.dis.g[1], wl.dis.g[2], wl.quad.extinction)
    for e in (None, ext):
        got = B.enumerate_hkl(B.make_cell(wl.cell), wl.quad.d_min, wl.quad.d_max, extinction=e).cpu().numpy()
        ref = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
        if e is not None:
            ref = ref[~O.extinct_mask(ref, wl.dis, wl.quad.extinction)]
        assert got.shape == ref.shape and np.array_equal(got, ref)


def test_enumeration_edge_cases():
    say("enumeration edge cases")
    cell = W.Cell(7.784, 8.201, 10.38, 90 * DEG, 90 * DEG, 96.55 * DEG)
    for dmin, dmax in [(1.8, 30.0), (1.8, 0.0), (9.0, 30.0), (20.0, 30.0)]:
        got = B.enumerate_hkl(B.make_cell(cell), dmin, dmax).cpu().numpy()
        ref = O.enumerate_hkl(cell, dmin, dmax)
        assert np.array_equal(got, ref), (dmin, dmax)
    # empty shell: nothing between 20 and 30 A for this cell
    assert B.enumerate_hkl(B.make_cell(cell), 20.0, 30.0).shape[0] == 0


@pytest.mark.parametrize("name", list(SMALL))
def test_pixel_map_and_tiles_bit_exact(name):
    wl = W.small(**SMALL[name])
    say(f"pixel map {name}")
    pix, tile = B.pixel_map(B.make_model(wl).geom)
    R, Z = O.pixel_rz(wl.geom)
    p = pix.cpu().numpy()
    assert np.array_equal(p[..., 0], R) and np.array_equal(p[..., 1], Z)
    tb = O.tile_boxes(wl.geom).reshape(-1, 6)
    assert np.array_equal(tile.cpu().numpy()[:, :6], tb)


def _prep_inputs(wl, n_sample=None, seed=0):
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    hkl = hkl[~O.extinct_mask(hkl, wl.dis, wl.quad.extinction)]
    if n_sample is not None and hkl.shape[0] > n_sample:
        rng = np.random.default_rng(seed)
        hkl = hkl[np.sort(rng.choice(hkl.shape[0], n_sample, replace=False))]
    return np.ascontiguousarray(hkl)


@pytest.mark.parametrize("cfg,n_sample", [(0, None), (1, None), (2, 20000)])
def test_structure_factors(cfg, n_sample):
    """All reflections of the tiny and medium workloads and a seeded 20,000 of the large one's
    293,298 (50,000 atoms each: 1e9 atom-reflection pairs in the oracle's C loop)."""
    wl = W.config(cfg)
    hkl = _prep_inputs(wl, n_sample)
    say(f"structure factors config {cfg}: {hkl.shape[0]} reflections x {wl.atoms.n} atoms")
    atoms = atoms_to_device(wl.atoms)
    F, F2 = B.structure_factors(B.make_cell(wl.cell), atoms, torch.from_numpy(hkl).cuda())
    F = F.cpu().numpy().astype(np.float64)
    F2 = F2.cpu().numpy().astype(np.float64)
    ref = O.structure_factors_c(hkl, wl.cell, wl.atoms)
    ref2 = np.abs(ref) ** 2
    r = rel_l2(F2, ref2)
    big = ref2 > 1e-3 * ref2.max()
    per = float(np.max(np.abs(F2[big] - ref2[big]) / ref2[big]))
    cplx = float(np.max(np.abs((F[:, 0] + 1j * F[:, 1]) - ref)) / np.abs(ref).max())
    say(f"  |F|^2 rel-L2 {r:.2e}, max rel (strong) {per:.2e}, max |dF|/max|F| {cplx:.2e}")
    assert r <= 2e-5 and per <= 1e-4 and cplx <= 1e-5


def test_structure_factor_invariants():
    """Friedel mates and a centrosymmetric model on the device."""
    say("structure factor invariants")
    wl = W.config1()
    hkl = O.enumerate_hkl(wl.cell, 4.0, 30.0)
    a = wl.atoms
    n = 500
    xyz = np.stack([a.x[:n], a.y[:n], a.z[:n]], 1).astype(np.float64)
    cen = np.concatenate([xyz, 1.0 - xyz]).astype(np.float32)
    at = W.Atoms(cen[:, 0].copy(), cen[:, 1].copy(), cen[:, 2].copy(), np.tile(a.B[:n], 2), np.ones(2 * n, np.float32),
                 np.tile(a.type[:n], 2), a.ff)
    F, _ = B.structure_factors(B.make_cell(wl.cell), atoms_to_device(at), torch.from_numpy(hkl).cuda())
    F = F.cpu().numpy().astype(np.float64)
    scale = np.abs(F).max()
    assert np.abs(F[:, 1]).max() < 2e-5 * scale
    np.testing.assert_allclose(F[::-1, 0], F[:, 0], atol=2e-5 * scale)


def _voigt_case(sigma_deg, eta, n_nodes=48):
    """A workload whose angular shape is the Voigt of width sigma and mixing eta (reading R9:
    sigma_theta = (1 - eta) sigma, gamma_theta = eta sigma)."""
    st, gt = W.voigt_split(sigma_deg * DEG, eta)
    return W.small(5, sigma_theta=st, gamma_theta=gt, n_nodes=n_nodes)


NODE_CASES = {
    "g0": W.config0, "l1": W.config2, "v1": W.config1,
    "wide": lambda: W.small(5, sigma_theta=0.5 * DEG, gamma_theta=6 * DEG, n_nodes=100),
    # near the Gaussian limit: Im z = gamma/(sigma sqrt 2) ~ 7e-7 and 7e-4 (the real axis)
    "eta1e-6": lambda: _voigt_case(3.0, 1e-6),
    "eta1e-3": lambda: _voigt_case(3.0, 1e-3),
    # Im z ~ 0.037 < 0.1
    "eta0.05": lambda: _voigt_case(3.0, 0.05),
    "eta0.5": lambda: _voigt_case(3.0, 0.5),
    # near the Lorentzian limit: |z| up to ~1e7
    "eta1-1e-6": lambda: _voigt_case(3.0, 1 - 1e-6),
}


@pytest.mark.parametrize("case", list(NODE_CASES))
def test_node_table(case):
    """Node records against the oracle's node table and width derivatives (closed form
    through the Faddeeva function), near both limits of the Voigt and in its small-Im z
    region.  The float32 records hold each value to a few units in the last place; the
    derivatives are compared relative to their largest magnitude."""
    wl = NODE_CASES[case]()
    say(f"node table {case}: sigma_theta {wl.dis.sigma_theta:.3e}, gamma_theta {wl.dis.gamma_theta:.3e}, "
        f"Im z0 {wl.dis.gamma_theta / (math.sqrt(2) * wl.dis.sigma_theta) if wl.dis.sigma_theta else float('inf'):.2e}")
    n = wl.quad.n_nodes
    table = B.node_table(B.make_model(wl)).cpu().numpy().astype(np.float64)
    nodes = table[:n * n]
    nd = O.node_table(wl.quad.n_nodes, wl.quad.T, wl.quad.sigma_r, wl.dis.sigma_theta, wl.dis.gamma_theta)
    np.testing.assert_allclose(nodes[:, 0], nd.c - 1.0, rtol=2e-7, atol=1e-9)
    np.testing.assert_allclose(nodes[:, 1], nd.c * nd.d1, rtol=2e-7, atol=1e-9)
    np.testing.assert_allclose(nodes[:, 2], nd.c * nd.d2, rtol=2e-7, atol=1e-9)
    np.testing.assert_allclose(nodes[:, 3], nd.omega, rtol=1e-6, atol=1e-7 * nd.omega.max())
    ds, dg = O.node_weight_derivs(nd, wl.quad.sigma_r, wl.dis.sigma_theta, wl.dis.gamma_theta)
    for col, ref, name in ((4, ds, "d omega/d sigma"), (5, dg, "d omega/d gamma")):
        big = np.max(np.abs(ref))
        err = float(np.max(np.abs(nodes[:, col] - ref))) / big if big > 0 else float(np.max(np.abs(nodes[:, col])))
        say(f"  {name}: max |ref| {big:.3e}, max error / max |ref| {err:.2e}")
        np.testing.assert_allclose(nodes[:, col], ref, rtol=1e-6, atol=1e-7 * big)
    np.testing.assert_allclose(nodes[:, 6], nd.d1, rtol=2e-7, atol=1e-9)
    np.testing.assert_allclose(nodes[:, 7], nd.d2, rtol=2e-7, atol=1e-9)
    check_block_records(table, n)


def check_block_records(table, n):
    """Block records after the n^2 node records: every node value of a block lies in
    centre +- half-width exactly (float32 values compared in float64), the half-width is
    the tight one up to one float32 ulp, and mag bounds |centre| + half-width."""
    nb = (n + B.NODE_BLOCK - 1) // B.NODE_BLOCK
    assert table.shape[0] == n * n + nb * nb == B.node_rows(n)
    xyz = table[:n * n, :3].reshape(n, n, 3)          # [i2][i1]
    blk = table[n * n:].reshape(nb, nb, 8)
    for b2 in range(nb):
        for b1 in range(nb):
            v = xyz[b2 * B.NODE_BLOCK:(b2 + 1) * B.NODE_BLOCK, b1 * B.NODE_BLOCK:(b1 + 1) * B.NODE_BLOCK].reshape(-1, 3)
            c, r = blk[b2, b1, 0:3], blk[b2, b1, 4:7]
            assert np.all(np.abs(v - c) <= r), (b1, b2)
            tight = np.max(np.abs(v - c), axis=0)
            assert np.all(r <= tight + np.spacing(np.float32(np.maximum(r, 1e-30))).astype(np.float64)), (b1, b2)
            assert blk[b2, b1, 3] >= np.max(np.abs(c) + r)
            assert blk[b2, b1, 7] == 0.0


@pytest.mark.parametrize("name", list(SMALL) + ["config0", "config1"])
def test_reflection_records(name):
    wl = W.config0() if name == "config0" else (W.config1() if name == "config1" else W.small(**SMALL[name]))
    say(f"reflection records {name}")
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    F2 = np.linspace(1.0, 2.0, hkl.shape[0]).astype(np.float32)
    model = B.make_model(wl)
    refl, cull = B.reflection_prep(model, torch.from_numpy(hkl).cuda(), torch.from_numpy(F2).cuda())
    rb = O.reflection_boxes(wl, hkl)
    assert np.array_equal(cull.cpu().numpy()[:, :13], rb)
    P = O.prepare(wl, hkl=hkl, F=np.sqrt(F2.astype(np.float64)).astype(complex), cull_extinct=False)
    raw = refl.cpu().numpy()
    assert raw.shape[1] == 64
    np.testing.assert_allclose(raw[:, 39].astype(np.float64), P.W, rtol=2e-6)
    np.testing.assert_allclose(raw[:, 43:46].astype(np.float64), P.N, rtol=2e-6)
    np.testing.assert_allclose(raw[:, 0].astype(np.float64), P.r0, rtol=2e-7)
    # the two binary64 fields behind the kernels' cancellation-free offsets R - R_D and Z - Z_D
    # (record floats 18..19: D.e_perp, 20..21: D_z, each a little-endian float64), bit for bit:
    # D = h a* + k b* + l c* and e_perp (reading R6) in the oracle's operation order
    f64 = np.ascontiguousarray(raw[:, 18:22]).view(np.float64)
    RD = (P.D[:, 0] * P.ep[:, 0] + P.D[:, 1] * P.ep[:, 1]) + P.D[:, 2] * P.ep[:, 2]
    assert np.array_equal(f64[:, 0], RD), int(np.sum(f64[:, 0] != RD))
    assert np.array_equal(f64[:, 1], P.D[:, 2])
    check_offset_coefficients(raw, P, wl.dis.lineshape)


def check_offset_coefficients(raw, P, lineshape):
    """The float32 residuals (record floats 46..63) of the offset coefficients B, G1, G2, T_R,
    T_Z (floats 2..16) and T_A (floats 34..36): each is within half a float32 unit of its
    coefficient's last place (a residual, not a second copy), and for the Hosemann lineshape
    (offsets y_i = u_i = a_i.(p - s)) hi + lo is the oracle's r0 a_i.S, r0 a_i.e1, r0 a_i.e2,
    a_i.e_perp, a_i,z and a_i.e_az (e_az = z x e_perp) to 2^-47 relative."""
    hi = np.concatenate([raw[:, 2:17], raw[:, 34:37]], axis=1)
    lo = raw[:, 46:64].astype(np.float64)
    assert np.all(np.abs(lo) <= 0.5 * np.spacing(np.abs(hi)).astype(np.float64))
    hi = hi.astype(np.float64)
    if lineshape != 2:
        return
    a = P.avec
    eaz = np.stack([-P.ep[:, 1], P.ep[:, 0], np.zeros_like(P.r0)], axis=1)
    want = np.concatenate([P.r0[:, None] * (P.S @ a.T), P.r0[:, None] * (P.e1 @ a.T), P.r0[:, None] * (P.e2 @ a.T),
                           P.ep @ a.T, np.broadcast_to(a[:, 2], (P.r0.shape[0], 3)), eaz @ a.T], axis=1)
    scale = np.abs(want).max(axis=1, keepdims=True)
    err = np.abs(hi + lo - want)
    assert np.all(err <= 2.0 ** -47 * scale), float((err / scale).max())
    # the float32 slot alone is off by up to 2^-25 relative: the residual carries the rest
    assert float((np.abs(hi - want) / scale).max()) > 2.0 ** -40


def test_reflection_records_hosemann():
    wl = W.with_disorder(W.config0(), lineshape=2)
    say("reflection records, config 0 with the Hosemann lineshape: the offset coefficients' residuals")
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    F2 = np.linspace(1.0, 2.0, hkl.shape[0]).astype(np.float32)
    refl, _ = B.reflection_prep(B.make_model(wl), torch.from_numpy(hkl).cuda(), torch.from_numpy(F2).cuda())
    P = O.prepare(wl, hkl=hkl, F=np.sqrt(F2.astype(np.float64)).astype(complex), cull_extinct=False)
    check_offset_coefficients(refl.cpu().numpy(), P, 2)


@pytest.mark.parametrize("name", list(SMALL) + ["config0", "config1_sample"])
def test_culling_lists_bit_exact(name):
    say(f"culling lists {name}")
    if name == "config0":
        wl = W.config0()
    elif name == "config1_sample":
        wl = W.config1()
    else:
        wl = W.small(**SMALL[name])
    hkl = _prep_inputs(wl)
    model = B.make_model(wl)
    F2 = torch.ones(hkl.shape[0], dtype=torch.float32, device="cuda")
    _, cull = B.reflection_prep(model, torch.from_numpy(hkl).cuda(), F2)
    pix, tile = B.pixel_map(model.geom)
    offsets, idx = B.cull(model.geom, tile, cull)
    off = offsets.cpu().numpy()
    ix = idx.cpu().numpy()
    n_tiles = tile.shape[0]
    tiles = range(n_tiles)
    if name == "config1_sample":
        tiles = np.random.default_rng(1).choice(n_tiles, 200, replace=False)
    ref = O.culling_lists(wl, hkl, tiles=tiles)
    for t, lst in zip(tiles, ref):
        assert np.array_equal(ix[off[t]:off[t + 1]], lst), t
    assert np.all(np.diff(off) >= 0) and off[-1] == ix.shape[0]


@pytest.mark.parametrize("name", list(SMALL))
def test_pattern_small(name):
    wl = W.small(**SMALL[name])
    say(f"pattern {name}")
    pipe = Pipeline(wl)
    img = pipe.pattern().cpu().numpy()
    ref = O.pattern(wl, O.prepare(wl, hkl=pipe.hkl.cpu().numpy()))
    check_pattern(img, ref, name)


def test_pattern_config0_full_and_counts():
    wl = W.config0()
    say("pattern config 0")
    pipe = Pipeline(wl)
    img = pipe.pattern().cpu().numpy()
    P = O.prepare(wl)
    ref, n_ref = O.pattern(wl, P, count=True)
    check_pattern(img, ref, "config0")
    # symmetries of the detector image: mirror about the centred beam, Friedel about the equator
    assert np.abs(img - img[:, ::-1]).max() <= 1e-5 * img.max()
    assert np.abs(img - img[::-1, :]).max() <= 1e-5 * img.max()
    # support-passing evaluations agree with the oracle's count up to float32 boundary flips
    model = pipe.model
    _, F2 = pipe.structure_factors()
    refl, cull = B.reflection_prep(model, pipe.hkl, F2)
    nodes = B.node_table(model)
    pix, tile = B.pixel_map(model.geom)
    off, idx = B.cull(model.geom, tile, cull)
    n_gpu = B.profile(model, refl, nodes, pix, tile, off, idx, count=True)
    say(f"  useful evaluations gpu {n_gpu} oracle {n_ref}")
    assert abs(n_gpu - n_ref) <= 1e-4 * n_ref


MEDIUM_STRATA = {"strong": 96, "meridian": 32, "equator": 32, "corners": 16, "uniform": 80}


def _oracle_full(wl):
    """The oracle's whole reflection list of wl (extinction cull applied) and its prepared
    problem, with the structure factors of every reflection from the oracle's C loop."""
    hkl = _prep_inputs(wl)
    return hkl, O.prepare(wl, hkl=hkl, F=O.structure_factors_c(hkl, wl.cell, wl.atoms), cull_extinct=False)


def _sampled(wl, counts=MEDIUM_STRATA, seed=0):
    """GPU image at full size; the oracle at stratified pixels (tests/strata.py: picked from
    the oracle's own weights and geometry, never from the GPU image), summed over the whole
    reflection list with the oracle's own exact skip, independent of the culling lists."""
    pipe = Pipeline(wl)
    img = pipe.pattern().cpu().numpy()
    torch.cuda.synchronize()
    hkl, P = _oracle_full(wl)
    assert np.array_equal(pipe.hkl.cpu().numpy(), hkl)
    pix = stratified_pixels(wl, P, counts, seed)
    q = np.array([p for p, _ in pix], dtype=np.int64)
    R, Z = O.pixel_rz(wl.geom)
    vals = O.pattern_at(P, R.ravel()[q], Z.ravel()[q])
    names = sorted({s for _, s in pix})
    say(f"  oracle at {q.size} pixels ({', '.join(f'{n} {sum(1 for _, s in pix if s == n)}' for n in names)}) "
        f"over all {hkl.shape[0]} reflections")
    return img.ravel()[q], vals


def test_pattern_tilted_medium_sampled():
    """The medium workload with its fibre tilted by 22 degrees toward the beam (the tilt of
    the paper's A-DNA example), full size, oracle at sampled pixels."""
    wl = W.with_tilt(W.config1(), 22 * DEG)
    say("pattern medium, fibre tilt 22 deg, stratified pixels")
    got, ref = _sampled(wl, seed=11)
    check_pattern(got, ref, "medium tilted sampled")


@pytest.mark.parametrize("lineshape", ["gaussian", "hosemann"])
def test_pattern_lineshapes_medium_sampled(lineshape):
    """The medium workload with the Gaussian or Hosemann lineshape and axis damping
    B = (10, 10, 10) A^2 (the tutorial's values), full size, oracle at sampled pixels."""
    wl = W.with_disorder(W.config1(), lineshape=W.LINESHAPES[lineshape], B_axis=(10.0, 10.0, 10.0))
    say(f"pattern medium, {lineshape} lineshape, damping, stratified pixels")
    got, ref = _sampled(wl, seed=12)
    check_pattern(got, ref, f"medium {lineshape} sampled")


@pytest.mark.parametrize("tile_w,mirror", [(8, 0), (16, 3)])
def test_pattern_medium_full_size_sampled(tile_w, mirror):
    """The medium workload at full size, unfolded in 8x8 tiles and in the benchmark's launch
    (16x4 tiles, both mirror folds), the oracle at 256 stratified pixels.  (The large workload
    is compared at 1024 stratified pixels in test_gpu_fullsize.py.)"""
    wl = W.config1()
    wl = dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, tile_w=tile_w, mirror=mirror))
    say(f"pattern medium, {tile_w}x{64 // tile_w} tiles, mirror bits {mirror}, stratified pixels")
    got, ref = _sampled(wl, seed=1)
    check_pattern(got, ref, "medium sampled")


@pytest.mark.parametrize("name", ["ragged", "tilted", "config0", "config1"])
def test_tile_order_is_a_schedule_and_leaves_results_unchanged(name):
    """fdtbx_tile_order lists every tile once (the rest is padding), and the per-tile kernels
    give the same image (bit for bit), the same counts and the same adjoint sums (up to the
    order of binary64 atomic adds) with it as without it."""
    wl = W.config0() if name == "config0" else W.config1() if name == "config1" else W.small(**SMALL[name])
    say(f"tile order {name}")
    pipe = Pipeline(wl)
    model = pipe.model
    _, F2 = pipe.structure_factors()
    refl, cull = B.reflection_prep(model, pipe.hkl, F2)
    nodes = B.node_table(model)
    pix, tile = B.pixel_map(model.geom)
    off, idx = B.cull(model.geom, tile, cull)
    order = B.tile_order(model.geom, off)
    o = order.cpu().numpy()
    n_tiles = tile.shape[0]
    assert np.array_equal(np.sort(o[o >= 0]), np.arange(n_tiles))
    img0 = B.profile(model, refl, nodes, pix, tile, off, idx)
    img1 = B.profile(model, refl, nodes, pix, tile, off, idx, order=order)
    torch.cuda.synchronize()
    assert torch.equal(img0, img1)
    assert B.profile(model, refl, nodes, pix, tile, off, idx, count=True) == \
        B.profile(model, refl, nodes, pix, tile, off, idx, count=True, order=order)
    G = torch.as_tensor(np.random.default_rng(3).normal(size=img0.shape), dtype=torch.float32).cuda()
    s0 = B.profile_adjoint(model, refl, nodes, pix, tile, off, idx, G).cpu().numpy()
    s1 = B.profile_adjoint(model, refl, nodes, pix, tile, off, idx, G, order=order).cpu().numpy()
    np.testing.assert_allclose(s1, s0, rtol=1e-9, atol=1e-12 * np.abs(s0).max())
    if name == "config1":
        # few rounds of workgroups: the longest lists start first
        lens = np.diff(off.cpu().numpy())
        first, last = lens[o[o >= 0][:512]], lens[o[o >= 0][-512:]]
        say(f"  list length of the first 512 tiles {first.mean():.0f}, of the last 512 {last.mean():.0f}")
        assert first.mean() > 2 * last.mean()
