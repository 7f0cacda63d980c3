"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties one oracle step to something other than the oracle itself: an
exact integer brute force, a textbook closed form, an invariant, a published
approximation, or an independent numerical integration.  A plausible slip in
the oracle (dropped term, wrong sign or index, transposed operand) fails at
least one of them.
"""
import dataclasses
import math
import os

import numpy as np
import pytest
from scipy import integrate, optimize, special

import workloads as W
from oracle import oracle as O

DEG = math.pi / 180.0


# ----------------------------------------------------------------------------- frame (Eq. recip_basis)
@pytest.mark.parametrize("cell", [
    W.Cell(10, 10, 20, 90 * DEG, 90 * DEG, 90 * DEG),
    W.Cell(40, 40, 60, 90 * DEG, 95 * DEG, 90 * DEG),
    W.Cell(10.4, 6.717, 5.962, 80.37 * DEG, 118.08 * DEG, 114.8 * DEG),   # cellulose I-alpha cell of the paper
    W.Cell(7.784, 8.201, 10.38, 90 * DEG, 90 * DEG, 96.55 * DEG),         # cellulose I-beta cell of the tutorial
])
def test_frame_duality_and_metric(cell):
    avec, astar, V = O.frame(cell)
    # a*_i . a_j = delta_ij (section "Scattered vector and scattering amplitude")
    np.testing.assert_allclose(astar @ avec.T, np.eye(3), atol=1e-14)
    # edge lengths and angles of the real cell
    np.testing.assert_allclose(np.linalg.norm(avec, axis=1), [cell.a, cell.b, cell.c], rtol=1e-14)
    ang = lambda u, v: math.acos(u @ v / np.linalg.norm(u) / np.linalg.norm(v))
    np.testing.assert_allclose([ang(avec[1], avec[2]), ang(avec[0], avec[2]), ang(avec[0], avec[1])],
                               [cell.alpha, cell.beta, cell.gamma], atol=1e-12)
    # textbook cell volume
    ca, cb, cg = math.cos(cell.alpha), math.cos(cell.beta), math.cos(cell.gamma)
    Vt = cell.a * cell.b * cell.c * math.sqrt(1 - ca * ca - cb * cb - cg * cg + 2 * ca * cb * cg)
    assert abs(V - Vt) < 1e-12 * Vt
    # tutorial convention: c along +z, b in the yz-plane, beam a* along +x
    assert avec[2, 0] == 0 and avec[2, 1] == 0 and avec[2, 2] > 0
    assert avec[1, 0] == 0
    assert astar[0, 1] == 0 and astar[0, 2] == 0 and astar[0, 0] > 0


# ----------------------------------------------------------------------------- enumeration
def _brute_orthogonal(a, b, c, d_min, d_max):
    """Exact integer test for orthogonal cells: h^2/a^2 + k^2/b^2 + l^2/c^2 <= 1/d^2,
    scaled to integers (a, b, c, d given as integers or halves)."""
    out = []
    H, K, L = int(a / d_min) + 1, int(b / d_min) + 1, int(c / d_min) + 1
    from fractions import Fraction as Fr
    a, b, c, d_min, d_max = Fr(a), Fr(b), Fr(c), Fr(d_min), Fr(d_max)
    for h in range(-H, H + 1):
        for k in range(-K, K + 1):
            for l in range(-L, L + 1):
                if h == 0 and k == 0 and l == 0:
                    continue
                q = Fr(h * h) / (a * a) + Fr(k * k) / (b * b) + Fr(l * l) / (c * c)
                if q <= 1 / (d_min * d_min) and q >= 1 / (d_max * d_max):
                    out.append((h, k, l))
    return np.array(out, dtype=np.int32)


def test_enumeration_tiny_config_exact():
    wl = W.config0()
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    ref = _brute_orthogonal(10, 10, 20, 4, 30)
    assert hkl.shape == ref.shape == (150, 3)
    assert np.array_equal(hkl, ref)
    # 10 exact ties at d = 4 A are kept (inclusive resolution limit)
    q4 = 4 * hkl[:, 0] ** 2 + 4 * hkl[:, 1] ** 2 + hkl[:, 2] ** 2
    assert int(np.sum(q4 == 25)) == 10


def test_enumeration_general_cell_matches_metric_tensor():
    """Reciprocal metric tensor G* = G^-1 from the cell constants alone (no lab frame)."""
    cell = W.Cell(40, 40, 60, 90 * DEG, 95 * DEG, 90 * DEG)
    d_min, d_max = 4.0, 30.0
    hkl = O.enumerate_hkl(cell, d_min, d_max)
    ca, cb, cg = math.cos(cell.alpha), math.cos(cell.beta), math.cos(cell.gamma)
    G = np.array([[cell.a ** 2, cell.a * cell.b * cg, cell.a * cell.c * cb],
                  [cell.a * cell.b * cg, cell.b ** 2, cell.b * cell.c * ca],
                  [cell.a * cell.c * cb, cell.b * cell.c * ca, cell.c ** 2]])
    Gs = np.linalg.inv(G)
    r = np.arange(-16, 17)
    cand = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    q = np.einsum("ni,ij,nj->n", cand.astype(float), Gs, cand.astype(float))
    keep = (q <= 1 / d_min ** 2 * (1 + 1e-9)) & (q >= 1 / d_max ** 2 * (1 - 1e-9)) & np.any(cand != 0, 1)
    ref = cand[keep]
    assert np.array_equal(hkl, ref)


def test_enumeration_order_negation_and_volume():
    wl = W.config1()
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    assert hkl.shape[0] == 49962
    # ascending lexicographic order, closed under negation with mate at n-1-i
    keys = hkl[:, 0].astype(np.int64) * 10 ** 6 + hkl[:, 1] * 10 ** 3 + hkl[:, 2]
    assert np.all(np.diff(keys) > 0)
    assert np.array_equal(hkl, -hkl[::-1])
    # count -> reciprocal-shell volume times cell volume
    _, _, V = O.frame(wl.cell)
    est = 4 * math.pi / 3 * V * (1 / wl.quad.d_min ** 3 - 1 / wl.quad.d_max ** 3)
    assert abs(hkl.shape[0] / est - 1) < 0.01


# ----------------------------------------------------------------------------- structure factors
def _atoms(x, y, z, B, occ, typ, zs=(6, 7, 8)):
    f = lambda a: np.asarray(a, dtype=np.float32)
    return W.Atoms(f(x), f(y), f(z), f(B), f(occ), np.asarray(typ, dtype=np.int32), W.ff_table(zs))


@pytest.mark.parametrize("sf", [O.structure_factors, O.structure_factors_c])
def test_sf_single_atom_modulus(sf):
    cell = W.Cell(9, 11, 13, 90 * DEG, 100 * DEG, 90 * DEG)
    hkl = O.enumerate_hkl(cell, 2.0, 30.0)
    at = _atoms([0.123], [0.456], [0.789], [12.0], [0.7], [1])
    F = sf(hkl, cell, at)
    _, astar, _ = O.frame(cell)
    # |D|^2 from the metric tensor, s = |D|/2
    D = hkl @ astar
    s2 = np.sum(D * D, 1) / 4
    occ, b = float(np.float32(0.7)), float(np.float32(W.FF_B))    # inputs are float32
    expect = occ * 7.0 * np.exp(-b * s2) * np.exp(-12.0 * s2)
    np.testing.assert_allclose(np.abs(F), expect, rtol=1e-12)
    # phase: exp(2 pi i h.x) with x taken as the float32 input value
    x = np.array([np.float32(0.123), np.float32(0.456), np.float32(0.789)], dtype=np.float64)
    ph = np.angle(F / expect) / (2 * np.pi)
    d = (ph - hkl @ x) % 1.0
    assert np.all(np.minimum(d, 1 - d) < 1e-10)


@pytest.mark.parametrize("sf", [O.structure_factors, O.structure_factors_c])
def test_sf_friedel_centric_and_body_centred(sf):
    cell = W.Cell(12, 12, 16, 90 * DEG, 90 * DEG, 90 * DEG)
    hkl = O.enumerate_hkl(cell, 2.5, 30.0)
    rng = np.random.default_rng(7)
    n = 30
    xyz = rng.random((n, 3))
    B = rng.uniform(5, 20, n)
    typ = rng.integers(0, 3, n)
    F = sf(hkl, cell, _atoms(xyz[:, 0], xyz[:, 1], xyz[:, 2], B, np.ones(n), typ))
    # Friedel: F(-h) = conj F(h), mate at n-1-i
    np.testing.assert_allclose(F[::-1], np.conj(F), atol=1e-9 * np.abs(F).max())
    # centrosymmetric model (atoms at +-x): F real
    cx = np.concatenate([xyz, (1.0 - xyz)])
    Fc = sf(hkl, cell, _atoms(cx[:, 0], cx[:, 1], cx[:, 2], np.tile(B, 2), np.ones(2 * n), np.tile(typ, 2)))
    assert np.abs(Fc.imag).max() < 1e-6 * np.abs(Fc.real).max()
    # body-centred pair (x, x + 1/2,1/2,1/2) with exactly representable coordinates
    base = np.round(xyz * 64) / 128
    bc = np.concatenate([base, base + 0.5])
    Fb = sf(hkl, cell, _atoms(bc[:, 0], bc[:, 1], bc[:, 2], np.tile(B, 2), np.ones(2 * n), np.tile(typ, 2)))
    F1 = sf(hkl, cell, _atoms(base[:, 0], base[:, 1], base[:, 2], B, np.ones(n), typ))
    odd = (hkl.sum(1) % 2) != 0
    assert np.abs(Fb[odd]).max() < 1e-9 * np.abs(Fb).max()
    np.testing.assert_allclose(Fb[~odd], 2 * F1[~odd], rtol=1e-10, atol=1e-10 * np.abs(F1).max())


@pytest.mark.parametrize("sf", [O.structure_factors, O.structure_factors_c])
def test_sf_exact_rational_phases(sf):
    """Coordinates on a 1/8 grid: exp(2 pi i phi) is known exactly (eighth roots of unity)."""
    cell = W.Cell(10, 10, 10, 90 * DEG, 90 * DEG, 90 * DEG)
    hkl = O.enumerate_hkl(cell, 2.0, 0.0)
    num = np.array([[1, 3, 5], [2, 7, 0], [6, 1, 4]])
    at = _atoms(num[:, 0] / 8, num[:, 1] / 8, num[:, 2] / 8, [0, 0, 0], [1, 1, 1], [0, 1, 2])
    F = sf(hkl, cell, at)
    s2 = np.sum(hkl.astype(float) ** 2, 1) / 100 / 4
    roots = np.exp(2j * np.pi * np.arange(8) / 8)
    ref = np.zeros(len(hkl), complex)
    for j, zz in enumerate((6, 7, 8)):
        ref += zz * np.exp(-float(np.float32(W.FF_B)) * s2) * roots[(hkl @ num[j]) % 8]
    np.testing.assert_allclose(F, ref, rtol=1e-12, atol=1e-12)


# ----------------------------------------------------------------------------- paracrystal factors
def test_coherence_factor_is_gaussian_characteristic_function():
    """|phi(h)| for a Gaussian spacing distribution of relative width g, evaluated by
    numerical integration of E[exp(2 pi i h eps)], eps ~ N(0, g^2) (Eq. Ah)."""
    hkl = np.array([[1, 0, 0], [3, 2, 0], [7, -5, 2], [12, 0, -9]], dtype=np.int32)
    dis = W.Disorder(0.01, 0.0, (10.0, 8.0, 6.0), (0.03, 0.05, 0.02))
    A, N, Ip = O.disorder_factors(hkl, dis)
    for r in range(hkl.shape[0]):
        for i in range(3):
            g, h = dis.g[i], hkl[r, i]
            val, _ = integrate.quad(lambda e: math.cos(2 * math.pi * h * e) * math.exp(-e * e / (2 * g * g)) / (g * math.sqrt(2 * math.pi)),
                                    -12 * g, 12 * g, limit=400, epsabs=1e-14)
            assert abs(A[r, i] - val) < 1e-10


def test_hosemann_breadth_and_neff():
    """Eq. Z with |phi| = A held at its value at the reflection is the Poisson kernel:
    integral over one period 1, peak (1+A)/(1-A) (Eq. breadth).  With N_base -> inf,
    1/N_eff equals that integral breadth (Eq. Neff); with g -> 0 N_eff = N_base."""
    hkl = np.array([[2, 0, 0], [5, 3, 1], [9, 0, 4]], dtype=np.int32)
    big = W.Disorder(0.01, 0.0, (1e300, 1e300, 1e300), (0.04, 0.02, 0.03))
    A, N, _ = O.disorder_factors(hkl, big)
    for r in range(hkl.shape[0]):
        for i in range(3):
            a = A[r, i]
            if hkl[r, i] == 0:
                assert a == 1.0 and 1 / N[r, i] < 1e-299     # sharp lattice along this axis
                continue
            Z = lambda u: (1 - a * a) / (1 - 2 * a * math.cos(2 * math.pi * u) + a * a)
            area, _ = integrate.quad(Z, -0.5, 0.5, points=[0.0], limit=400, epsabs=1e-13)
            assert abs(area - 1) < 1e-9
            breadth = area / Z(0.0)
            assert abs(1 / N[r, i] - breadth) < 1e-10 * max(breadth, 1e-3)
    sharp = W.Disorder(0.01, 0.0, (7.0, 5.0, 3.0), (0.0, 0.0, 0.0))
    A0, N0, Ip0 = O.disorder_factors(hkl, sharp)
    assert np.all(A0 == 1.0) and np.all(Ip0 == 1.0)
    assert np.array_equal(N0, np.tile([7.0, 5.0, 3.0], (3, 1)))


@pytest.mark.parametrize("N", [0.8, 1.7, 3.75, 8.0, 25.0])
def test_axis_profiles_peak_integral_breadth(N):
    """Every lineshape is a per-axis peak of height N_eff, unit integral per lattice period
    and integral breadth 1/N_eff (Eq. breadth for the Hosemann form; the Laue form's mass
    is the Dirichlet integral, the Gaussian's the Gaussian integral)."""
    f = lambda ls, u: float(O.axis_profile(ls, N, u))
    # Laue: peak N, integral over the line 1 (sinc^2 integrates to 1)
    assert f(0, 0.0) == pytest.approx(N, rel=1e-15)
    lim = 400.0 / N
    mass = sum(integrate.quad(lambda u: f(0, u), a, a + 1.0 / N, limit=200)[0] for a in np.arange(-lim, lim, 1.0 / N))
    assert mass == pytest.approx(1.0, abs=2.0 / (math.pi ** 2 * 400.0))
    # Gaussian of matched integral breadth
    assert f(1, 0.0) == pytest.approx(N, rel=1e-15)
    assert integrate.quad(lambda u: f(1, u), -np.inf, np.inf)[0] == pytest.approx(1.0, rel=1e-10)
    # Hosemann: one period integrates to 1; peak (1 + A)/(1 - A) = N when N > 1, flat otherwise
    per = integrate.quad(lambda u: f(2, u), -0.5, 0.5, limit=200)[0]
    assert per == pytest.approx(1.0, rel=1e-10)
    assert f(2, 0.0) == pytest.approx(max(N, 1.0), rel=1e-12)
    assert f(2, 0.3) == pytest.approx(f(2, 1.3), rel=1e-12) and f(2, 0.3) == pytest.approx(f(2, -0.3), rel=1e-12)


def test_hosemann_profile_is_poisson_kernel():
    """Eq. Z is the Poisson kernel: (1 - A^2)/(1 - 2A cos t + A^2) = 1 + 2 sum_k A^k cos(k t)."""
    u = np.linspace(-0.5, 0.5, 41)
    for N in (1.5, 4.0, 12.0):
        A = (N - 1.0) / (N + 1.0)
        series = 1.0 + 2.0 * sum(A ** k * np.cos(2.0 * math.pi * k * u) for k in range(1, 2000))
        np.testing.assert_allclose(O.axis_profile(2, N, u), series, rtol=1e-10)


def test_axis_profile_n_derivatives_match_fd():
    """d/dN of each per-axis profile at fixed u (used by the adjoint) against central
    differences of axis_profile, through the compiled oracle's derivative routine."""
    wl = W.small(32, n_atoms=4, width=10, height=9, sigma_theta=3 * DEG, g=(0.02, 0.0, 0.01), n_nodes=10, d_min=5.0)
    for ls in (0, 1, 2):
        wl2 = W.with_disorder(wl, lineshape=ls)
        hkl = O.enumerate_hkl(wl2.cell, wl2.quad.d_min, wl2.quad.d_max)
        P = O.prepare(wl2, hkl=hkl, cull_extinct=False)
        R, Z = O.pixel_rz(wl2.geom)
        G = np.random.default_rng(ls).normal(size=R.shape)
        ds, dg = O.node_weight_derivs(P.nodes, wl2.quad.sigma_r, wl2.dis.sigma_theta, wl2.dis.gamma_theta)
        sums = O.grad_sums(P, ds, dg, R, Z, G, use_skip=False)
        # sums[:, 3 + i] = sum G L r0^2 omega dZ/dN_i: compare with (S(N + h) - S(N - h))/2h of sums[:, 0]
        for i in range(3):
            h = 1e-5
            Pp, Pm = O.prepare(wl2, hkl=hkl, cull_extinct=False), O.prepare(wl2, hkl=hkl, cull_extinct=False)
            Pp.N = P.N.copy()
            Pm.N = P.N.copy()
            Pp.N[:, i] += h
            Pm.N[:, i] -= h
            fd = (O.grad_sums(Pp, ds, dg, R, Z, G, use_skip=False)[:, 0] -
                  O.grad_sums(Pm, ds, dg, R, Z, G, use_skip=False)[:, 0]) / (2 * h)
            scale = np.abs(fd).max()
            assert scale > 0
            np.testing.assert_allclose(sums[:, 3 + i], fd, atol=2e-6 * scale, rtol=1e-5)


def test_axis_damping():
    """D(S) = exp(-1/4 sum B_i (S.a_i/|a_i|)^2): S.a_i = h_i for S = D_hkl, so the exponent is
    sum B_i h_i^2/|a_i|^2 / 4; equal B on an orthogonal cell gives the isotropic form
    exp(-2 pi^2 <u^2> S^2) with B = 8 pi^2 <u^2>."""
    skew = W.Cell(9.0, 11.0, 13.0, 80 * DEG, 100 * DEG, 110 * DEG)
    hkl = O.enumerate_hkl(skew, 3.0, 30.0)
    B = (3.0, 7.0, 11.0)
    lens = (skew.a, skew.b, skew.c)
    want = np.exp(-0.25 * sum(B[i] * hkl[:, i].astype(np.float64) ** 2 / lens[i] ** 2 for i in range(3)))
    np.testing.assert_allclose(O.axis_damping(hkl, skew, B), want, rtol=1e-13)
    ortho = W.Cell(9.0, 11.0, 13.0, 90 * DEG, 90 * DEG, 90 * DEG)
    hkl = O.enumerate_hkl(ortho, 3.0, 30.0)
    S2 = O.q_of(O.recip_vectors(hkl, O.frame(ortho)[1]))
    u2 = 0.07
    np.testing.assert_allclose(O.axis_damping(hkl, ortho, (8 * math.pi ** 2 * u2,) * 3),
                               np.exp(-2 * math.pi ** 2 * u2 * S2), rtol=1e-13)
    assert np.all(O.axis_damping(hkl, ortho, (0.0, 0.0, 0.0)) == 1.0)


def test_intensity_loss_is_sech():
    """2A/(1+A^2) with A = exp(-t) is 1/cosh(t) (Eq. Ipara)."""
    hkl = np.array([[1, 2, 3], [10, -4, 7], [0, 0, 15]], dtype=np.int32)
    dis = W.Disorder(0.01, 0.0, (5.0, 5.0, 5.0), (0.05, 0.03, 0.04))
    A, _, Ip = O.disorder_factors(hkl, dis)
    t = 2 * math.pi ** 2 * np.array(dis.g) ** 2 * hkl.astype(float) ** 2
    np.testing.assert_allclose(Ip, np.prod(1 / np.cosh(t), 1), rtol=1e-13)
    np.testing.assert_allclose(O.extinction_arg(hkl, dis.g), t.sum(1), rtol=1e-14)
    off = W.Disorder(0.01, 0.0, (5.0, 5.0, 5.0), (0.05, 0.03, 0.04), intensity_model=0)
    assert np.all(O.disorder_factors(hkl, off)[2] == 1.0)


# ----------------------------------------------------------------------------- angular shapes
def test_angular_shapes_peak_fwhm_and_limits():
    s, gm = 3 * DEG, 2 * DEG
    for st, gt in [(s, 0.0), (0.0, gm), (s, gm)]:
        assert abs(O.angular_shape(0.0, st, gt) - 1.0) < 1e-14
    half = lambda st, gt: optimize.brentq(lambda x: O.angular_shape(x, st, gt) - 0.5, 0.0, 20 * max(st, gt))
    # FWHM_G = 2 sqrt(2 ln 2) sigma ~ 2.3548 sigma, FWHM_L = 2 gamma
    assert abs(2 * half(s, 0.0) / s - 2 * math.sqrt(2 * math.log(2))) < 1e-10
    assert abs(2 * half(0.0, gm) / gm - 2.0) < 1e-10
    # for sigma = gamma the Gaussian is broader at half maximum by sqrt(2 ln 2) ~ 1.177
    assert abs(half(s, 0.0) / half(0.0, s) - math.sqrt(2 * math.log(2))) < 1e-10
    # Voigt FWHM vs Olivero-Longbothum (1977), accuracy 0.02%
    fG, fL = 2 * math.sqrt(2 * math.log(2)) * s, 2 * gm
    fV = 0.5346 * fL + math.sqrt(0.2166 * fL * fL + fG * fG)
    assert abs(2 * half(s, gm) / fV - 1) < 3e-4
    # Voigt limits: gamma -> 0 gives the Gaussian, sigma -> 0 the Lorentzian
    x = np.linspace(0, 15 * DEG, 31)
    # (the Voigt keeps Lorentzian tails ~gamma sigma/x^2, visible only where the Gaussian is ~1e-5)
    np.testing.assert_allclose(O.angular_shape(x, s, 1e-9 * s), O.angular_shape(x, s, 0.0), rtol=2e-6, atol=1e-10)
    np.testing.assert_allclose(O.angular_shape(x, 1e-7 * gm, gm), O.angular_shape(x, 0.0, gm), rtol=2e-6)
    with pytest.raises(ValueError):
        O.angular_shape(x, 0.0, 0.0)


def test_voigt_is_normalised_convolution():
    """g_V = (G*L)(x)/(G*L)(0), G of standard deviation sigma, L of HWHM gamma,
    by direct numerical convolution."""
    s, gm = 1.5 * DEG, 1.5 * DEG
    G = lambda t: math.exp(-t * t / (2 * s * s))
    L = lambda t: gm * gm / (t * t + gm * gm)
    conv = lambda x: integrate.quad(lambda t: G(t) * L(x - t), -40 * s, 40 * s, points=[0.0, x], limit=500, epsabs=1e-15)[0]
    c0 = conv(0.0)
    for x in [0.3 * DEG, 1.0 * DEG, 3.0 * DEG, 8.0 * DEG]:
        assert abs(O.angular_shape(x, s, gm) - conv(x) / c0) < 1e-7


def _richardson(f, x0, h):
    """Richardson-extrapolated central difference of f at x0 (error O(h^4))."""
    D = lambda hh: (f(x0 + hh) - f(x0 - hh)) / (2.0 * hh)
    return (4.0 * D(h / 2) - D(h)) / 3.0


@pytest.mark.parametrize("sig_deg,eta", [(3.0, 1e-6), (3.0, 1e-3), (3.0, 0.5), (3.0, 1 - 1e-3), (3.0, 1 - 1e-6),
                                         (1.0, 0.2), (8.0, 0.9)])
def test_angular_shape_width_derivatives_match_differences(sig_deg, eta):
    """The closed-form width derivatives (through the Faddeeva function's derivative) agree
    with Richardson differences of the unit-peak Voigt itself (scipy's voigt_profile, a
    different routine) at every angle of a node patch."""
    st, gt = (1 - eta) * sig_deg * DEG, eta * sig_deg * DEG
    x = np.linspace(0.0, 12 * sig_deg * DEG, 41)
    ds, dg = O.angular_shape_derivs(x, st, gt)
    # steps on the scale of the wider width (the shape varies on that scale), kept inside (0, width)
    width = max(st, gt)
    fs = _richardson(lambda v: O.angular_shape(x, v, gt), st, min(1e-3 * width, 0.5 * st))
    fg = _richardson(lambda v: O.angular_shape(x, st, v), gt, min(1e-3 * width, 0.5 * gt))
    scale = 1.0 / max(st, gt)      # derivatives of a unit-peak shape are O(1/width)
    np.testing.assert_allclose(ds, fs, rtol=1e-7, atol=1e-9 * scale)
    np.testing.assert_allclose(dg, fg, rtol=1e-7, atol=1e-9 * scale)


def test_angular_shape_width_derivatives_at_the_gaussian_and_lorentzian_limits():
    """Continuity of the derivatives across the branch points eta = 0 and eta = 1, and the
    one-sided gamma derivative of the Gaussian written with Dawson's integral F:
    d g/d gamma at gamma = 0+ = (2/sqrt(pi)) (2 x F(x) - 1 + exp(-x^2))/(sigma sqrt 2),
    x = delta/(sigma sqrt 2) (from w(x) = exp(-x^2) + (2i/sqrt(pi)) F(x) on the real axis and
    erfcx'(0) = -2/sqrt(pi))."""
    s = 3 * DEG
    x = np.linspace(0.0, 14 * s, 57)
    ds0, dg0 = O.angular_shape_derivs(x, s, 0.0)
    xx = x / (s * math.sqrt(2.0))
    closed = (2 / math.sqrt(math.pi)) * (2 * xx * special.dawsn(xx) - 1 + np.exp(-xx * xx)) / (s * math.sqrt(2.0))
    np.testing.assert_allclose(dg0, closed, rtol=1e-10, atol=1e-12 / s)
    np.testing.assert_allclose(ds0, np.exp(-xx * xx) * x * x / s ** 3, rtol=1e-13, atol=0)
    # the Voigt branch just above gamma = 0 tends to both
    ds1, dg1 = O.angular_shape_derivs(x, s, 1e-9 * s)
    np.testing.assert_allclose(ds1, ds0, rtol=1e-6, atol=1e-6 / s)
    np.testing.assert_allclose(dg1, dg0, rtol=1e-6, atol=1e-6 / s)
    # one-sided difference of the shape at gamma = 0 (second order)
    h = 1e-6 * s
    fd = (-3 * O.angular_shape(x, s, 0.0) + 4 * O.angular_shape(x, s, h) - O.angular_shape(x, s, 2 * h)) / (2 * h)
    np.testing.assert_allclose(dg0, fd, rtol=1e-5, atol=1e-5 / s)
    # sigma -> 0: the Lorentzian's gamma derivative, and a sigma derivative that vanishes like sigma
    gm = 2 * DEG
    x = np.linspace(0.0, 14 * gm, 57)
    dsL, dgL = O.angular_shape_derivs(x, 0.0, gm)
    np.testing.assert_allclose(dgL, 2 * gm * x * x / (x * x + gm * gm) ** 2, rtol=1e-14, atol=0)
    assert np.all(dsL == 0.0)
    for eps in (1e-4, 1e-6):
        dsV, dgV = O.angular_shape_derivs(x, eps * gm, gm)
        np.testing.assert_allclose(dgV, dgL, rtol=0, atol=10 * eps / gm)
        assert np.max(np.abs(dsV)) < 10 * eps / gm


@pytest.mark.parametrize("eta", [0.5, 1 - 1e-3, 1 - 1e-6])
def test_voigt_sigma_derivative_follows_the_heat_equation(eta):
    """The Voigt is a Lorentzian convolved with a Gaussian of variance sigma^2, and a Gaussian
    kernel obeys dG/dsigma = sigma d^2G/dt^2, so dV/dsigma = sigma V''(x) and the unit-peak
    shape has dg/dsigma = sigma (V''(x) V(0) - V(x) V''(0))/V(0)^2.  V'' by Richardson second
    differences of scipy's voigt_profile in x: an independent route to the sigma derivative
    that stays accurate next to the Lorentzian limit, where the derivative is of size sigma."""
    sig = 3 * DEG
    st, gt = (1 - eta) * sig, eta * sig
    x = np.linspace(0.0, 10 * sig, 21)
    V = lambda t: special.voigt_profile(t, st, gt)
    h = 1e-2 * min(gt, max(st, 1e-3 * gt)) if eta < 1 - 1e-4 else 1e-3 * gt

    def Vxx(t):
        d2 = lambda hh: (V(t + hh) - 2 * V(t) + V(t - hh)) / (hh * hh)
        return (4 * d2(h / 2) - d2(h)) / 3

    ref = st * (Vxx(x) * V(0.0) - V(x) * Vxx(0.0)) / V(0.0) ** 2
    ds, _ = O.angular_shape_derivs(x, st, gt)
    big = np.abs(ref).max()
    np.testing.assert_allclose(ds, ref, rtol=2e-5, atol=2e-5 * big)


# ----------------------------------------------------------------------------- nodes
def test_node_solid_angle_converges_to_gnomonic_square():
    """With g = 1 the node weights sum to the solid angle of the gnomonic square
    [-T,T]^2, 4 atan(T^2/sqrt(1+2T^2)), with O(h^2) error of the midpoint rule."""
    T = math.tan(20 * DEG)
    exact = 4 * math.atan(T * T / math.sqrt(1 + 2 * T * T))
    assert abs(exact - 0.4689848726) < 1e-9
    errs = []
    for n in (16, 32, 64):
        nd = O.node_table(n, T, 1.0, 1e6, 0.0)     # sigma huge: g = 1 to ~1e-13
        errs.append(abs(nd.omega.sum() / math.sqrt(2 * math.pi) - exact))
    assert errs[2] < 2e-5
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_node_gaussian_cap_mass():
    """sum_k omega_k / (sigma_r sqrt(2 pi)) -> integral of g over the sphere,
    2 pi int_0^pi exp(-D^2/2 s^2) sin(D) dD, when the grid covers the cap."""
    s = 2 * DEG
    nd = O.node_table(96, math.tan(12 * s), 1e-4, s, 0.0)
    cap, _ = integrate.quad(lambda d: 2 * math.pi * math.exp(-d * d / (2 * s * s)) * math.sin(d), 0, math.pi, limit=400)
    assert abs(nd.omega.sum() / (1e-4 * math.sqrt(2 * math.pi)) / cap - 1) < 2e-4
    # exact great-circle angle: Delta = arccos(c) = atan(rho)
    rho = np.hypot(nd.d1, nd.d2)
    np.testing.assert_allclose(nd.Delta, np.arctan(rho), rtol=1e-12, atol=1e-15)


# ----------------------------------------------------------------------------- Ewald geometry
def test_pixel_points_lie_on_ewald_sphere_and_round_trip():
    wl = W.small(3, width=23, height=17, center=(10.3, 9.1))
    R, Z = O.pixel_rz(wl.geom)
    lam = wl.geom.wavelength
    # rebuild S at azimuth psi for each pixel and check |k_in + S| = 1/lambda for psi = 0
    rng = np.random.default_rng(0)
    for j, i in [(0, 0), (16, 22), (9, 10), (3, 17)]:
        psi = rng.uniform(0, 2 * math.pi)
        S = np.array([R[j, i] * math.cos(psi), R[j, i] * math.sin(psi), Z[j, i]])
        p1, p2 = O.ewald_project(S, wl.geom)
        hits = np.stack([p1[0], p2[0]])
        # one of the two rotations lands on the pixel, the other on its mirror (lab y -> -y)
        mirror_i = 2 * (wl.geom.center_x - 0.5) - i
        targets = {(i, j), (mirror_i, j)}
        got = sorted([tuple(np.round(h, 9)) for h in hits])
        want = sorted([tuple(np.round(t, 9)) for t in targets])
        np.testing.assert_allclose(got, want, atol=1e-7)
    # the pixel's own scattering vector (psi such that S_x < 0 branch) is on the sphere
    SF = wl.geom.distance
    y = ((np.arange(wl.geom.width) + 0.5) - wl.geom.center_x) * wl.geom.pixel
    z = ((np.arange(wl.geom.height) + 0.5) - wl.geom.center_y) * wl.geom.pixel
    yy, zz = np.meshgrid(y, z)
    kout = np.stack([np.full_like(yy, SF), yy, zz], -1)
    kout /= np.linalg.norm(kout, axis=-1, keepdims=True) * lam
    S = kout - np.array([1 / lam, 0, 0])
    np.testing.assert_allclose(np.hypot(S[..., 0], S[..., 1]), R, rtol=1e-12)
    np.testing.assert_allclose(S[..., 2], Z, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("tilt_deg,det_deg", [(22.0, 0.0), (-35.0, 0.0), (60.0, 0.0), (0.0, 25.0), (22.0, -18.0)])
def test_tilted_fibre_round_trip(tilt_deg, det_deg):
    """Fibre tilted toward the beam (k_in . n != 0, so the D term of Eq. harmonic is
    nonzero), detector normal to the beam or turned about its horizontal axis: every point
    of the ring of a pixel's (R, Z) about the tilted axis, rotated into the diffraction
    condition by Eqs. harmonic/solutions and intersected with the detector plane (a ray and
    plane intersection in vector form), lands on the pixel or on its mirror (lab y -> -y).
    The pixel's (R, Z) come from its position X = (SF - z sin d, y, z cos d)."""
    t = tilt_deg * DEG
    wl = W.small(4, width=29, height=23, center=(12.3, 8.6), tilt=t)
    wl = dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, det_tilt=det_deg * DEG))
    n = np.array([math.sin(t), 0.0, math.cos(t)])
    m = np.array([math.cos(t), 0.0, -math.sin(t)])
    y = np.array([0.0, 1.0, 0.0])
    R, Z = O.pixel_rz(wl.geom)
    rng = np.random.default_rng(7)
    for j, i in [(0, 0), (22, 28), (11, 12), (5, 20), (17, 3)]:
        psi = rng.uniform(0, 2 * math.pi)
        S = R[j, i] * (math.cos(psi) * m + math.sin(psi) * y) + Z[j, i] * n
        p1, p2 = O.ewald_project(S, wl.geom, fibre=n)
        hits = np.stack([p1[0], p2[0]])
        mirror_i = 2 * (wl.geom.center_x - 0.5) - i
        got = sorted([tuple(np.round(h, 9)) for h in hits])
        want = sorted([tuple(np.round(v, 9)) for v in {(i, j), (mirror_i, j)}])
        np.testing.assert_allclose(got, want, atol=1e-7)
    if det_deg != 0.0 or tilt_deg == 0.0:
        return
    # tilt 0 leaves the map unchanged; a tilt mixes S_x into Z, so Z is no longer odd in z
    R0, Z0 = O.pixel_rz(W.small(4, width=29, height=23, center=(12.3, 8.6)).geom)
    assert not np.allclose(Z, Z0)
    assert np.all(R >= 0)
    # the tilt is a rotation about lab y: the pattern of a centred beam keeps its exact
    # mirror y -> -y and loses the up/down (Friedel) symmetry
    wc = W.small(6, width=20, height=18, n_nodes=10, tilt=t)
    img = O.pattern(wc, O.prepare(wc))
    assert img.max() > 0 and np.array_equal(img, img[:, ::-1])
    assert np.abs(img - img[::-1, :]).max() > 1e-3 * img.max()


@pytest.mark.parametrize("tilt_deg,det_deg", [(0.0, 0.0), (22.0, 0.0), (-35.0, 0.0), (0.0, 30.0), (-35.0, -20.0)])
def test_splat_projection_matches_ewald_solution(tilt_deg, det_deg):
    """The forward splat's algebraic projection (S_x = -lambda |S|^2/2, S.n = Z_S, S_y from
    |S|, then y = SF k_y cos d / D, z = SF k_z / D) lands where Eqs. harmonic/solutions
    (rotation about the tilted fibre axis, then k_out = k_in + S_phi intersected with the
    detector plane) put the point, for both rotations and detector tilts d."""
    t = tilt_deg * DEG
    wl = W.small(4, width=60, height=50, center=(31.3, 22.6), tilt=t)
    wl = dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, det_tilt=det_deg * DEG))
    n = np.array([math.sin(t), 0.0, math.cos(t)])
    m = np.array([math.cos(t), 0.0, -math.sin(t)])
    R, Z = O.pixel_rz(wl.geom)
    rng = np.random.default_rng(3)
    pts = []
    for _ in range(40):
        j, i = rng.integers(0, 50), rng.integers(0, 60)
        psi = rng.uniform(0, 2 * math.pi)
        pts.append((R[j, i] * math.cos(psi), R[j, i] * math.sin(psi), Z[j, i]))     # fibre frame
    S = np.array(pts)
    a1, a2 = O.splat_project(S, wl.geom)
    lab = np.array([np.hypot(s[0], s[1]) * m + s[2] * n for s in S])               # same (R, Z) about n
    e1, e2 = O.ewald_project(lab, wl.geom, fibre=n)
    for k in range(S.shape[0]):
        got = sorted([tuple(np.round(a1[k] - 0.5, 9)), tuple(np.round(a2[k] - 0.5, 9))])
        want = sorted([tuple(np.round(e1[k], 9)), tuple(np.round(e2[k], 9))])
        np.testing.assert_allclose(got, want, atol=1e-7)


@pytest.mark.parametrize("lineshape", [0, 1])
def test_splat_mass_converges_to_closed_form(lineshape):
    """With L = 1 (delta -> infinity) the splatted weight of one reflection integrates its
    profile over reciprocal space, twice (both rotations): 2 W r0^2 sum_k omega_k prod_i m_i / V,
    m_i the per-axis mass inside the support ((2/pi) Si(2 pi m) for Laue, erf(m sqrt(pi)) for
    the Gaussian).  The midpoint sampling converges to it as the grid refines."""
    wl = W.small(40, n_atoms=8, width=400, height=400, sigma_theta=1.5 * DEG, gamma_theta=0.0, n_nodes=12,
                 d_min=3.0, size_A=(60.0, 60.0, 80.0), lineshape=lineshape)
    wl.quad.delta = 1e6
    P = O.prepare(wl, hkl=np.array([[1, 1, 1]], dtype=np.int32), F=np.ones(1, complex), cull_extinct=False)
    V = O.frame(wl.cell)[2]
    m = wl.quad.m
    mass = ((2 / math.pi) * special.sici(2 * math.pi * m)[0]) ** 3 if lineshape == 0 else special.erf(m * math.sqrt(math.pi)) ** 3
    want = 2.0 * P.W[0] * P.r0[0] ** 2 * P.nodes.omega.sum() * mass / V
    coarse = O.splat(wl, P, 16, 96).sum() / want
    fine = O.splat(wl, P, 32, 192).sum() / want
    assert abs(fine - 1.0) < 5e-4 and abs(fine - 1.0) < abs(coarse - 1.0) / 20


def test_splat_symmetry_and_counts():
    """Centred beam, untilted fibre: the splat is mirror-symmetric bit for bit; every deposit
    of a sample of reflection h lands on a pixel whose ring coordinates are those of the sample."""
    wl = W.config0()
    P = O.prepare(wl)
    img, n = O.splat(wl, P, 4, 16, count=True)
    assert img.max() > 0 and n > 0 and np.array_equal(img, img[:, ::-1])
    R, Z = O.pixel_rz(wl.geom)
    S = np.array([[0.05, 0.07, 0.1], [0.11, -0.02, -0.04]])
    for a in O.splat_project(S, wl.geom):
        i, j = np.floor(a[:, 0]).astype(int), np.floor(a[:, 1]).astype(int)
        RS, ZS = np.hypot(S[:, 0], S[:, 1]), S[:, 2]
        pitch = wl.geom.pixel / wl.geom.distance / wl.geom.wavelength
        assert np.all(np.abs(R[j, i] - RS) < pitch) and np.all(np.abs(Z[j, i] - ZS) < pitch)


def test_cyl_single_node_ring_integral():
    """Eq. cyl-average for a one-node shell (the node at D) of an orthogonal cell: with D
    in the x-z plane the ring offset is (R cos phi - R_D, R sin phi, Z - Z_D), so the ring
    average is W r0^2 omega f_c (1/2 pi) int f_a(a R cos phi - h) f_b(b R sin phi) dphi,
    computed here by adaptive quadrature; the oracle's trapezoid rule converges to it."""
    wl = W.small(50, n_atoms=4, width=10, height=10, sigma_theta=2 * DEG, n_nodes=1, size_A=(60.0, 66.0, 78.0))
    P = O.prepare(wl, hkl=np.array([[2, 0, 1]], dtype=np.int32), F=np.ones(1, complex), cull_extinct=False)
    a, b, c = wl.cell.a, wl.cell.b, wl.cell.c
    N, m = P.N[0], wl.quad.m
    R, Z = 2 / a + 0.004, 1 / c + 0.003

    def f(i, u):
        return float(O.axis_profile(0, N[i], u)) if abs(u) <= m / N[i] else 0.0

    ring = integrate.quad(lambda ph: f(0, a * R * math.cos(ph) - 2) * f(1, b * R * math.sin(ph)), -0.5, 0.5,
                          limit=500, epsabs=0, epsrel=1e-12)[0]
    want = P.W[0] * P.r0[0] ** 2 * P.nodes.omega[0] * f(2, c * Z - 1) * ring / (2 * math.pi)
    for arc, tol in ((5e-4, 1e-6), (1e-4, 1e-8)):
        got = O.cyl_at(P, np.array([R]), np.array([Z]), arc, use_skip=False)[0]
        assert abs(got / want - 1) < tol, (arc, got, want)
    # the exact skip leaves the sum unchanged
    assert O.cyl_at(P, np.array([R]), np.array([Z]), 5e-4) == O.cyl_at(P, np.array([R]), np.array([Z]), 5e-4, use_skip=False)


def test_cyl_culling_is_conservative():
    """Every reflection whose ring average is nonzero at some pixel of a tile is in that tile's
    list under the cylindrical culling description."""
    wl = W.small(51, n_atoms=6, width=40, height=30, sigma_theta=1.5 * DEG, n_nodes=10, d_min=4.5, g=(0.02, 0.02, 0.0),
                 pixel=1.6)
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    P = O.prepare(wl, hkl=hkl, F=np.ones(hkl.shape[0], complex), cull_extinct=False)
    lists = O.culling_lists(wl, hkl, boxes=O.cyl_boxes(wl, hkl))
    R, Z = O.pixel_rz(wl.geom)
    H, Wd = R.shape
    tx_n = (Wd + 7) // 8
    missed = 0
    for r in range(hkl.shape[0]):
        Pr = _single(P, r)
        vals = O.cyl_at(Pr, R, Z, 2e-3, use_skip=False).reshape(H, Wd)
        for j, i in zip(*np.nonzero(vals)):
            t = (j // 8) * tx_n + i // 8
            missed += r not in set(lists[t].tolist())
    assert missed == 0
    assert sum(len(x) for x in lists) < hkl.shape[0] * len(lists)   # the description does cull


def test_ewald_validity():
    """Beam normal to the fibre: S can be rotated onto the sphere iff lambda |S|^2 <= 2 R
    (Eq. valid); otherwise both angles are NaN."""
    lam = 1.0
    rng = np.random.default_rng(1)
    S = rng.uniform(-0.8, 0.8, (2000, 3))
    p1, p2 = O.ewald_angles(S, lam)
    R = np.hypot(S[:, 0], S[:, 1])
    q = np.sum(S * S, 1)
    ok = lam * q <= 2 * R
    margin = np.abs(lam * q - 2 * R) > 1e-9
    assert np.array_equal(np.isfinite(p1)[margin], ok[margin])
    assert np.array_equal(np.isfinite(p2)[margin], ok[margin])
    # valid angles do satisfy |k_in + S_phi| = 1/lambda
    Sphi = O.rodrigues(S[ok], p1[ok])
    np.testing.assert_allclose(np.linalg.norm(Sphi + np.array([1 / lam, 0, 0]), axis=1), 1 / lam, rtol=1e-12)


def test_lorentz_bounds():
    d = 1e-5
    R = np.concatenate([[0.0], np.logspace(-9, 0, 50)])
    L = O.lorentz(R, d)
    assert L[0] == 1.0 and np.all(L > 0) and np.all(L <= 1)
    np.testing.assert_allclose(L[-5:] * R[-5:] / d, 1.0, rtol=1e-4)


# ----------------------------------------------------------------------------- Laue kernel through the profile loop
def _probe_problem(N, cell=None, m=3):
    """Single node at d = 0 with omega = 1: the profile at p is r0^2 Z(p - D)."""
    cell = cell or W.Cell(9, 11, 13, 90 * DEG, 100 * DEG, 90 * DEG)
    avec, astar, _ = O.frame(cell)
    hkl = np.array([[2, -1, 3]], dtype=np.int32)
    D = O.recip_vectors(hkl, astar)
    r0, S, e1, e2, ep = O.reflection_frames(D)
    nodes = O.Nodes(np.zeros(1), np.zeros(1), np.ones(1), np.zeros(1), np.ones(1), 1.0)
    P = O.Prepared(hkl, np.ones(1, complex), np.ones(1), np.array([N], float), np.ones((1, 3)), np.ones(1),
                   D, r0, S, e1, e2, ep, avec, astar, nodes, m, 1e-5)
    return P


def _profile_points(P, pts):
    """Profile of reflection 0 at arbitrary Cartesian points: express each point as
    R e_perp + Z z with e_perp rotated to the point's azimuth."""
    out = []
    for p in pts:
        Q = O.Prepared(**{**P.__dict__})
        R = math.hypot(p[0], p[1])
        Q.ep = np.array([[p[0] / R, p[1] / R, 0.0]])
        out.append(O.profile_table(Q, np.array([R]), np.array([p[2]]))[0, 0])
    return np.array(out)


def test_laue_kernel_peak_zeros_and_laue_function():
    N = (4.0, 5.0, 3.0)
    P = _probe_problem(N)
    D = P.D[0]
    r0 = P.r0[0]
    # peak value r0^2 N_a N_b N_c (Eq. I_shape)
    assert abs(_profile_points(P, [D])[0] / (r0 * r0) - 60.0) < 1e-12
    # zeros at a_i.(p - D) = k/N_i
    for i in range(3):
        for k in (1, 2):
            v = _profile_points(P, [D + (k / N[i]) * P.astar[i]])[0]
            assert abs(v) < 1e-25
    # near the peak the envelope matches the 1-D Laue function (Eq. laue1d):
    # sum_n |exp(2 pi i u n)|^2 over N cells, divided by N, per axis
    u = np.array([0.004, 0.013, -0.021])
    v = _profile_points(P, [D + (u[0] * P.astar[0] + u[1] * P.astar[1] + u[2] * P.astar[2])])[0] / (r0 * r0)
    lattice = 1.0
    for i, n in enumerate((4, 5, 3)):
        amp = abs(sum(np.exp(2j * np.pi * u[i] * np.arange(n)))) ** 2
        lattice *= amp / n
    assert abs(v / lattice - 1) < 3 * (math.pi * 0.021) ** 2


def test_laue_kernel_truncated_mass():
    """Along one axis the kept mass is (2/pi) Si(2 pi m) = 0.966410 for m = 3."""
    N = (4.0, 5.0, 3.0)
    P = _probe_problem(N)
    D = P.D[0]
    frac = 2 / math.pi * special.sici(2 * math.pi * 3)[0]
    assert abs(frac - 0.966410) < 1e-6
    u = np.linspace(-1.0, 1.0, 4001)     # beyond the support m/N = 0.75
    vals = _profile_points(P, [D + x * P.astar[0] for x in u]) / (P.r0[0] ** 2) / (N[1] * N[2])
    mass = np.trapezoid(vals, u)
    assert abs(mass - frac) < 2e-5
    assert np.all(vals[np.abs(u) > 3 / N[0] + 1e-12] == 0.0)


# ----------------------------------------------------------------------------- shell quadrature vs brute force
def test_shell_quadrature_matches_volume_integral():
    """Eq. shell_conv integrated directly: finite radial Gaussian shell (width sigma_r)
    times the angular Gaussian, convolved with the truncated Laue kernel, in spherical
    coordinates about S over the same angular square.  Agrees with the node sum within
    the delta-collapse error plus quadrature error."""
    wl = W.small(11, sigma_theta=4 * DEG, size_A=(40.0, 40.0, 50.0), n_nodes=48)
    P = O.prepare(wl, hkl=np.array([[1, 1, 1], [2, 0, 1]], dtype=np.int32), F=np.ones(2, complex), cull_extinct=False)
    sig_r = wl.quad.sigma_r
    T = wl.quad.T
    st = wl.dis.sigma_theta
    for r in range(2):
        D = P.D[r]
        S, e1, e2 = P.S[r], P.e1[r], P.e2[r]
        r0 = P.r0[r]
        N = P.N[r]
        # three query points: on the peak, along the arc, off the shell radially
        qs = [D, r0 * (math.cos(0.05) * S + math.sin(0.05) * e2), D * (1 + 0.4 / (N[2] * r0 * wl.cell.c))]
        # node-sum value
        node_vals = _profile_points(_single(P, r), qs)
        # brute force
        th = np.linspace(0, math.atan(T * math.sqrt(2)), 500)
        ph = np.linspace(0, 2 * math.pi, 800, endpoint=False)
        dth, dph = th[1] - th[0], ph[1] - ph[0]
        TH, PH = np.meshgrid(th[:-1] + dth / 2, ph + dph / 2, indexing="ij")
        d1 = np.tan(TH) * np.cos(PH)
        d2 = np.tan(TH) * np.sin(PH)
        inside = (np.abs(d1) <= T) & (np.abs(d2) <= T)
        nhat = (np.cos(TH)[..., None] * S + np.sin(TH)[..., None] * (np.cos(PH)[..., None] * e1 + np.sin(PH)[..., None] * e2))
        gx, gw = np.polynomial.hermite_e.hermegauss(12)
        for qi, p in enumerate(qs):
            tot = 0.0
            for x, wgt in zip(gx, gw):
                rr = r0 + sig_r * x
                s = rr * nhat
                u = (p - s) @ P.avec.T
                ok = np.all(np.abs(u) <= 3 / N, axis=-1) & inside
                z = np.prod(N * np.sinc(N * u) ** 2, axis=-1)
                integrand = np.where(ok, z, 0.0) * np.exp(-TH ** 2 / (2 * st * st)) * np.sin(TH) * rr * rr
                # radial Gaussian exp(-(r-r0)^2/2 s_r^2) dr -> hermegauss weights times sig_r
                tot += wgt * sig_r * integrand.sum() * dth * dph
            assert abs(node_vals[qi] / tot - 1) < 5e-4, (r, qi, node_vals[qi], tot)


def _single(P, r):
    sl = slice(r, r + 1)
    return O.Prepared(P.hkl[sl], P.F[sl], P.W[sl], P.N[sl], P.A[sl], P.Ip[sl], P.D[sl], P.r0[sl], P.S[sl],
                      P.e1[sl], P.e2[sl], P.ep[sl], P.avec, P.astar, P.nodes, P.m, P.delta)


def test_node_refinement_converges():
    """Profile values at fixed points converge under n -> 2n -> 4n (midpoint rule, O(h^2))."""
    vals = []
    for n in (24, 48, 96):
        wl = W.small(5, sigma_theta=3 * DEG, size_A=(50.0, 50.0, 60.0), n_nodes=n)
        P = O.prepare(wl, hkl=np.array([[1, 2, 1]], dtype=np.int32), F=np.ones(1, complex), cull_extinct=False)
        D, S, e2, r0 = P.D[0], P.S[0], P.e2[0], P.r0[0]
        pts = [D, r0 * (math.cos(0.04) * S + math.sin(0.04) * e2)]
        vals.append(_profile_points(P, pts))
    vals = np.array(vals)
    e1 = np.abs(vals[0] - vals[2])
    e2 = np.abs(vals[1] - vals[2])
    assert np.all(e2 < e1 / 2.5)
    assert np.all(np.abs(vals[1] / vals[2] - 1) < 2e-3)


# ----------------------------------------------------------------------------- pattern invariants
def test_pattern_symmetries_and_skip():
    wl = W.config0()
    P = O.prepare(wl)
    img, n = O.pattern(wl, P, count=True)
    img2, n2 = O.pattern(wl, P, use_skip=False, count=True)
    assert np.array_equal(img, img2) and n == n2
    # mirror y -> -y about the centred beam is exact; Friedel z -> -z holds to rounding
    assert np.array_equal(img, img[:, ::-1])
    assert np.abs(img - img[::-1, :]).max() <= 1e-12 * img.max()
    assert np.all(img >= 0) and img.max() > 0


@pytest.mark.parametrize("kw", [
    dict(seed=2, sigma_theta=3 * DEG, gamma_theta=1 * DEG, g=(0.02, 0.01, 0.03)),
    dict(seed=3, lineshape=2, g=(0.03, 0.02, 0.01), sigma_theta=2 * DEG),
    dict(seed=4, lineshape=1, sigma_theta=2 * DEG, B_axis=(4.0, 9.0, 2.5), cell=W.Cell(11.0, 9.0, 13.0, 1.55, 1.68, 1.49)),
])
def test_friedel_up_down_symmetry_and_its_conditions(kw):
    """The up-down fold's premise: with the fibre normal to the beam and the beam centred on the
    rows, the pattern is symmetric under z -> -z to rounding (Friedel mates, even lineshapes,
    point-symmetric node sets) for any lineshape, disorder and skewed cell, also with the beam off
    the middle column; a tilted fibre or a beam off the middle row breaks it."""
    base = dict(width=30, height=28, **kw)
    sym = O.pattern(W.small(center=(11.3, 14.0), **base), O.prepare(W.small(center=(11.3, 14.0), **base)))
    assert sym.max() > 0 and np.abs(sym - sym[::-1, :]).max() <= 1e-12 * sym.max()
    for extra in (dict(center=(15.0, 14.0), tilt=10 * DEG), dict(center=(15.0, 14.3))):
        wl = W.small(**base, **extra)
        img = O.pattern(wl, O.prepare(wl))
        assert np.abs(img - img[::-1, :]).max() > 1e-3 * img.max()


def test_g_zero_reduces_to_plain_laue():
    """g -> 0: A = 1, N_eff = N_base, I_para = 1, and the pattern equals the one computed
    with the plain Laue kernel of size N_base."""
    wl = W.small(2, g=(1e-12, 1e-12, 1e-12))
    P = O.prepare(wl)
    assert np.allclose(P.N, np.array(wl.dis.N_base)[None, :], rtol=1e-15)
    assert np.all(P.Ip == 1.0)
    wl0 = W.small(2)
    P0 = O.prepare(wl0)
    np.testing.assert_allclose(O.pattern(wl, P), O.pattern(wl0, P0), rtol=1e-13, atol=0)


@pytest.mark.parametrize("tw,th", [(8, 8), (4, 16), (16, 4), (2, 32), (32, 2)])
def test_culling_lists_are_conservative(tw, th):
    """Every reflection with a nonzero profile at some pixel of a tile is in that tile's list,
    for tiles of every shape the GPU launches take."""
    wl = W.small(4, width=37, height=19, g=(0.04, 0.02, 0.0), center=(17.7, 10.2))
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    P = O.prepare(wl, hkl=hkl, F=np.ones(len(hkl), complex), cull_extinct=False)
    R, Z = O.pixel_rz(wl.geom)
    tab = O.profile_table(P, R, Z).reshape(R.shape[0], R.shape[1], -1)
    lists = O.culling_lists(wl, hkl, tw, th)
    ny, nx = (R.shape[0] + th - 1) // th, (R.shape[1] + tw - 1) // tw
    assert len(lists) == ny * nx
    nonempty, listed = 0, 0
    for ty in range(ny):
        for tx in range(nx):
            blk = tab[ty * th:(ty + 1) * th, tx * tw:(tx + 1) * tw]
            hit = np.nonzero(np.any(blk != 0, axis=(0, 1)))[0]
            assert set(hit.tolist()) <= set(lists[ty * nx + tx].tolist())
            nonempty += len(hit)
            listed += len(lists[ty * nx + tx])
    assert nonempty > 0 and listed < 4 * nonempty


# ----------------------------------------------------------------------------- adjoint vs finite differences
def _fd_problem(sigma_theta, gamma_theta, g=(0.03, 0.02, 0.01), intensity_model=1, seed=31):
    wl = W.small(seed, n_atoms=6, width=14, height=12, sigma_theta=sigma_theta, gamma_theta=gamma_theta, g=g,
                 n_nodes=14, d_min=4.5, center=(6.2, 5.7))
    wl.dis.intensity_model = intensity_model
    a = wl.atoms
    f64 = lambda v: np.asarray(v, dtype=np.float64).copy()
    wl.atoms = W.Atoms(f64(a.x), f64(a.y), f64(a.z), f64(a.B), f64(a.occ) * 0.9, a.type.copy(), a.ff.astype(np.float64))
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    G = np.random.default_rng(seed).normal(size=(wl.geom.height, wl.geom.width))
    return wl, hkl, G


def _loss(wl, hkl, G):
    P = O.prepare(wl, hkl=hkl, cull_extinct=False)
    return float(np.sum(G * O.pattern(wl, P, use_skip=False)))


@pytest.mark.parametrize("st,gt", [(3 * DEG, 2 * DEG), (4 * DEG, 0.0), (0.0, 3 * DEG)])
def test_oracle_gradients_match_finite_differences(st, gt):
    """L = sum G * image; the oracle's adjoint against FP64 central differences of its own
    forward for every global parameter and every atom field."""
    import copy
    wl, hkl, G = _fd_problem(st, gt)
    P = O.prepare(wl, hkl=hkl, cull_extinct=False)
    gr = O.gradients(wl, P, G, use_skip=False)

    def fd(mut, h):
        w1, w2 = copy.deepcopy(wl), copy.deepcopy(wl)
        mut(w1, +h)
        mut(w2, -h)
        return (_loss(w1, hkl, G) - _loss(w2, hkl, G)) / (2 * h)

    checks = []
    if st > 0:
        checks.append(("sigma", gr["sigma_theta"], fd(lambda w, h: setattr(w.dis, "sigma_theta", w.dis.sigma_theta + h), 1e-7)))
    if gt > 0:
        checks.append(("gamma", gr["gamma_theta"], fd(lambda w, h: setattr(w.dis, "gamma_theta", w.dis.gamma_theta + h), 1e-7)))
    for i in range(3):
        def mN(w, h, i=i):
            nb = list(w.dis.N_base)
            nb[i] += h
            w.dis.N_base = tuple(nb)
        checks.append((f"N{i}", gr["N_base"][i], fd(mN, 1e-5)))

        def mg(w, h, i=i):
            gg = list(w.dis.g)
            gg[i] += h
            w.dis.g = tuple(gg)
        checks.append((f"g{i}", gr["g"][i], fd(mg, 1e-6)))
    for j in range(wl.atoms.n):
        for field, h in (("x", 1e-6), ("y", 1e-6), ("z", 1e-6), ("B", 1e-4), ("occ", 1e-5)):
            def ma(w, hh, field=field, j=j):
                getattr(w.atoms, field)[j] += hh
            checks.append((f"{field}{j}", gr["atoms"][field][j], fd(ma, h)))
    scale = max(abs(c[2]) for c in checks)
    for name, an, num in checks:
        assert abs(an - num) <= 1e-6 * scale + 1e-5 * abs(num), (name, an, num)


@pytest.mark.parametrize("lineshape", [1, 2])
def test_oracle_gradients_lineshapes_and_damping_fd(lineshape):
    """Gaussian and Hosemann lineshapes with axis damping: the oracle's adjoint for the
    globals (sigma, N_base, g, B_axis) and a few atom fields against central differences."""
    import copy
    wl, hkl, G = _fd_problem(3 * DEG, 1 * DEG)
    wl.dis.lineshape = lineshape
    wl.dis.B_axis = (4.0, 9.0, 2.5)
    P = O.prepare(wl, hkl=hkl, cull_extinct=False)
    gr = O.gradients(wl, P, G, use_skip=False)

    def fd(mut, h):
        w1, w2 = copy.deepcopy(wl), copy.deepcopy(wl)
        mut(w1, +h)
        mut(w2, -h)
        return (_loss(w1, hkl, G) - _loss(w2, hkl, G)) / (2 * h)

    def tup(name, i):
        def mut(w, h):
            v = list(getattr(w.dis, name))
            v[i] += h
            setattr(w.dis, name, tuple(v))
        return mut

    checks = [("sigma", gr["sigma_theta"], fd(lambda w, h: setattr(w.dis, "sigma_theta", w.dis.sigma_theta + h), 1e-7))]
    for i in range(3):
        checks.append((f"N{i}", gr["N_base"][i], fd(tup("N_base", i), 1e-5)))
        checks.append((f"g{i}", gr["g"][i], fd(tup("g", i), 1e-6)))
        checks.append((f"B{i}", gr["B_axis"][i], fd(tup("B_axis", i), 1e-4)))
    for j in range(2):
        for field, h in (("x", 1e-6), ("B", 1e-4), ("occ", 1e-5)):
            def ma(w, hh, field=field, j=j):
                getattr(w.atoms, field)[j] += hh
            checks.append((f"{field}{j}", gr["atoms"][field][j], fd(ma, h)))
    scale = max(abs(c[2]) for c in checks)
    for name, an, num in checks:
        assert abs(an - num) <= 1e-6 * scale + 1e-5 * abs(num), (name, an, num)


def test_oracle_intensity_model_none_and_dot_product():
    """intensity_model 0 drops the I_para term of the g gradient; the adjoint is linear in G."""
    wl, hkl, G = _fd_problem(3 * DEG, 1 * DEG, intensity_model=0)
    P = O.prepare(wl, hkl=hkl, cull_extinct=False)
    g1 = O.gradients(wl, P, G, use_skip=False)
    g2 = O.gradients(wl, P, 2.0 * G, use_skip=False)
    np.testing.assert_allclose(g2["g"], 2.0 * g1["g"], rtol=1e-12)
    # <J v, G> = <v, J^T G> for v along sigma: directional FD of the image
    import copy
    h = 1e-7
    w1, w2 = copy.deepcopy(wl), copy.deepcopy(wl)
    w1.dis.sigma_theta += h
    w2.dis.sigma_theta -= h
    Jv = (O.pattern(w1, O.prepare(w1, hkl=hkl, cull_extinct=False), use_skip=False)
          - O.pattern(w2, O.prepare(w2, hkl=hkl, cull_extinct=False), use_skip=False)) / (2 * h)
    assert abs(np.sum(Jv * G) - g1["sigma_theta"]) <= 1e-6 * abs(g1["sigma_theta"])


def test_profile_points_single_node_closed_form():
    """With one node the shell quadrature is the node at D alone: at p = D + sum_i u_i a*_i
    (so that a_i.(p - D) = u_i) the term of Eq. direct_sum is W r0^2 omega prod_i N_i sinc^2(N_i u_i)
    inside the support |u_i| <= m/N_i and zero outside (sinc from numpy)."""
    wl = W.small(52, n_atoms=5, n_nodes=1, size_A=(45.0, 55.0, 65.0), sigma_theta=2 * DEG)
    P = O.prepare(wl, hkl=np.array([[1, 2, 1], [0, 0, 2], [-2, 1, 0]], np.int32), cull_extinct=False)
    rng = np.random.default_rng(3)
    ridx, pts, want = [], [], []
    for r in range(3):
        N = P.N[r]
        for _ in range(40):
            u = rng.uniform(-2.0 * wl.quad.m, 2.0 * wl.quad.m, 3) / N
            ridx.append(r)
            pts.append(P.D[r] + u @ P.astar)
            inside = np.all(np.abs(u) <= wl.quad.m / N)
            want.append(P.W[r] * P.r0[r] ** 2 * P.nodes.omega[0] * np.prod(N * np.sinc(N * u) ** 2) if inside else 0.0)
    got = O.profile_points(P, np.array(ridx), np.array(pts))
    assert np.count_nonzero(want) > 10 and np.count_nonzero(np.array(want) == 0.0) > 10
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=0.0)


def test_profile_points_sum_to_the_pattern():
    """Each pixel of the pattern is L(R) times the sum over reflections of their terms at the
    pixel's query points p*_h = R e_perp,h + Z z (Eqs. direct_sum, lorentz)."""
    wl = W.small(53, width=9, height=7, sigma_theta=3 * DEG, gamma_theta=1 * DEG, g=(0.02, 0.02, 0.0))
    P = O.prepare(wl)
    R, Z = O.pixel_rz(wl.geom)
    R, Z = R.ravel()[::5], Z.ravel()[::5]
    n_h = P.hkl.shape[0]
    pts = (R[:, None, None] * P.ep[None, :, :] + Z[:, None, None] * np.array([0.0, 0.0, 1.0])).reshape(-1, 3)
    vals = O.profile_points(P, np.tile(np.arange(n_h), R.size), pts).reshape(R.size, n_h)
    L = P.delta / (R + P.delta)
    ref = O.pattern_at(P, R, Z, use_skip=False)
    assert ref.max() > 0
    np.testing.assert_allclose(L * vals.sum(1), ref, rtol=1e-11, atol=1e-14 * ref.max())


def _golden(name):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            key, value, decimals = line.split()[:3]
            out[key] = (float(value), None if decimals == "-" else int(decimals))
    return out


def test_oracle_reproduces_the_numbers_the_paper_prints():
    """The oracle's angular weights and Lorentz factor give, at the precision the paper prints
    them, the numbers of tests/golden/paper_printed_values.txt; the synthetic detectors follow
    Eq. SF with its 0.9 fill."""
    g = _golden("paper_printed_values.txt")
    s = 2.5 * DEG
    half = lambda st, gt: optimize.brentq(lambda x: O.angular_shape(x, st, gt) - 0.5, 0.0, 20 * max(st, gt))
    v, d = g["gaussian_fwhm_over_sigma"]
    assert round(2 * half(s, 0.0) / s, d) == v
    v, d = g["gaussian_over_lorentz_half_width"]
    assert round(half(s, 0.0) / half(0.0, s), d) == v
    delta = g["lorentz_delta"][0]
    assert W.config1().quad.delta == delta and W.config0().quad.delta == delta
    assert O.lorentz(0.0, delta) == 1.0
    assert abs(O.lorentz(1e3 * delta, delta) * 1e3 - 1.0) < 2e-3      # L ~ delta / R for R >> delta
    fill = g["detector_fill"][0]
    for wl in W.config4(n_models=4):
        geo = wl.geom
        two_theta = 2 * math.asin(geo.wavelength / (2 * wl.quad.d_min))
        want = fill * min(geo.width, geo.height) * geo.pixel / (2 * math.tan(two_theta))
        assert abs(geo.distance - want) <= 1e-12 * want


@pytest.mark.parametrize("det_deg", [20.0, -30.0])
def test_detector_tilt_geometry(det_deg):
    """A detector turned by d about its horizontal axis (top toward the sample for d > 0):
    the pixel at detector coordinates (y, z) sits at X = (SF - z sin d, y, z cos d), so its
    scattering angle obeys tan(2 theta) = sqrt(y^2 + (z cos d)^2) / (SF - z sin d) and
    |S| = 2 sin(theta) / lambda, with S along X/|X| - x.  The beam-centre row keeps its
    angles; for d > 0 the rows above the beam move toward the sample (larger angles) and the
    rows below away from it."""
    d = det_deg * DEG
    base = W.small(4, width=31, height=27, center=(15.5, 13.5), distance=60.0, pixel=0.8)
    g = dataclasses.replace(base.geom, det_tilt=d)
    Sx, Sy, Sz = O.pixel_S(g)
    i = np.arange(g.width, dtype=np.float64)
    j = np.arange(g.height, dtype=np.float64)
    y, z = np.meshgrid(((i + 0.5) - g.center_x) * g.pixel, ((j + 0.5) - g.center_y) * g.pixel)
    two_theta = np.arctan2(np.sqrt(y ** 2 + (z * math.cos(d)) ** 2), g.distance - z * math.sin(d))
    lam = g.wavelength
    np.testing.assert_allclose(np.sqrt(Sx ** 2 + Sy ** 2 + Sz ** 2), 2.0 * np.sin(0.5 * two_theta) / lam, rtol=1e-12,
                               atol=1e-15)
    # direction: S along the unit ray minus the beam, the ray built as a vector sum: the beam
    # centre P0 = SF x plus y along u = y and z along v = x sin(-d) + z cos(d), the vertical
    # axis turned about u by d toward the sample
    u = np.array([0.0, 1.0, 0.0])
    v = math.cos(d) * np.array([0.0, 0.0, 1.0]) - math.sin(d) * np.array([1.0, 0.0, 0.0])
    X = g.distance * np.array([1.0, 0.0, 0.0]) + y[..., None] * u + z[..., None] * v
    dirn = X / np.linalg.norm(X, axis=-1, keepdims=True) - np.array([1.0, 0.0, 0.0])
    np.testing.assert_allclose(np.stack([Sx, Sy, Sz], -1) * lam, dirn, rtol=0, atol=1e-14)
    # law of cosines: |X|^2 = SF^2 + y^2 + z^2 - 2 SF z sin d (the angle at P0 between the
    # detector's vertical axis and the way back to the sample is 90 deg - d)
    np.testing.assert_allclose(np.sum(X ** 2, -1), g.distance ** 2 + y ** 2 + z ** 2 - 2 * g.distance * z * math.sin(d),
                               rtol=1e-13)
    # the row through the beam centre keeps its angles; the up-down fold needs the symmetry
    # z -> -z, which a detector tilt breaks
    S0 = np.stack(O.pixel_S(base.geom), -1)
    mid = np.abs(z[:, 0]) < 1e-12
    assert mid.sum() == 0 or np.array_equal(np.stack([Sx, Sy, Sz], -1)[mid], S0[mid])
    S1 = np.sqrt(Sx ** 2 + Sy ** 2 + Sz ** 2)
    assert not np.allclose(S1, S1[::-1, :])
