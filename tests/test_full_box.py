"""The full box of the forward walk's split queue, checked in float32 on the host.

The profile kernels' pair set-up bounds the node offsets kappa that lie inside the support
|y| <= m/2 of every pixel of a tile, y = alpha - kappa with alpha linear in the pixel's (R, Z)
(the Laue offsets of Eq. Z's quadrature point).  Nodes in that box are walked without the
support test, so the box must be conservative in float32: for every pixel of the tile's box
and every kappa the box admits, the y the walk computes satisfies |y| <= m/2 exactly as the
test would decide.  This test repeats the kernel's float32 operations (the same order, the
same roundings, the last-bit tags of alpha and kappa) with numpy on random geometries, puts
kappa on the box's edges and the pixels on the tile box's corners and inside it, and checks
that no computed |y| exceeds m/2.  It also checks that the margin is not so wide that the box
is empty for tiles much smaller than the support.
"""
import numpy as np

MARGIN = np.float32(1.0e-3)  # the kernels' tile-level margin, in y units
F32 = np.float32


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def fma32(a, b, c):
    """float32 fused multiply-add: the float32 product is exact in float64, and the float64 sum
    is rounded once more to float32 (a double rounding that can differ from a true fma by one
    unit in the last place, far below the margin)."""
    return f32(a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64))


def tag_alpha(v):
    a = np.clip(np.abs(v), F32(2.0 ** -18), F32(2.0 ** 30)).astype(np.float32)
    a = (a.view(np.int32) | 1).view(np.float32)
    return np.copysign(a, v).astype(np.float32)


def tag_kappa(v):
    return (v.astype(np.float32).view(np.int32) & ~1).view(np.float32)


def full_box(tr, tz, RD, ZD, Rlo, Rhi, Zlo, Zhi, half_m):
    """The set-up's full box [fl, fh] of one axis, in the kernel's float32 operation order."""
    dRl, dRh = f32(Rlo - RD), f32(Rhi - RD)
    dZl, dZh = f32(Zlo - ZD), f32(Zhi - ZD)
    r1, r2, z1, z2 = tr * dRl, tr * dRh, tz * dZl, tz * dZh
    amin = (np.minimum(r1, r2) + np.minimum(z1, z2)).astype(np.float32)
    amax = (np.maximum(r1, r2) + np.maximum(z1, z2)).astype(np.float32)
    mag = (np.maximum(np.abs(r1), np.abs(r2)) + np.maximum(np.abs(z1), np.abs(z2))).astype(np.float32)
    m = fma32(mag, np.full_like(mag, F32(2.0 ** -19)), np.full_like(mag, MARGIN))
    fl = ((amax - half_m).astype(np.float32) + m).astype(np.float32)
    fh = ((amin + half_m).astype(np.float32) - m).astype(np.float32)
    return fl, fh


def walk_y(tr, tz, RD, ZD, R, Z, kappa):
    """The walk's y = tag(alpha) - tag(kappa) at pixel (R, Z)."""
    dR, dZ = f32(R - RD), f32(Z - ZD)
    al = tag_alpha(fma32(tr, dR, (tz * dZ).astype(np.float32)))
    return (al - tag_kappa(kappa)).astype(np.float32)


def draw(rng, n):
    """Random tiles and reflections: coefficients over six decades, either sign; the
    reflection's centre within a few support widths of the tile or far along its zero line;
    tile extents from a hundredth to a tenth of the support."""
    sign = lambda: rng.choice([-1.0, 1.0], n)  # noqa: E731
    tr = f32(sign() * 10.0 ** rng.uniform(-3, 3, n))
    tz = f32(sign() * 10.0 ** rng.uniform(-3, 3, n))
    half_m = f32(rng.choice([0.5, 1.0, 2.0, 4.5], n))
    RD = rng.uniform(-2.0, 2.0, n)
    ZD = rng.uniform(-2.0, 2.0, n)
    # the tile box around a point where |alpha| is a few half-widths; for a third of the
    # draws that point lies far out along the line alpha = 0, where the two products that
    # make up alpha are large and cancel
    scale = half_m / (np.abs(tr) + np.abs(tz))
    far = np.where(rng.uniform(0, 1, n) < 1 / 3, 10.0 ** rng.uniform(1, 4, n), 0.0) * scale
    Rc = RD + rng.uniform(-3, 3, n) * scale + far * tz / (np.abs(tr) + np.abs(tz))
    Zc = ZD + rng.uniform(-3, 3, n) * scale - far * tr / (np.abs(tr) + np.abs(tz))
    w = scale * 10.0 ** rng.uniform(-2, -1, n)
    h = scale * 10.0 ** rng.uniform(-2, -1, n)
    return tr, tz, half_m, RD, ZD, Rc - w, Rc + w, Zc - h, Zc + h


def test_full_box_nodes_pass_the_support_test_at_every_pixel():
    rng = np.random.default_rng(20261203)
    n = 200_000
    tr, tz, half_m, RD, ZD, Rlo, Rhi, Zlo, Zhi = draw(rng, n)
    fl, fh = full_box(tr, tz, RD, ZD, Rlo, Rhi, Zlo, Zhi, half_m)
    ok = fl <= fh
    assert ok.mean() > 0.5  # most tiles much smaller than the support have a full box
    idx = np.nonzero(ok)[0]
    worst = 0.0
    # kappa on either edge of the full box (and just inside), pixels on the corners and inside
    kap_choices = [fl[idx], fh[idx], np.nextafter(fl[idx], fh[idx]), np.nextafter(fh[idx], fl[idx])]
    for kappa in kap_choices:
        pts = [(Rlo, Zlo), (Rlo, Zhi), (Rhi, Zlo), (Rhi, Zhi)]
        for _ in range(4):
            u, v = rng.uniform(0, 1, n), rng.uniform(0, 1, n)
            pts.append((Rlo + u * (Rhi - Rlo), Zlo + v * (Zhi - Zlo)))
        for R, Z in pts:
            y = walk_y(tr[idx], tz[idx], RD[idx], ZD[idx], R[idx], Z[idx], kappa.astype(np.float32))
            excess = np.abs(y) - half_m[idx]
            worst = max(worst, float(excess.max()))
            assert np.all(np.abs(y) <= half_m[idx]), float(excess.max())
    assert worst <= 0.0


def test_full_box_is_the_support_box_shrunk_by_the_tile_and_the_margin():
    """A tile of zero extent at the reflection's centre: the full box is [-m/2, m/2] shrunk by
    the margin alone; a tile as wide as the support in alpha has an empty full box."""
    one = lambda v: f32([v])  # noqa: E731
    fl, fh = full_box(one(1.0), one(0.0), 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, one(2.0))
    assert np.isclose(fl[0], -2.0 + 1e-3, rtol=0, atol=1e-6) and np.isclose(fh[0], 2.0 - 1e-3, rtol=0, atol=1e-6)
    fl, fh = full_box(one(1.0), one(0.0), 0.0, 0.0, -2.0, 2.0, 0.0, 0.0, one(2.0))
    assert fl[0] > fh[0]
