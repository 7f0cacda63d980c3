"""Stratified pixel samples of a detector, chosen from the oracle alone (never from a GPU
image), for the full-size parity tests and the stored expected values under golden/.

Strata (pixel (i, j): column, row; row 0 at the bottom):
  strong    the detector pixels of the diffraction-condition rotations (Eqs. harmonic,
            solutions) of the reflections with the largest weights W = |F|^2 I_para
  meridian  the two columns next to the beam centre, random rows
  equator   the two rows next to the beam centre, random columns
  corners   a 4 x 4 block at each corner of the detector
  uniform   uniformly random pixels
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def stratified_pixels(wl, P, counts, seed):
    """[(flat pixel index j*W + i, stratum)] without repeats; P: the oracle's prepared problem
    over the whole reflection list (its weights W and reciprocal vectors D pick the strong
    pixels); counts: pixels per stratum (corners: at most 64)."""
    g = wl.geom
    Wd, H = g.width, g.height
    rng = np.random.default_rng(seed)
    taken, out = set(), []

    def add(i, j, name):
        i, j = int(i), int(j)
        q = j * Wd + i
        if 0 <= i < Wd and 0 <= j < H and q not in taken:
            taken.add(q)
            out.append((q, name))
            return True
        return False

    n = 0
    for r in np.argsort(-P.W, kind="stable"):
        if n >= counts.get("strong", 0):
            break
        for pos in O.ewald_project(P.D[r], g):
            x, y = pos[0]
            if np.isfinite(x) and np.isfinite(y) and n < counts["strong"] and add(round(x), round(y), "strong"):
                n += 1
    cx, cy = int(g.center_x), int(g.center_y)
    for name, draw in (("meridian", lambda: (cx - 1 + rng.integers(2), rng.integers(H))),
                       ("equator", lambda: (rng.integers(Wd), cy - 1 + rng.integers(2))),
                       ("uniform", lambda: (rng.integers(Wd), rng.integers(H)))):
        want = min(counts.get(name, 0), Wd * H - len(out))
        n = 0
        while n < want:
            n += add(*draw(), name)
    if counts.get("corners", 0):
        k = 0
        for ci, cj in ((0, 0), (Wd - 4, 0), (0, H - 4), (Wd - 4, H - 4)):
            for dj in range(4):
                for di in range(4):
                    if k < counts["corners"] and add(ci + di, cj + dj, "corners"):
                        k += 1
    return out
