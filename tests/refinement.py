"""The refinement workload's loss restricted to a seeded pixel support, from the oracle alone.

The model is the medium workload; the target is its perturbed copy (coordinates N(0, 0.1 A),
B x 1.2, sigma 3.5 deg, g .035 lateral).  On a support S of 256 stratified pixels (strata.py:
128 strong, 16 meridian, 16 equator, 96 uniform; seed 3) the loss is
    L = sum_{q in S} w_q (I_q - T_q)^2,   w_q = 1/(T_q + 1e-3 max_S T),
with I the model's and T the target's oracle image (each over its own whole reflection list,
the extinction cull of its own g), so dL/dI_q = G_q = 2 w_q (I_q - T_q) on S and 0 elsewhere.
The 64 parameters of the finite-difference check: the 8 globals (sigma_theta, gamma_theta,
N_base (3), g (3)) and 56 seeded (atom, field) pairs, field in x, y, z (fractional), B, occ.
"""
from __future__ import annotations

import dataclasses

import numpy as np

import workloads as W
from oracle import oracle as O
from strata import stratified_pixels

COUNTS = {"strong": 128, "meridian": 16, "equator": 16, "uniform": 96}
SEED = 3
FIELDS = ("x", "y", "z", "B", "occ")


@dataclasses.dataclass
class Refinement:
    wl: object          # the model (medium workload)
    target: object      # the target workload
    hkl: np.ndarray     # the model's reflection list (extinction cull of its g)
    F: np.ndarray       # the model's structure factors (oracle C loop)
    P: object           # oracle prepared problem of the model
    q: np.ndarray       # flat pixel indices of the support
    R: np.ndarray       # ring coordinates of the support pixels
    Z: np.ndarray
    I: np.ndarray       # model image at the support
    T: np.ndarray       # target image at the support
    w: np.ndarray       # residual weights
    G: np.ndarray       # dL/dI at the support


def model_list(wl):
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    return np.ascontiguousarray(hkl[~O.extinct_mask(hkl, wl.dis, wl.quad.extinction)])


def build() -> Refinement:
    gw = W.config3()
    wl, tl = gw.model, gw.target
    hkl = model_list(wl)
    F = O.structure_factors_c(hkl, wl.cell, wl.atoms)
    P = O.prepare(wl, hkl=hkl, F=F, cull_extinct=False)
    pix = stratified_pixels(wl, P, COUNTS, SEED)
    q = np.array([p for p, _ in pix], dtype=np.int64)
    R, Z = O.pixel_rz(wl.geom)
    Rq, Zq = R.ravel()[q], Z.ravel()[q]
    I = O.pattern_at(P, Rq, Zq)
    T, _ = O.pattern_sampled(tl, Rq, Zq)
    w = 1.0 / (T + 1e-3 * T.max())
    G = 2.0 * w * (I - T)
    return Refinement(wl, tl, hkl, F, P, q, Rq, Zq, I, T, w, G)


def fd_parameters(n_atoms, n_pairs=56):
    """The 56 seeded (atom, field) pairs of the finite-difference check (seed 3)."""
    rng = np.random.default_rng(SEED)
    atoms = rng.choice(n_atoms, n_pairs, replace=False)
    fields = rng.integers(0, len(FIELDS), n_pairs)
    return [(int(a), FIELDS[int(f)]) for a, f in zip(atoms, fields)]
