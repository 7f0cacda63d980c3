"""Seeded synthetic workloads shared by the oracle-side tests and the GPU path.

This module only draws random numbers and fills parameter records.  It holds
none of the method's arithmetic (no frames, no structure factors, no profile
evaluation); both the FP64 oracle and the HIP library consume the arrays it
returns unchanged.

The paper's own workloads are real polymer structures (cellulose, chitin,
cellulose triacetate, A-DNA) read from PDB files with small cells, a few
hundred reflections and an 800x800 detector (tutorial section, Tables
"unitcell", "experiment", "hkl", "paracrystal", "simulate").  Those files are
not available, so the seeded inputs below stand in for them at the sizes of
the benchmark configurations:

  0  tiny    10x10x20 A orthorhombic, 200 atoms, 4 A, 64^2 detector, Gaussian 5 deg
  1  medium  40x40x60 A beta=95 deg, 5000 atoms, 2 A, 1024^2, Voigt 3 deg eta=.5
  2  large   100x100x120 A, 50000 atoms, 1.5 A, 2048^2, Lorentzian 2 deg
  3  grad    config 1 plus a perturbed target model
  4  batch   256 ragged models

Random draws use numpy's PCG64 (``numpy.random.default_rng(seed)``) in the
order written in each generator.  Angles are radians, lengths Angstrom,
detector distance and pixel size millimetres.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

DEG = math.pi / 180.0

# Scattering-factor model used by every configuration: f(s) = Z exp(-s^2 / (2*0.6^2)),
# s = sin(theta)/lambda, written as the first term of a four-Gaussian-plus-constant
# table row (a1..a4, b1..b4, c) so that general tables fit the same layout.
FF_B = 1.0 / (2.0 * 0.6 * 0.6)


@dataclasses.dataclass
class Cell:
    a: float
    b: float
    c: float
    alpha: float
    beta: float
    gamma: float


@dataclasses.dataclass
class Geometry:
    wavelength: float      # Angstrom
    distance: float        # sample-detector distance, mm
    pixel: float           # pixel pitch, mm
    width: int             # pixels along the detector horizontal (lab y)
    height: int            # pixels along the detector vertical (lab z, fibre)
    center_x: float        # beam centre, pixel units
    center_y: float
    tilt: float = 0.0      # fibre axis tilted by this angle (rad) about lab y, toward +x
    tile_w: int = 0        # pixel tile width of the GPU launches (0: 8 x 8 tiles); no effect on the pattern
    mirror: int = 0        # GPU launch folds, bit 0: left-right (needs center_x = width/2); bit 1: up-down
                           # (needs center_y = height/2 and tilt 0)
    tile_waves: int = 0    # waves per tile of the GPU profile launch (0: the library's choice)
    unit_pairs: int = 0    # pairs per work unit of the balanced GPU launch (0: the library's choice)
    det_tilt: float = 0.0  # detector plane turned by this angle (rad) about its horizontal axis, its
                           # top toward the sample (0: normal to the beam)


@dataclasses.dataclass
class Disorder:
    sigma_theta: float     # Gaussian angular width, rad
    gamma_theta: float     # Lorentzian HWHM, rad
    N_base: tuple          # coherent cells along a, b, c
    g: tuple               # Hosemann g along a, b, c
    intensity_model: int = 1   # 1 = Hosemann intensity loss, 0 = none
    lineshape: int = 0         # per-axis peak form: 0 Laue (sinc^2), 1 Gaussian, 2 Hosemann
    B_axis: tuple = (0.0, 0.0, 0.0)  # axis-dependent Debye-Waller damping B_a, B_b, B_c (A^2)


@dataclasses.dataclass
class Quadrature:
    n_nodes: int           # nodes per side of the (d1,d2) grid
    T: float               # grid half extent in tangent-plane units
    sigma_r: float = 1e-4  # radial shell width, 1/A
    m: int = 3             # kernel zeros kept per lattice axis
    delta: float = 1e-5    # Lorentz regulariser, 1/A
    d_min: float = 2.0
    d_max: float = 30.0
    extinction: float = 30.0   # skip hkl with 2 pi^2 sum g_i^2 h_i^2 above this


@dataclasses.dataclass
class Atoms:
    x: np.ndarray          # fractional, float32 [n]
    y: np.ndarray
    z: np.ndarray
    B: np.ndarray          # isotropic B, A^2, float32
    occ: np.ndarray        # occupancy, float32
    type: np.ndarray       # int32 index into ff
    ff: np.ndarray         # float32 [n_types][9] = a1..a4, b1..b4, c

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


@dataclasses.dataclass
class Workload:
    name: str
    cell: Cell
    geom: Geometry
    dis: Disorder
    quad: Quadrature
    atoms: Atoms


def extent_T(sigma_theta: float, gamma_theta: float) -> float:
    """Node-grid half extent: tan(kappa*sqrt(sigma^2+gamma^2)), kappa = 4 for a
    pure Gaussian and 10 when a Lorentzian component is present (the extent is
    scaled by the combined width, section "Angular peak shapes").  Held fixed
    as an input afterwards."""
    kappa = 4.0 if gamma_theta == 0.0 else 10.0
    return math.tan(kappa * math.sqrt(sigma_theta * sigma_theta + gamma_theta * gamma_theta))


def voigt_split(sigma: float, eta: float):
    """Map a total width sigma and Lorentzian fraction eta onto the paper's
    (sigma_theta, gamma_theta) pair: sigma_theta=(1-eta)sigma, gamma_theta=eta sigma."""
    return (1.0 - eta) * sigma, eta * sigma


def ff_table(zs) -> np.ndarray:
    t = np.zeros((len(zs), 9), dtype=np.float32)
    for i, z in enumerate(zs):
        t[i, 0] = float(z)
        t[i, 4] = FF_B
    return t


def _atoms(rng, n, zs, probs, b_lo, b_hi) -> Atoms:
    frac = rng.random((n, 3))
    if probs is None:
        typ = rng.integers(0, len(zs), n)
    else:
        typ = rng.choice(len(zs), size=n, p=np.asarray(probs, dtype=np.float64))
    B = rng.uniform(b_lo, b_hi, n)
    return Atoms(
        x=np.ascontiguousarray(frac[:, 0], dtype=np.float32),
        y=np.ascontiguousarray(frac[:, 1], dtype=np.float32),
        z=np.ascontiguousarray(frac[:, 2], dtype=np.float32),
        B=B.astype(np.float32),
        occ=np.ones(n, dtype=np.float32),
        type=typ.astype(np.int32),
        ff=ff_table(zs),
    )


def config0() -> Workload:
    rng = np.random.default_rng(0)
    atoms = _atoms(rng, 200, (6, 7, 8), None, 10.0, 30.0)
    cell = Cell(10.0, 10.0, 20.0, 90 * DEG, 90 * DEG, 90 * DEG)
    st, gt = 5 * DEG, 0.0
    return Workload(
        "tiny: 10x10x20 A P1, 200 atoms, d_min 4 A, 64x64 px, Gaussian 5 deg, 16x16 nodes",
        cell, Geometry(1.0, 100.0, 0.5, 64, 64, 32.0, 32.0),
        Disorder(st, gt, (100.0 / 10.0, 100.0 / 10.0, 100.0 / 20.0), (0.0, 0.0, 0.0)),
        Quadrature(16, extent_T(st, gt), d_min=4.0), atoms)


def config1() -> Workload:
    rng = np.random.default_rng(1)
    atoms = _atoms(rng, 5000, (6, 7, 8, 16), (0.98 / 3, 0.98 / 3, 0.98 / 3, 0.02), 10.0, 40.0)
    cell = Cell(40.0, 40.0, 60.0, 90 * DEG, 95 * DEG, 90 * DEG)
    st, gt = voigt_split(3 * DEG, 0.5)
    return Workload(
        "medium: 40x40x60 A beta 95, 5000 atoms, d_min 2 A, 1024x1024 px, Voigt 3 deg eta .5, 64x64 nodes",
        cell, Geometry(1.0, 150.0, 0.1, 1024, 1024, 512.0, 512.0),
        Disorder(st, gt, (150.0 / 40.0, 150.0 / 40.0, 300.0 / 60.0), (0.03, 0.03, 0.0)),
        Quadrature(64, extent_T(st, gt), d_min=2.0), atoms)


def config2() -> Workload:
    rng = np.random.default_rng(2)
    atoms = _atoms(rng, 50000, (6, 7, 8, 16), (0.60, 0.17, 0.22, 0.01), 15.0, 50.0)
    cell = Cell(100.0, 100.0, 120.0, 90 * DEG, 90 * DEG, 90 * DEG)
    st, gt = 0.0, 2 * DEG
    return Workload(
        "large: 100x100x120 A, 50000 atoms, d_min 1.5 A, 2048x2048 px, Lorentzian 2 deg, 96x96 nodes",
        cell, Geometry(0.8, 200.0, 0.075, 2048, 2048, 1024.0, 1024.0),
        Disorder(st, gt, (200.0 / 100.0, 200.0 / 100.0, 500.0 / 120.0), (0.05, 0.05, 0.0)),
        Quadrature(96, extent_T(st, gt), d_min=1.5), atoms)


def config(i: int) -> Workload:
    return {0: config0, 1: config1, 2: config2}[i]()


@dataclasses.dataclass
class GradWorkload:
    """Refinement workload: the model being refined and the target model whose
    simulated pattern is the data."""
    model: Workload
    target: Workload


def config3() -> GradWorkload:
    """Config 1 as the model; the target perturbs it: coordinates by N(0, 0.1 A)
    per axis (drawn in fractional units as 0.1 A / edge length), B x 1.2,
    sigma 3.5 deg (eta .5), g_a = g_b = .035.  The target keeps the model's
    node-grid extent T."""
    model = config1()
    rng = np.random.default_rng(3)
    a = model.atoms
    n = a.n
    noise = rng.normal(0.0, 0.1, (n, 3))
    edges = np.array([model.cell.a, model.cell.b, model.cell.c])
    frac = np.stack([a.x, a.y, a.z], axis=1).astype(np.float64) + noise / edges
    st, gt = voigt_split(3.5 * DEG, 0.5)
    tatoms = Atoms(
        x=np.ascontiguousarray(frac[:, 0], dtype=np.float32),
        y=np.ascontiguousarray(frac[:, 1], dtype=np.float32),
        z=np.ascontiguousarray(frac[:, 2], dtype=np.float32),
        B=(a.B.astype(np.float64) * 1.2).astype(np.float32),
        occ=a.occ.copy(), type=a.type.copy(), ff=a.ff.copy())
    target = Workload(
        "target for the refinement workload", model.cell, model.geom,
        Disorder(st, gt, model.dis.N_base, (0.035, 0.035, 0.0)),
        dataclasses.replace(model.quad), tatoms)
    return GradWorkload(model, target)


def detector_distance(wavelength: float, d_min: float, side_px: int, pixel: float) -> float:
    """Detector distance rule of the tutorial (Eq. SF): the highest-angle
    reflection lands at 90% of the half detector."""
    two_theta = 2.0 * math.asin(wavelength / (2.0 * d_min))
    return 0.9 * side_px * pixel / (2.0 * math.tan(two_theta))


def config4(n_models: int = 256, seed: int = 4) -> List[Workload]:
    """Batch of ragged models.  Per model, in this order: three cell edges
    U(10,80) A, log-uniform atom count in [500, 20000], detector side
    64*U{4..16} px, sigma U(1,8) deg, eta U(0,1), g U(0,.06) (lateral), d_min U(2,3) A;
    then its atoms as in config 1."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_models):
        edges = rng.uniform(10.0, 80.0, 3)
        n_atoms = int(round(math.exp(rng.uniform(math.log(500.0), math.log(20000.0)))))
        side = 64 * int(rng.integers(4, 17))
        sigma = rng.uniform(1.0, 8.0) * DEG
        eta = rng.uniform(0.0, 1.0)
        g = rng.uniform(0.0, 0.06)
        d_min = rng.uniform(2.0, 3.0)
        atoms = _atoms(rng, n_atoms, (6, 7, 8, 16), (0.98 / 3, 0.98 / 3, 0.98 / 3, 0.02), 10.0, 40.0)
        st, gt = voigt_split(sigma, eta)
        cell = Cell(float(edges[0]), float(edges[1]), float(edges[2]), 90 * DEG, 90 * DEG, 90 * DEG)
        geom = Geometry(1.0, detector_distance(1.0, d_min, side, 0.1), 0.1, side, side, side / 2.0, side / 2.0)
        dis = Disorder(st, gt, (150.0 / edges[0], 150.0 / edges[1], 300.0 / edges[2]), (g, g, 0.0))
        out.append(Workload(f"batch model {i}", cell, geom, dis,
                            Quadrature(32, extent_T(st, gt), d_min=float(d_min)), atoms))
    return out


def small(seed: int, n_atoms: int = 24, width: int = 24, height: int = 20,
          cell: Optional[Cell] = None, sigma_theta: float = 4 * DEG, gamma_theta: float = 0.0,
          g=(0.0, 0.0, 0.0), n_nodes: int = 12, d_min: float = 5.0,
          size_A=(60.0, 60.0, 80.0), distance: float = 60.0, pixel: float = 0.8,
          center=None, tilt: float = 0.0, lineshape: int = 0, B_axis=(0.0, 0.0, 0.0),
          intensity_model: int = 1, det_tilt: float = 0.0) -> Workload:
    """Tiny seeded workload for oracle pins and parity edge cases (ragged detector
    sizes, off-centre beams, skewed cells)."""
    rng = np.random.default_rng(seed)
    atoms = _atoms(rng, n_atoms, (6, 7, 8), None, 5.0, 20.0)
    if cell is None:
        cell = Cell(9.0, 11.0, 13.0, 90 * DEG, 90 * DEG, 90 * DEG)
    if center is None:
        center = (width / 2.0, height / 2.0)
    N = (size_A[0] / cell.a, size_A[1] / cell.b, size_A[2] / cell.c)
    return Workload(
        f"small seed {seed}", cell,
        Geometry(1.0, distance, pixel, width, height, float(center[0]), float(center[1]), float(tilt),
                 det_tilt=float(det_tilt)),
        Disorder(sigma_theta, gamma_theta, N, tuple(g), intensity_model, lineshape, tuple(B_axis)),
        Quadrature(n_nodes, extent_T(sigma_theta, gamma_theta), d_min=d_min), atoms)


LINESHAPES = {"laue": 0, "gaussian": 1, "hosemann": 2}


def with_disorder(wl: Workload, **changes) -> Workload:
    """The same workload with some disorder fields replaced (lineshape, B_axis, ...)."""
    return dataclasses.replace(wl, dis=dataclasses.replace(wl.dis, **changes))


def with_tilt(wl: Workload, tilt: float) -> Workload:
    """The same workload with its fibre axis tilted by `tilt` (rad) toward the beam."""
    return dataclasses.replace(wl, name=f"{wl.name}, fibre tilt {math.degrees(tilt):.0f} deg",
                               geom=dataclasses.replace(wl.geom, tilt=float(tilt)))
