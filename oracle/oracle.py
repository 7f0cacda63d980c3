"""FP64 CPU oracle of the fibre-diffraction profile-quadrature path.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers; the product library never imports,
links or runs anything here, and this module imports nothing from the
product package.

Plain, slow and written to be checked against the paper by eye: IEEE binary64
throughout, numpy for elementwise arrays (numpy does not fuse multiply-adds),
scipy.special.voigt_profile for the Voigt shape as the paper itself does (and
the Faddeeva function in mpmath's extended precision for its width
derivatives), and a
small C file (oracle_c.c, built with -ffp-contract=off) for the per-pixel
loops that are too slow in Python.

Steps, in the order of the method:
  frame             reciprocal basis            Eq. recip_basis, tutorial frame convention
  enumerate_hkl     reflection list             Eq. laue3d + resolution shell (tutorial, Table hkl)
  structure_factors F(hkl)                      Eq. structure_factor, isotropic Debye-Waller
  disorder_factors  A_i, N_eff, I_para          Eqs. Ah, Neff, Ipara
  reflection_frames S, e1, e2, e_perp           Eq. gnomonic (tangent vectors)
  node_table        (d1, d2) grid and weights   Eqs. gnomonic, node_weight; angular shapes
  pixel_rz          (R, Z) of each pixel        Eqs. laue, squared, harmonic (Ewald condition)
  pattern           detector image              Eqs. I_shape, direct_sum, lorentz
  culling_lists     per-tile reflection lists   (contract of the GPU path, exact predicate)
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import mpmath
import numpy as np
from scipy.special import voigt_profile

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_oracle_c.so")
_lib = None


def build_c(force: bool = True) -> str:
    """Compile oracle_c.c (plain C, OpenMP, no FMA contraction)."""
    src = os.path.join(_HERE, "oracle_c.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _c():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_c()
        _lib = ctypes.CDLL(_LIB_PATH)
    return _lib


# --------------------------------------------------------------------------- O1
def frame(cell):
    """Real and reciprocal basis (Eq. recip_basis) in the tutorial's laboratory
    frame: c along z, b in the yz-plane, a completing the cell with a_x > 0.
    Returns (avec, astar, V) with avec rows a, b, c and astar rows a*, b*, c*."""
    a, b, c = cell.a, cell.b, cell.c
    ca, cb, cg = math.cos(cell.alpha), math.cos(cell.beta), math.cos(cell.gamma)
    sa = math.sin(cell.alpha)
    cvec = np.array([0.0, 0.0, c])
    bvec = np.array([0.0, b * sa, b * ca])
    az = a * cb
    ay = a * (cg - ca * cb) / sa
    ax = math.sqrt(a * a - ay * ay - az * az)
    avec = np.array([ax, ay, az])

    def cross(u, v):
        return np.array([u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]])

    bxc = cross(bvec, cvec)
    V = (avec[0] * bxc[0] + avec[1] * bxc[1]) + avec[2] * bxc[2]
    astar = np.stack([bxc / V, cross(cvec, avec) / V, cross(avec, bvec) / V])
    return np.stack([avec, bvec, cvec]), astar, V


def recip_vectors(hkl, astar):
    """D = h a* + k b* + l c*, componentwise as (h a*_j + k b*_j) + l c*_j."""
    h = hkl[:, 0].astype(np.float64)
    k = hkl[:, 1].astype(np.float64)
    l = hkl[:, 2].astype(np.float64)
    D = np.empty((hkl.shape[0], 3))
    for j in range(3):
        D[:, j] = (h * astar[0, j] + k * astar[1, j]) + l * astar[2, j]
    return D


def q_of(D):
    """|D|^2 as (Dx^2 + Dy^2) + Dz^2."""
    return (D[:, 0] * D[:, 0] + D[:, 1] * D[:, 1]) + D[:, 2] * D[:, 2]


# --------------------------------------------------------------------------- O2
def enumerate_hkl(cell, d_min, d_max):
    """All (h,k,l) != 0 with d_min <= d <= d_max (1/d = |D|), both ends inclusive with
    a relative slack of 1e-9 on |D|^2, in ascending lexicographic order; d_max <= 0
    means no low-resolution limit.  Since h = D.a, |h| <= |a|/d_min bounds the search."""
    _, astar, _ = frame(cell)
    hm = int(math.floor(cell.a / d_min)) + 1
    km = int(math.floor(cell.b / d_min)) + 1
    lm = int(math.floor(cell.c / d_min)) + 1
    hs, ks, ls = np.meshgrid(np.arange(-hm, hm + 1), np.arange(-km, km + 1), np.arange(-lm, lm + 1), indexing="ij")
    cand = np.stack([hs.ravel(), ks.ravel(), ls.ravel()], axis=1).astype(np.int32)
    q = q_of(recip_vectors(cand, astar))
    t_hi = (1.0 / (d_min * d_min)) * (1.0 + 1e-9)
    keep = q <= t_hi
    if d_max > 0:
        t_lo = (1.0 / (d_max * d_max)) * (1.0 - 1e-9)
        keep &= q >= t_lo
    keep &= np.any(cand != 0, axis=1)
    return np.ascontiguousarray(cand[keep])


# --------------------------------------------------------------------------- O3
def structure_factors(hkl, cell, atoms, chunk=2048):
    """F_hkl = sum_j occ_j f_t(j)(s) exp(-B_j s^2) exp(2 pi i (h x_j + k y_j + l z_j))
    (Eq. structure_factor with the isotropic Debye-Waller factor of the section
    "Paracrystalline disorder", B = 8 pi^2 <u^2>), s = |D|/2 = sin(theta)/lambda,
    f_t(s) = sum_g a_g exp(-b_g s^2) + c.  The phase is reduced modulo one turn."""
    _, astar, _ = frame(cell)
    q = q_of(recip_vectors(hkl, astar))
    s2 = q / 4.0
    x = atoms.x.astype(np.float64)
    y = atoms.y.astype(np.float64)
    z = atoms.z.astype(np.float64)
    B = atoms.B.astype(np.float64)
    occ = atoms.occ.astype(np.float64)
    ff = atoms.ff.astype(np.float64)
    F = np.zeros(hkl.shape[0], dtype=np.complex128)
    for i0 in range(0, hkl.shape[0], chunk):
        sl = slice(i0, i0 + chunk)
        hh = hkl[sl].astype(np.float64)
        ss = s2[sl][:, None]
        f = np.zeros((hh.shape[0], ff.shape[0]))
        for t in range(ff.shape[0]):
            f[:, t] = ff[t, 8]
            for g in range(4):
                f[:, t] += ff[t, g] * np.exp(-ff[t, 4 + g] * s2[sl])
        phase = (hh[:, 0:1] * x[None, :] + hh[:, 1:2] * y[None, :]) + hh[:, 2:3] * z[None, :]
        phase = phase - np.floor(phase)
        amp = occ[None, :] * f[:, atoms.type] * np.exp(-B[None, :] * ss)
        F[sl] = (amp * np.cos(2 * np.pi * phase)).sum(axis=1) + 1j * (amp * np.sin(2 * np.pi * phase)).sum(axis=1)
    return F


def structure_factors_c(hkl, cell, atoms):
    """The same sum as structure_factors, as a plain C loop (OpenMP over reflections)
    for reflection lists too long for numpy."""
    _, astar, _ = frame(cell)
    hkl = np.ascontiguousarray(hkl, dtype=np.int32)
    s2 = np.ascontiguousarray(q_of(recip_vectors(hkl, astar)) / 4.0)
    cv = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    x, y, z, B, occ = cv(atoms.x), cv(atoms.y), cv(atoms.z), cv(atoms.B), cv(atoms.occ)
    typ = np.ascontiguousarray(atoms.type, dtype=np.int32)
    ff = cv(atoms.ff)
    re = np.zeros(hkl.shape[0])
    im = np.zeros(hkl.shape[0])
    vp = lambda a: ctypes.c_void_p(a.ctypes.data)
    _c().oracle_structure_factors(ctypes.c_int64(hkl.shape[0]), vp(hkl), vp(s2), ctypes.c_int64(x.shape[0]), vp(x), vp(y),
                                  vp(z), vp(B), vp(occ), vp(typ), ctypes.c_int32(ff.shape[0]), vp(ff), vp(re), vp(im))
    return re + 1j * im


# --------------------------------------------------------------------------- O4
PI2 = math.pi * math.pi


def extinction_arg(hkl, g):
    """2 pi^2 sum_i g_i^2 h_i^2, the exponent of prod_i A_i (Eq. Ah)."""
    h = hkl.astype(np.float64)
    t = (g[0] * g[0]) * (h[:, 0] * h[:, 0]) + (g[1] * g[1]) * (h[:, 1] * h[:, 1])
    t = t + (g[2] * g[2]) * (h[:, 2] * h[:, 2])
    return (2.0 * PI2) * t


def disorder_factors(hkl, dis):
    """Per reflection and axis: A_i = exp(-2 pi^2 g_i^2 h_i^2) (Eq. Ah),
    1/N_eff = 1/N_base + (1 - A)/(1 + A) (Eq. Neff), and
    I_para = prod_i 2 A_i/(1 + A_i^2) (Eq. Ipara; 1 when intensity_model is none)."""
    h = hkl.astype(np.float64)
    g = np.asarray(dis.g, dtype=np.float64)
    Nb = np.asarray(dis.N_base, dtype=np.float64)
    A = np.exp(-2.0 * PI2 * (g[None, :] ** 2) * h * h)
    N = 1.0 / (1.0 / Nb[None, :] + (1.0 - A) / (1.0 + A))
    if dis.intensity_model:
        Ip = np.prod(2.0 * A / (1.0 + A * A), axis=1)
    else:
        Ip = np.ones(hkl.shape[0])
    return A, N, Ip


def axis_damping(hkl, cell, B_axis):
    """Axis-dependent Debye-Waller damping of section "Paracrystalline disorder",
    D(S) = exp(-1/4 sum_i B_i (S.a_i/|a_i|)^2), evaluated at S = D_hkl."""
    avec, astar, _ = frame(cell)
    S = recip_vectors(hkl, astar)
    ex = np.zeros(hkl.shape[0])
    for i in range(3):
        ahat = avec[i] / np.linalg.norm(avec[i])
        ex = ex + B_axis[i] * (S @ ahat) ** 2
    return np.exp(-0.25 * ex)


def axis_profile(lineshape, N, u):
    """Per-axis peak of integral breadth 1/N (unit integral per lattice period, peak N),
    in the form selected by lineshape:
      0 Laue:     N sinc^2(N u)                                  (Eq. I_shape with N -> N_eff)
      1 Gaussian: N exp(-pi N^2 u^2)                             (matched integral breadth)
      2 Hosemann: (1 - A^2)/(1 - 2 A cos(2 pi u) + A^2), A = max(0, (N - 1)/(N + 1)),
                  Eq. Z with its breadth (1 - A)/(1 + A) (Eq. breadth) equal to 1/N."""
    N = np.asarray(N, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    if lineshape == 0:
        return N * np.sinc(N * u) ** 2
    if lineshape == 1:
        return N * np.exp(-math.pi * N * N * u * u)
    A = np.maximum(0.0, (N - 1.0) / (N + 1.0))
    return (1.0 - A * A) / (1.0 - 2.0 * A * np.cos(2.0 * math.pi * u) + A * A)


def support_half(lineshape, m, N):
    """Support half-width in u = a_i.(p - s) per axis: m/N (Laue, Gaussian) or half a
    lattice period (Hosemann, whose factor is periodic in u)."""
    N = np.asarray(N, dtype=np.float64)
    return np.full_like(N, 0.5) if lineshape == 2 else m / N


def extinct_mask(hkl, dis, limit):
    """Reflections whose paracrystalline intensity loss prod A_i is below exp(-limit)
    (and I_para below 8 exp(-limit)); the pattern skips them."""
    return extinction_arg(hkl, dis.g) > limit


# --------------------------------------------------------------------------- O5
def reflection_frames(D):
    """Unit vector S = D/r0, tangent vectors e1 = z x S/|z x S| (azimuthal),
    e2 = S x e1 (meridional) and the radial unit vector e_perp of D about the fibre
    axis z.  On the meridian (R_D = |D_xy| <= 1e-12) e1 = x x S/|x x S| and
    e_perp = sign(D_z) y, so the frames of D and -D are exact negatives."""
    n = D.shape[0]
    r0 = np.sqrt(q_of(D))
    S = D / r0[:, None]
    RD = np.sqrt(D[:, 0] * D[:, 0] + D[:, 1] * D[:, 1])
    e1 = np.zeros((n, 3))
    ep = np.zeros((n, 3))
    off = RD > 1e-12
    # z x D = (-D_y, D_x, 0), |z x D| = R_D
    e1[off, 0] = -D[off, 1] / RD[off]
    e1[off, 1] = D[off, 0] / RD[off]
    ep[off, 0] = D[off, 0] / RD[off]
    ep[off, 1] = D[off, 1] / RD[off]
    on = ~off
    # x x D = (0, -D_z, D_y), |x x D| = sqrt(D_y^2 + D_z^2)
    nrm = np.sqrt(D[on, 1] * D[on, 1] + D[on, 2] * D[on, 2])
    e1[on, 1] = -D[on, 2] / nrm
    e1[on, 2] = D[on, 1] / nrm
    ep[on, 1] = np.sign(D[on, 2])
    e2 = np.stack([S[:, 1] * e1[:, 2] - S[:, 2] * e1[:, 1],
                   S[:, 2] * e1[:, 0] - S[:, 0] * e1[:, 2],
                   S[:, 0] * e1[:, 1] - S[:, 1] * e1[:, 0]], axis=1)
    return r0, S, e1, e2, ep


# --------------------------------------------------------------------------- O6/O7
def angular_shape(delta, sigma_theta, gamma_theta):
    """Unit-peak angular weight g(delta) (section "Angular peak shapes"):
    Gaussian when gamma = 0, Lorentzian when sigma = 0, otherwise the Voigt profile
    divided by its value at zero, evaluated with scipy.special.voigt_profile."""
    delta = np.asarray(delta, dtype=np.float64)
    if sigma_theta == 0.0 and gamma_theta == 0.0:
        raise ValueError("sigma_theta and gamma_theta are both zero")
    if gamma_theta == 0.0:
        return np.exp(-delta * delta / (2.0 * sigma_theta * sigma_theta))
    if sigma_theta == 0.0:
        return gamma_theta * gamma_theta / (delta * delta + gamma_theta * gamma_theta)
    return voigt_profile(delta, sigma_theta, gamma_theta) / voigt_profile(0.0, sigma_theta, gamma_theta)


@dataclass
class Nodes:
    d1: np.ndarray
    d2: np.ndarray
    c: np.ndarray
    Delta: np.ndarray
    omega: np.ndarray
    h: float


def node_table(n, T, sigma_r, sigma_theta, gamma_theta):
    """Midpoint grid of n x n tangent-plane offsets on [-T, T]^2, node index
    k = i2*n + i1 with d_j = -T + (i_j + 1/2) h, h = 2T/n.  Each node carries
    omega = sigma_r sqrt(2 pi) g(Delta) c^3 h^2 with c = (1 + d1^2 + d2^2)^(-1/2)
    and Delta = arccos(c) (Eq. node_weight without the r0^2 factor, which is per
    reflection)."""
    h = 2.0 * T / n
    d = -T + (np.arange(n, dtype=np.float64) + 0.5) * h
    d1 = np.tile(d, n)
    d2 = np.repeat(d, n)
    rho2 = d1 * d1 + d2 * d2
    c = 1.0 / np.sqrt(1.0 + rho2)
    Delta = np.arccos(c)
    omega = sigma_r * math.sqrt(2.0 * math.pi) * angular_shape(Delta, sigma_theta, gamma_theta) * c ** 3 * h * h
    return Nodes(d1, d2, c, Delta, omega, h)


# --------------------------------------------------------------------------- O8
def pixel_S(geom):
    """Scattering vectors (S_x, S_y, S_z), arrays [H][W], of every pixel centre (lab frame).
    Pixel (i, j) (column, row; row 0 at the bottom) has detector coordinates
    y = (i + 1/2 - c_x) p, z = (j + 1/2 - c_y) p.  The detector is normal to the beam at
    distance SF, or turned by geom.det_tilt = d about its horizontal axis through the beam
    centre, its top toward the sample: the pixel then sits at X = (SF - z sin d, y, z cos d).
    Its outgoing direction X/|X| gives S = (X/|X| - x)/lambda, on the Ewald sphere (Eq. laue),
    written without cancellation as S = (-(X_y^2 + X_z^2)/(r (r + X_x)), X_y/r, X_z/r)/lambda."""
    W, H = geom.width, geom.height
    i = np.arange(W, dtype=np.float64)
    j = np.arange(H, dtype=np.float64)
    y = ((i + 0.5) - geom.center_x) * geom.pixel
    z = ((j + 0.5) - geom.center_y) * geom.pixel
    y, z = np.meshgrid(y, z)          # [H][W]
    SF = geom.distance
    dt = float(getattr(geom, "det_tilt", 0.0))
    sd, cd = math.sin(dt), math.cos(dt)
    Xx = SF - z * sd
    Xz = z * cd
    r = np.sqrt((Xx * Xx + y * y) + Xz * Xz)
    lam = geom.wavelength
    Sx = -(y * y + Xz * Xz) / ((r * (r + Xx)) * lam)
    Sy = y / (r * lam)
    Sz = Xz / (r * lam)
    return Sx, Sy, Sz


def pixel_rz(geom):
    """Ring coordinates (R, Z) of every pixel centre, arrays [H][W], from the pixels'
    scattering vectors S (pixel_S: a detector normal to the beam at distance SF, or tilted).
    (R, Z) are the cylindrical coordinates of S about the fibre axis n (Eq.
    cyl-average's coordinates): Z = S.n, R = |S - Z n|.  The fibre axis is z tilted
    by geom.tilt about the lab y axis (the detector horizontal), n = (sin t, 0, cos t);
    with m = (cos t, 0, -sin t), R = sqrt((S.m)^2 + S_y^2).  At tilt 0 this is
    R = sqrt(S_x^2 + S_y^2), Z = S_z."""
    Sx, Sy, Sz = pixel_S(geom)
    tilt = float(getattr(geom, "tilt", 0.0))
    st, ct = math.sin(tilt), math.cos(tilt)
    Z = Sx * st + Sz * ct
    Sm = Sx * ct - Sz * st
    R = np.sqrt(Sm * Sm + Sy * Sy)
    return R, Z


# --------------------------------------------------------------------------- prepared problem
@dataclass
class Prepared:
    hkl: np.ndarray
    F: np.ndarray
    W: np.ndarray        # |F|^2 * I_para * axis damping
    N: np.ndarray        # N_eff [n][3]
    A: np.ndarray
    Ip: np.ndarray
    D: np.ndarray
    r0: np.ndarray
    S: np.ndarray
    e1: np.ndarray
    e2: np.ndarray
    ep: np.ndarray
    avec: np.ndarray
    astar: np.ndarray
    nodes: Nodes
    m: int
    delta: float
    Dw: np.ndarray = None     # axis damping D(D_hkl)
    lineshape: int = 0


def prepare(wl, hkl=None, F=None, cull_extinct=True):
    """Run O1-O7 for a workload: reflection list, structure factors, disorder
    factors, frames and the node table.  Reflections removed by the extinction
    cull are dropped."""
    avec, astar, _ = frame(wl.cell)
    if hkl is None:
        hkl = enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    if cull_extinct:
        keep = ~extinct_mask(hkl, wl.dis, wl.quad.extinction)
        hkl = np.ascontiguousarray(hkl[keep])
        if F is not None:
            F = F[keep]
    if F is None:
        F = structure_factors(hkl, wl.cell, wl.atoms)
    A, N, Ip = disorder_factors(hkl, wl.dis)
    D = recip_vectors(hkl, astar)
    r0, S, e1, e2, ep = reflection_frames(D)
    nodes = node_table(wl.quad.n_nodes, wl.quad.T, wl.quad.sigma_r, wl.dis.sigma_theta, wl.dis.gamma_theta)
    Dw = axis_damping(hkl, wl.cell, getattr(wl.dis, "B_axis", (0.0, 0.0, 0.0)))
    W = (F.real * F.real + F.imag * F.imag) * Ip * Dw
    return Prepared(hkl, F, W, N, A, Ip, D, r0, S, e1, e2, ep, avec, astar, nodes, wl.quad.m, wl.quad.delta, Dw,
                    int(getattr(wl.dis, "lineshape", 0)))


class _Problem(ctypes.Structure):
    _fields_ = [("n_hkl", ctypes.c_int64), ("W", ctypes.c_void_p), ("N", ctypes.c_void_p),
                ("r0", ctypes.c_void_p), ("S", ctypes.c_void_p), ("e1", ctypes.c_void_p),
                ("e2", ctypes.c_void_p), ("ep", ctypes.c_void_p), ("astar", ctypes.c_void_p),
                ("avec", ctypes.c_void_p), ("n_nodes", ctypes.c_int64), ("d1", ctypes.c_void_p),
                ("d2", ctypes.c_void_p), ("omega", ctypes.c_void_p), ("m", ctypes.c_int32),
                ("delta", ctypes.c_double), ("use_skip", ctypes.c_int32), ("lineshape", ctypes.c_int32)]


def _c_problem(P: Prepared, use_skip: bool):
    keep = []

    def ptr(a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        return a.ctypes.data

    prob = _Problem(P.hkl.shape[0], ptr(P.W), ptr(P.N), ptr(P.r0), ptr(P.S), ptr(P.e1), ptr(P.e2),
                    ptr(P.ep), ptr(P.astar), ptr(P.avec), P.nodes.d1.shape[0], ptr(P.nodes.d1),
                    ptr(P.nodes.d2), ptr(P.nodes.omega), P.m, P.delta, 1 if use_skip else 0, P.lineshape)
    return prob, keep


def pattern_at(P: Prepared, R, Z, use_skip=True, count=False):
    """Image values at pixels with ring coordinates (R, Z) (flat arrays):
    L(R) sum_hkl W_hkl I_hkl(p*), p* = R e_perp + Z z (Eqs. direct_sum, lorentz)."""
    R = np.ascontiguousarray(np.ravel(R), dtype=np.float64)
    Z = np.ascontiguousarray(np.ravel(Z), dtype=np.float64)
    out = np.zeros(R.shape[0])
    n_ev = ctypes.c_int64(0)
    prob, keep = _c_problem(P, use_skip)
    lib = _c()
    lib.oracle_pattern(ctypes.byref(prob), ctypes.c_int64(R.shape[0]), ctypes.c_void_p(R.ctypes.data),
                       ctypes.c_void_p(Z.ctypes.data), ctypes.c_void_p(out.ctypes.data), ctypes.byref(n_ev))
    del keep
    if count:
        return out, int(n_ev.value)
    return out


def threads() -> int:
    """OpenMP threads of the compiled oracle loops."""
    return int(_c().oracle_threads())


def set_threads(n: int) -> None:
    """Set the OpenMP threads of the compiled oracle loops."""
    _c().oracle_set_threads(ctypes.c_int(int(n)))


def reachable(wl, hkl, R, Z):
    """Ascending indices of the reflections of hkl (extinction cull already applied) whose
    support can reach the query point of at least one pixel with ring coordinates (R, Z):
    the complement of the exact skip of oracle_pattern, which needs no structure factors.
    The pattern at those pixels over these reflections alone equals the pattern over all of
    hkl bit for bit (same terms, same ascending order)."""
    hkl = np.ascontiguousarray(hkl)
    P = prepare(wl, hkl=hkl, F=np.zeros(hkl.shape[0], dtype=np.complex128), cull_extinct=False)
    R = np.ascontiguousarray(np.ravel(R), dtype=np.float64)
    Z = np.ascontiguousarray(np.ravel(Z), dtype=np.float64)
    mask = np.zeros(hkl.shape[0], dtype=np.uint8)
    prob, keep = _c_problem(P, True)
    _c().oracle_reach(ctypes.byref(prob), ctypes.c_int64(R.shape[0]), ctypes.c_void_p(R.ctypes.data),
                      ctypes.c_void_p(Z.ctypes.data), ctypes.c_void_p(mask.ctypes.data))
    del keep
    return np.nonzero(mask)[0]


def pattern_sampled(wl, R, Z, hkl=None, count=False):
    """The image at pixels with ring coordinates (R, Z) over the workload's whole reflection
    list (extinction cull applied): the reachable reflections' structure factors from the
    C loop, then oracle_pattern with its exact skip.  Returns (values, reflection indices
    used, evaluations if count)."""
    if hkl is None:
        hkl = enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
        hkl = np.ascontiguousarray(hkl[~extinct_mask(hkl, wl.dis, wl.quad.extinction)])
    sub = reachable(wl, hkl, R, Z)
    hs = np.ascontiguousarray(hkl[sub])
    P = prepare(wl, hkl=hs, F=structure_factors_c(hs, wl.cell, wl.atoms), cull_extinct=False)
    res = pattern_at(P, R, Z, count=count)
    if count:
        return res[0], sub, res[1]
    return res, sub


def profile_table(P: Prepared, R, Z, use_skip=False):
    """Per-reflection shell-quadrature profiles I_hkl(p*) at each pixel, [n_pix][n_hkl]
    (with use_skip, 0 for the reflections the exact skip rules out, the value the profile
    has there)."""
    R = np.ascontiguousarray(np.ravel(R), dtype=np.float64)
    Z = np.ascontiguousarray(np.ravel(Z), dtype=np.float64)
    out = np.zeros((R.shape[0], P.hkl.shape[0]))
    prob, keep = _c_problem(P, use_skip)
    _c().oracle_profile_table(ctypes.byref(prob), ctypes.c_int64(R.shape[0]), ctypes.c_void_p(R.ctypes.data),
                              ctypes.c_void_p(Z.ctypes.data), ctypes.c_void_p(out.ctypes.data))
    del keep
    return out


def pattern(wl, P: Prepared = None, use_skip=True, count=False):
    """Full detector image [H][W] (row 0 at the bottom)."""
    if P is None:
        P = prepare(wl)
    R, Z = pixel_rz(wl.geom)
    res = pattern_at(P, R, Z, use_skip=use_skip, count=count)
    if count:
        img, n = res
        return img.reshape(R.shape), n
    return res.reshape(R.shape)


# --------------------------------------------------------------------------- adjoint
def _voigt_width_derivs(delta, sigma, gamma, digits=50):
    """(d g/d sigma, d g/d gamma) of the unit-peak Voigt g = Re w(z)/Re w(z0) at one angle,
    z = (delta + i gamma)/(sigma sqrt 2), z0 = i gamma/(sigma sqrt 2), evaluated entirely in
    mpmath with `digits` significant digits: w(z) = exp(-z^2) erfc(-i z), w'(z) = -2 z w(z) +
    2 i/sqrt(pi), dz/dsigma = -z/sigma, dz/dgamma = i/(sigma sqrt 2), d Re w = Re(w' dz), and
    the quotient rule.  Near the Lorentzian limit the quotient rule cancels terms of size sigma
    to a result of size sigma^3, and w' cancels two terms of size 1 to |z|^-2; fifty digits keep
    the result exact to double precision for sigma/gamma and |z|^-1 down to about 1e-15."""
    with mpmath.workdps(digits):
        s, g, d = mpmath.mpf(sigma), mpmath.mpf(gamma), mpmath.mpf(delta)
        k = 1 / (s * mpmath.sqrt(2))
        c = 2j / mpmath.sqrt(mpmath.pi)

        def w_and_wp(z):
            w = mpmath.exp(-z * z) * mpmath.erfc(-1j * z)
            return w, -2 * z * w + c

        z, z0 = mpmath.mpc(d * k, g * k), mpmath.mpc(0, g * k)
        w, wp = w_and_wp(z)
        w0, wp0 = w_and_wp(z0)
        u, v = mpmath.re(w), mpmath.re(w0)
        du_s, dv_s = mpmath.re(wp * (-z / s)), mpmath.re(wp0 * (-z0 / s))
        du_g, dv_g = mpmath.re(wp * 1j * k), mpmath.re(wp0 * 1j * k)
        return float((du_s * v - u * dv_s) / (v * v)), float((du_g * v - u * dv_g) / (v * v))


def angular_shape_derivs(delta, sigma_theta, gamma_theta):
    """d g/d sigma_theta and d g/d gamma_theta of the unit-peak angular weight (section
    "Angular peak shapes"), in closed form.

    Voigt: g = Re w(z)/Re w(z0) with z = (delta + i gamma)/(sigma sqrt 2), z0 = i gamma/(sigma
    sqrt 2) and w the Faddeeva function, whose derivative is w'(z) = -2 z w(z) + 2 i/sqrt(pi);
    dz/dsigma = -z/sigma and dz/dgamma = i/(sigma sqrt 2), so d Re w(z) = Re(w'(z) dz), and the
    quotient rule gives both derivatives (in extended precision, _voigt_width_derivs).
    Gaussian (gamma = 0): dg/dsigma = g delta^2/sigma^3; dg/dgamma is the one-sided derivative
    of the Voigt at gamma = 0+, the Voigt formula above evaluated at gamma = 0.
    Lorentzian (sigma = 0): dg/dgamma = 2 gamma delta^2/(delta^2 + gamma^2)^2; the Voigt is a
    smooth function of sigma^2 (the Lorentzian convolved with a Gaussian of variance sigma^2),
    so dg/dsigma = 0 there."""
    delta = np.asarray(delta, dtype=np.float64)
    s, g = float(sigma_theta), float(gamma_theta)
    if s == 0.0 and g == 0.0:
        raise ValueError("sigma_theta and gamma_theta are both zero")
    if s == 0.0:
        den = delta * delta + g * g
        return np.zeros_like(delta), 2.0 * g * delta * delta / (den * den)
    vals, inverse = np.unique(delta.ravel(), return_inverse=True)   # node angles repeat by symmetry
    d = np.array([_voigt_width_derivs(x, s, g) for x in vals])
    d_sigma = d[:, 0][inverse].reshape(delta.shape)
    d_gamma = d[:, 1][inverse].reshape(delta.shape)
    if g == 0.0:
        gau = np.exp(-delta * delta / (2.0 * s * s))
        return gau * delta * delta / (s * s * s), d_gamma
    return d_sigma, d_gamma


def node_weight_derivs(nodes: Nodes, sigma_r, sigma_theta, gamma_theta):
    """d omega/d sigma_theta and d omega/d gamma_theta (Eq. node_weight, T held fixed)."""
    dgs, dgg = angular_shape_derivs(nodes.Delta, sigma_theta, gamma_theta)
    base = sigma_r * math.sqrt(2.0 * math.pi) * nodes.c ** 3 * nodes.h * nodes.h
    return base * dgs, base * dgg


def grad_sums(P: Prepared, domega_ds, domega_dg, R, Z, G, use_skip=True):
    """Per reflection: [dL/dW, sum W-free terms for sigma, gamma, N_a, N_b, N_c] of
    L = sum_q G_q P_q over the pixels listed by (R, Z, G) (see oracle_grad_sums)."""
    R = np.ascontiguousarray(np.ravel(R), dtype=np.float64)
    Z = np.ascontiguousarray(np.ravel(Z), dtype=np.float64)
    G = np.ascontiguousarray(np.ravel(G), dtype=np.float64)
    ds = np.ascontiguousarray(domega_ds, dtype=np.float64)
    dg = np.ascontiguousarray(domega_dg, dtype=np.float64)
    out = np.zeros((P.hkl.shape[0], 6))
    prob, keep = _c_problem(P, use_skip)
    vp = lambda a: ctypes.c_void_p(a.ctypes.data)
    _c().oracle_grad_sums(ctypes.byref(prob), vp(ds), vp(dg), ctypes.c_int64(R.shape[0]), vp(R), vp(Z), vp(G), vp(out))
    del keep
    return out


def sf_adjoint(hkl, cell, atoms, F, dF2):
    """Gradients of L through |F|^2 with dL/d|F|^2 = dF2 per reflection, for each atom:
    d|F|^2/dx_j = 2 Re(F* dF/dx_j), dF/dx_j = 2 pi i h t_j (fractional x; likewise y with k,
    z with l), dF/dB_j = -s^2 t_j, dF/docc_j = t_j/occ_j, t_j = occ_j f_j(s) exp(-B_j s^2)
    exp(2 pi i (h x_j + k y_j + l z_j)) (Eq. structure_factor)."""
    _, astar, _ = frame(cell)
    s2 = q_of(recip_vectors(hkl, astar)) / 4.0
    x, y, z = (atoms.x.astype(np.float64), atoms.y.astype(np.float64), atoms.z.astype(np.float64))
    B, occ, ff = atoms.B.astype(np.float64), atoms.occ.astype(np.float64), atoms.ff.astype(np.float64)
    n = x.shape[0]
    out = {k: np.zeros(n) for k in ("x", "y", "z", "B", "occ")}
    for i0 in range(0, hkl.shape[0], 1024):
        sl = slice(i0, i0 + 1024)
        hh = hkl[sl].astype(np.float64)
        f = np.zeros((hh.shape[0], ff.shape[0]))
        for t in range(ff.shape[0]):
            f[:, t] = ff[t, 8]
            for g in range(4):
                f[:, t] += ff[t, g] * np.exp(-ff[t, 4 + g] * s2[sl])
        phase = (hh[:, 0:1] * x[None, :] + hh[:, 1:2] * y[None, :]) + hh[:, 2:3] * z[None, :]
        phase = phase - np.floor(phase)
        t_over_occ = f[:, atoms.type] * np.exp(-B[None, :] * s2[sl][:, None]) * np.exp(2j * np.pi * phase)
        Fc = np.conj(F[sl])[:, None]
        w = dF2[sl][:, None]
        prod = Fc * t_over_occ             # F* t_j / occ_j
        out["x"] += np.sum(w * 2.0 * np.real(2j * np.pi * hh[:, 0:1] * prod), axis=0) * occ
        out["y"] += np.sum(w * 2.0 * np.real(2j * np.pi * hh[:, 1:2] * prod), axis=0) * occ
        out["z"] += np.sum(w * 2.0 * np.real(2j * np.pi * hh[:, 2:3] * prod), axis=0) * occ
        out["B"] += np.sum(w * 2.0 * np.real(-s2[sl][:, None] * prod), axis=0) * occ
        out["occ"] += np.sum(w * 2.0 * np.real(prod), axis=0)
    return out


def gradients(wl, P: Prepared, G, R=None, Z=None, use_skip=True):
    """Gradients of L = sum_pixels G * image with respect to the atoms (fractional x, y, z,
    B, occupancy) and the globals sigma_theta, gamma_theta, N_base (3), g (3), B_axis (3),
    with T held fixed.  Chain: W = |F|^2 I_para D, N_eff from Eq. Neff, I_para from Eq.
    Ipara, A_i = exp(-2 pi^2 g_i^2 h_i^2) (Eq. Ah), D the axis damping; the lineshape's
    dependence on N_eff enters through the per-reflection sums."""
    if R is None:
        R, Z = pixel_rz(wl.geom)
    nd = P.nodes
    ds, dg = node_weight_derivs(nd, wl.quad.sigma_r, wl.dis.sigma_theta, wl.dis.gamma_theta)
    sums = grad_sums(P, ds, dg, R, Z, G, use_skip=use_skip)
    dW = sums[:, 0]
    d_sigma = float(np.sum(P.W * sums[:, 1]))
    d_gamma = float(np.sum(P.W * sums[:, 2]))
    dN = P.W[:, None] * sums[:, 3:6]                       # dL/dN_eff per reflection and axis
    Nb = np.asarray(wl.dis.N_base, dtype=np.float64)
    d_Nbase = np.sum(dN * P.N ** 2 / Nb[None, :] ** 2, axis=0)
    F2 = P.F.real ** 2 + P.F.imag ** 2
    Dw = P.Dw if P.Dw is not None else np.ones_like(F2)
    dIp = dW * F2 * Dw
    A = P.A
    dN_dA = 2.0 * P.N ** 2 / (1.0 + A) ** 2
    dA = dN * dN_dA
    if wl.dis.intensity_model:
        dA = dA + (dIp * P.Ip)[:, None] * (1.0 - A * A) / (A * (1.0 + A * A))
    g = np.asarray(wl.dis.g, dtype=np.float64)
    h2 = P.hkl.astype(np.float64) ** 2
    d_g = np.sum(dA * (-4.0 * PI2 * g[None, :] * h2 * A), axis=0)
    # axis damping: dW/dB_i = -W (S.a_i/|a_i|)^2 / 4
    avec = P.avec
    d_B = np.zeros(3)
    for i in range(3):
        ahat = avec[i] / np.linalg.norm(avec[i])
        d_B[i] = np.sum(dW * P.W * (-0.25) * (P.D @ ahat) ** 2)
    # reflections with dL/dW = 0 add nothing to the atom sums
    nz = np.nonzero(dW)[0]
    atom = sf_adjoint(np.ascontiguousarray(P.hkl[nz]), wl.cell, wl.atoms, P.F[nz], (dW * P.Ip * Dw)[nz])
    return {"atoms": atom, "sigma_theta": d_sigma, "gamma_theta": d_gamma, "N_base": d_Nbase, "g": d_g,
            "B_axis": d_B, "dW": dW, "sums": sums}


# --------------------------------------------------------------------------- forward splat
class _SplatParams(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("SF", ctypes.c_double), ("pixel", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("st", ctypes.c_double), ("ct", ctypes.c_double),
                ("sd", ctypes.c_double), ("cd", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("n_r", ctypes.c_int32), ("n_s", ctypes.c_int32),
                ("dr", ctypes.c_void_p), ("Ts", ctypes.c_void_p)]


def splat_extents(wl, hkl):
    """Per reflection, the sampling box of the forward splat: radial half-extent dr and
    tangent-plane half-extent Ts.  dr = sum_i w_i |a*_i| is the corner radius of the support
    box, with w_i the culling contract's bound on the support half-width (m/N_i bounded
    without transcendentals, or 1/2 for the Hosemann lineshape); Ts = min(T + 2 dr/r0, 10)
    widens the node patch by the support.  +, -, *, /, sqrt only, in a fixed order."""
    _, astar, _ = frame(wl.cell)
    D = recip_vectors(hkl, astar)
    r0 = np.sqrt((D[:, 0] * D[:, 0] + D[:, 1] * D[:, 1]) + D[:, 2] * D[:, 2])
    rb_w = _support_bounds(wl, hkl)
    dr = rb_w[:, 0] * math.sqrt((astar[0, 0] * astar[0, 0] + astar[0, 1] * astar[0, 1]) + astar[0, 2] * astar[0, 2])
    dr = dr + rb_w[:, 1] * math.sqrt((astar[1, 0] * astar[1, 0] + astar[1, 1] * astar[1, 1]) + astar[1, 2] * astar[1, 2])
    dr = dr + rb_w[:, 2] * math.sqrt((astar[2, 0] * astar[2, 0] + astar[2, 1] * astar[2, 1]) + astar[2, 2] * astar[2, 2])
    Ts = np.minimum(wl.quad.T + 2.0 * dr / r0, 10.0)
    return dr, Ts


def splat(wl, P: Prepared, n_r, n_s, count=False):
    """Deterministic forward splat of every reflection of P onto the detector (see
    oracle_splat): image [H][W] of sum over samples of W I(S) L(R_S) dV, deposited at both
    diffraction-condition rotations of each sample."""
    g = wl.geom
    dr, Ts = splat_extents(wl, P.hkl)
    dr = np.ascontiguousarray(dr)
    Ts = np.ascontiguousarray(Ts)
    tilt = float(getattr(g, "tilt", 0.0))
    dt = float(getattr(g, "det_tilt", 0.0))
    sp = _SplatParams(g.wavelength, g.distance, g.pixel, g.center_x, g.center_y, math.sin(tilt), math.cos(tilt),
                      math.sin(dt), math.cos(dt), g.width, g.height, int(n_r), int(n_s), dr.ctypes.data, Ts.ctypes.data)
    img = np.zeros(g.width * g.height)
    n_ev = ctypes.c_int64(0)
    prob, keep = _c_problem(P, False)
    _c().oracle_splat(ctypes.byref(prob), ctypes.byref(sp), ctypes.c_void_p(img.ctypes.data), ctypes.byref(n_ev))
    del keep
    img = img.reshape(g.height, g.width)
    return (img, int(n_ev.value)) if count else img


def splat_project(S, geom):
    """Detector pixels (column, row; fractional, pixel centres at integer + 1/2 from the
    pixel's lower edge) of the two diffraction-condition rotations of fibre-frame points S,
    by the algebraic form used by the splat (see oracle_splat); both coordinates NaN where
    no rotation satisfies the condition (Eq. valid) or the diffracted ray runs away from the
    detector plane (D = k_x cos d + k_z sin d <= 0 with d the detector tilt, which
    oracle_splat skips as well).  The outgoing ray t k_out meets the plane (normal
    (cos d, 0, sin d) through (SF, 0, 0)) at detector coordinates y = SF k_y cos d / D,
    z = SF k_z / D."""
    S = np.atleast_2d(np.asarray(S, dtype=np.float64))
    tilt = float(getattr(geom, "tilt", 0.0))
    st, ct = math.sin(tilt), math.cos(tilt)
    q = (S[:, 0] * S[:, 0] + S[:, 1] * S[:, 1]) + S[:, 2] * S[:, 2]
    sx = -(geom.wavelength * q) / 2.0
    sz = (S[:, 2] - sx * st) / ct
    sy2 = (q - sx * sx) - sz * sz
    with np.errstate(invalid="ignore"):
        sy = np.where(sy2 >= 0.0, np.sqrt(sy2), np.nan)
    kx = 1.0 / geom.wavelength + sx
    # the detector plane, normal (cos d, 0, sin d) through (SF, 0, 0), met by t k_out
    dt = float(getattr(geom, "det_tilt", 0.0))
    sd, cd = math.sin(dt), math.cos(dt)
    D = kx * cd + sz * sd
    bad = ~(sy2 >= 0.0) | ~(D > 0.0)
    out = []
    for sgn in (1.0, -1.0):
        y = geom.distance * (sgn * sy) * cd / D
        z = geom.distance * sz / D
        o = np.stack([y / geom.pixel + geom.center_x, z / geom.pixel + geom.center_y], axis=1)
        o[bad] = np.nan
        out.append(o)
    return out[0], out[1]


# --------------------------------------------------------------------------- cylindrical average
def cyl_at(P: Prepared, R, Z, arc, use_skip=True, count=False):
    """Exact cylindrical average (Eq. cyl-average) of the pattern at pixels with ring
    coordinates (R, Z), by the periodic trapezoid rule over the ring with arc step `arc`
    (see oracle_cyl)."""
    R = np.ascontiguousarray(np.ravel(R), dtype=np.float64)
    Z = np.ascontiguousarray(np.ravel(Z), dtype=np.float64)
    out = np.zeros(R.shape[0])
    n_ev = ctypes.c_int64(0)
    prob, keep = _c_problem(P, use_skip)
    _c().oracle_cyl(ctypes.byref(prob), ctypes.c_int64(R.shape[0]), ctypes.c_void_p(R.ctypes.data),
                    ctypes.c_void_p(Z.ctypes.data), ctypes.c_double(arc), ctypes.c_void_p(out.ctypes.data),
                    ctypes.byref(n_ev))
    del keep
    return (out, int(n_ev.value)) if count else out


def profile_points(P: Prepared, ridx, points):
    """W_h I_h(p) for reflection ridx[k] at Cartesian points[k] (Eq. direct_sum, one
    reflection's term of the pattern sum before the Lorentz factor; see oracle_profile_points)."""
    ridx = np.ascontiguousarray(np.ravel(ridx), dtype=np.int32)
    pts = np.ascontiguousarray(np.reshape(points, (-1, 3)), dtype=np.float64)
    out = np.zeros(pts.shape[0])
    prob, keep = _c_problem(P, False)
    _c().oracle_profile_points(ctypes.byref(prob), ctypes.c_int64(pts.shape[0]), ctypes.c_void_p(ridx.ctypes.data),
                               ctypes.c_void_p(pts.ctypes.data), ctypes.c_void_p(out.ctypes.data))
    del keep
    return out


def cyl_boxes(wl, hkl):
    """Culling description for the cylindrical average, in the layout of reflection_boxes:
    every query point that a ring point at any azimuth can reach lies in the ball of radius
    rho_B = 2 r0 sqrt((1 - c_min)/2) + rho about D (the nodes lie within the great-circle
    angle arccos(c_min) of S; rho = sum_i w_i |a*_i| bounds the support), so its ring
    coordinates satisfy |R - R_D| <= rho_B and |Z - Z_D| <= rho_B, and |p| is within rho of
    r0.  No wedge.  +, -, *, /, sqrt only."""
    _, astar, _ = frame(wl.cell)
    D = recip_vectors(hkl, astar)
    r0 = np.sqrt((D[:, 0] * D[:, 0] + D[:, 1] * D[:, 1]) + D[:, 2] * D[:, 2])
    RD = np.sqrt(D[:, 0] * D[:, 0] + D[:, 1] * D[:, 1])
    T = wl.quad.T
    cmin = 1.0 / math.sqrt(1.0 + 2.0 * T * T)
    w = _support_bounds(wl, hkl)
    rho = w[:, 0] * math.sqrt((astar[0, 0] * astar[0, 0] + astar[0, 1] * astar[0, 1]) + astar[0, 2] * astar[0, 2])
    rho = rho + w[:, 1] * math.sqrt((astar[1, 0] * astar[1, 0] + astar[1, 1] * astar[1, 1]) + astar[1, 2] * astar[1, 2])
    rho = rho + w[:, 2] * math.sqrt((astar[2, 0] * astar[2, 0] + astar[2, 1] * astar[2, 1]) + astar[2, 2] * astar[2, 2])
    rB = (2.0 * r0) * math.sqrt((1.0 - cmin) / 2.0) + rho
    out = np.zeros((hkl.shape[0], 13))
    out[:, 0], out[:, 1] = RD - rB, RD + rB
    out[:, 2], out[:, 3] = D[:, 2] - rB, D[:, 2] + rB
    a_lo, a_hi = r0 - rho, r0 + rho
    out[:, 4] = np.where(a_lo > 0.0, a_lo * a_lo, 0.0)
    out[:, 5] = a_hi * a_hi
    out[:, 6:12] = [0.0, 0.0, -1.0, 0.0, 0.0, -1.0]
    ext_lim = wl.quad.extinction
    alive = ~((ext_lim > 0) & (extinction_arg(hkl, wl.dis.g) > ext_lim))
    out[:, 12] = alive.astype(np.float64)
    return out


# --------------------------------------------------------------------------- culling contract
def _support_bounds(wl, hkl):
    """Per reflection and axis, the culling contract's upper bound on the support half-width
    in u: m (1/N_base + min(pi^2 g^2 h^2, 1)), or 1/2 for the Hosemann lineshape."""
    h = hkl.astype(np.float64)
    m = float(wl.quad.m)
    mN = np.empty((hkl.shape[0], 3))
    for i in range(3):
        g = wl.dis.g[i]
        t = PI2 * (g * g) * (h[:, i] * h[:, i])
        mN[:, i] = m * (1.0 / wl.dis.N_base[i] + np.minimum(t, 1.0))
    if getattr(wl.dis, "lineshape", 0) == 2:
        mN[:] = 0.5
    return mN


def tile_boxes(geom, tile_w=8, tile_h=8):
    """Per tile of tile_w x tile_h pixels (clipped at the detector edge), the ranges
    of R, Z and R^2 + Z^2 over its pixel centres: [n_tiles_y][n_tiles_x][6] =
    (R_lo, R_hi, Z_lo, Z_hi, P2_lo, P2_hi)."""
    R, Z = pixel_rz(geom)
    P2 = R * R + Z * Z
    H, W = R.shape
    ny, nx = (H + tile_h - 1) // tile_h, (W + tile_w - 1) // tile_w
    box = np.zeros((ny, nx, 6))
    for ty in range(ny):
        for tx in range(nx):
            sl = (slice(ty * tile_h, (ty + 1) * tile_h), slice(tx * tile_w, (tx + 1) * tile_w))
            box[ty, tx] = (R[sl].min(), R[sl].max(), Z[sl].min(), Z[sl].max(), P2[sl].min(), P2[sl].max())
    return box


def reflection_boxes(wl, hkl):
    """Conservative description of the query points a reflection can reach, as
    the 13 numbers (R_lo, R_hi, Z_lo, Z_hi, P2_lo, P2_hi, n1R, n1Z, rho1, n2R, n2Z,
    rho2, alive) per reflection.

    Nodes s = r0 c (S + d1 e1 + d2 e2) have |d_j| <= T and c in [c_min, 1] with
    c_min = (1 + 2T^2)^(-1/2); a query point p lies in the support box
    {x : |a_i.x| <= w_i} of some node, whose extent along a unit vector v is
    sum_i w_i |a*_i.v|.  For the Laue and Gaussian lineshapes w_i = m/N_i, with 1/N_i
    bounded without transcendentals by 1/N_base,i + min(pi^2 g_i^2 h_i^2, 1) (since
    tanh(t) <= min(t, 1)); for the Hosemann lineshape w_i = 1/2.  Hence:
      - (R, Z) box: s.v over the node set, widened by the support extent, v = e_perp, z;
      - annulus: |s| = r0, so |p| is within sum_i (m/N_i)|a*_i| of r0;
      - wedge (reflections off the meridian): in the (R, Z) plane every node lies in
        the cone spanned by S + d2 e2, |d2| <= T, so p lies on the inner side of each
        edge line up to the support extent along that edge's normal.
    All arithmetic is +, -, *, /, sqrt in a fixed order (reproducible bit for bit)."""
    _, astar, _ = frame(wl.cell)
    D = recip_vectors(hkl, astar)
    r0, S, e1, e2, ep = reflection_frames(D)
    RD = np.sqrt(D[:, 0] * D[:, 0] + D[:, 1] * D[:, 1])
    merid = ~(RD > 1e-12)
    T = wl.quad.T
    m = float(wl.quad.m)
    cmin = 1.0 / math.sqrt(1.0 + 2.0 * T * T)
    n = hkl.shape[0]
    mN = _support_bounds(wl, hkl)
    ez = np.zeros_like(ep)
    ez[:, 2] = 1.0

    def dot(u, v):
        return (u[:, 0] * v[:, 0] + u[:, 1] * v[:, 1]) + u[:, 2] * v[:, 2]

    def ext(v):
        e = mN[:, 0] * np.abs(dot(np.broadcast_to(astar[0], v.shape), v))
        e = e + mN[:, 1] * np.abs(dot(np.broadcast_to(astar[1], v.shape), v))
        e = e + mN[:, 2] * np.abs(dot(np.broadcast_to(astar[2], v.shape), v))
        return e

    def span(v):
        l0, l1, l2 = dot(S, v), dot(e1, v), dot(e2, v)
        spread = T * (np.abs(l1) + np.abs(l2))
        lo, hi = l0 - spread, l0 + spread
        s_lo = r0 * np.minimum(cmin * lo, lo)
        s_hi = r0 * np.maximum(cmin * hi, hi)
        e = ext(v)
        return s_lo - e, s_hi + e

    out = np.zeros((n, 13))
    out[:, 0], out[:, 1] = span(ep)
    out[:, 2], out[:, 3] = span(ez)
    rho = mN[:, 0] * math.sqrt((astar[0, 0] * astar[0, 0] + astar[0, 1] * astar[0, 1]) + astar[0, 2] * astar[0, 2])
    rho = rho + mN[:, 1] * math.sqrt((astar[1, 0] * astar[1, 0] + astar[1, 1] * astar[1, 1]) + astar[1, 2] * astar[1, 2])
    rho = rho + mN[:, 2] * math.sqrt((astar[2, 0] * astar[2, 0] + astar[2, 1] * astar[2, 1]) + astar[2, 2] * astar[2, 2])
    a_lo, a_hi = r0 - rho, r0 + rho
    out[:, 4] = np.where(a_lo > 0.0, a_lo * a_lo, 0.0)
    out[:, 5] = a_hi * a_hi
    # wedge of the in-plane node directions
    SR, SZ, e2R, e2Z = dot(S, ep), S[:, 2], dot(e2, ep), e2[:, 2]
    vmR, vmZ = SR - T * e2R, SZ - T * e2Z
    vpR, vpZ = SR + T * e2R, SZ + T * e2Z
    n1R, n1Z = -vmZ, vmR
    flip = n1R * vpR + n1Z * vpZ < 0.0
    n1R, n1Z = np.where(flip, -n1R, n1R), np.where(flip, -n1Z, n1Z)
    n2R, n2Z = -vpZ, vpR
    flip = n2R * vmR + n2Z * vmZ < 0.0
    n2R, n2Z = np.where(flip, -n2R, n2R), np.where(flip, -n2Z, n2Z)
    v1 = np.stack([n1R * ep[:, 0], n1R * ep[:, 1], n1R * ep[:, 2] + n1Z], axis=1)
    v2 = np.stack([n2R * ep[:, 0], n2R * ep[:, 1], n2R * ep[:, 2] + n2Z], axis=1)
    out[:, 6], out[:, 7], out[:, 8] = n1R, n1Z, ext(v1)
    out[:, 9], out[:, 10], out[:, 11] = n2R, n2Z, ext(v2)
    out[merid, 6:12] = [0.0, 0.0, -1.0, 0.0, 0.0, -1.0]
    ext_lim = wl.quad.extinction
    alive = ~((ext_lim > 0) & (extinction_arg(hkl, wl.dis.g) > ext_lim))
    out[:, 12] = alive.astype(np.float64)
    return out


def culling_lists(wl, hkl, tile_w=8, tile_h=8, tiles=None, boxes=None):
    """Per tile (row-major over tiles, or the given flat tile indices), ascending
    indices into hkl of the reflections that are alive and pass every test of the
    reflection's description (reflection_boxes, or the given boxes) against the tile's box
    (the box corners stand in for the tile's pixels in the wedge test)."""
    tb = tile_boxes(wl.geom, tile_w, tile_h).reshape(-1, 6)
    rb = reflection_boxes(wl, hkl) if boxes is None else boxes
    if tiles is None:
        tiles = range(tb.shape[0])
    lists = []
    for t in tiles:
        b = tb[t]
        ok = rb[:, 12] != 0.0
        ok &= (rb[:, 0] <= b[1]) & (b[0] <= rb[:, 1]) & (rb[:, 2] <= b[3]) & (b[2] <= rb[:, 3])
        ok &= (rb[:, 4] <= b[5]) & (b[4] <= rb[:, 5])
        wedge = rb[:, 8] >= 0.0
        m1 = np.maximum(rb[:, 6] * b[0], rb[:, 6] * b[1]) + np.maximum(rb[:, 7] * b[2], rb[:, 7] * b[3])
        m2 = np.maximum(rb[:, 9] * b[0], rb[:, 9] * b[1]) + np.maximum(rb[:, 10] * b[2], rb[:, 10] * b[3])
        ok &= ~wedge | ((m1 >= -rb[:, 8]) & (m2 >= -rb[:, 11]))
        lists.append(np.nonzero(ok)[0].astype(np.int32))
    return lists


# --------------------------------------------------------------------------- Ewald projection
def rodrigues(S, phi, n=np.array([0.0, 0.0, 1.0])):
    """S rotated by phi about unit axis n (Eq. rodrigues)."""
    S = np.asarray(S, dtype=np.float64)
    nxS = np.cross(n, S)
    nS = S @ n
    return S * np.cos(phi)[..., None] + nxS * np.sin(phi)[..., None] + n * (nS * (1.0 - np.cos(phi)))[..., None]


def ewald_angles(S, wavelength, beam=np.array([1.0, 0.0, 0.0]), fibre=np.array([0.0, 0.0, 1.0])):
    """Rotation angles about the fibre axis that bring S onto the Ewald sphere
    (Eqs. laue, squared, harmonic, solutions): P cos(phi) + Q sin(phi) = R with
    A = k.S, B = k.(n x S), D = (k.n)(n.S), C = |k|^2 + |S|^2, E = (1/lambda^2 - C)/2 - D,
    P = A - D, Q = B, R = E, |k| = 1/lambda.  Returns (phi1, phi2), NaN where
    |R|/sqrt(P^2 + Q^2) > 1 (Eq. valid)."""
    S = np.atleast_2d(np.asarray(S, dtype=np.float64))
    k = beam / wavelength
    A = S @ k
    Bc = np.cross(fibre, S) @ k
    Dc = (k @ fibre) * (S @ fibre)
    C = k @ k + np.sum(S * S, axis=1)
    E = (1.0 / wavelength ** 2 - C) / 2.0 - Dc
    P, Q, R = A - Dc, Bc, E
    amp = np.sqrt(P * P + Q * Q)
    with np.errstate(invalid="ignore", divide="ignore"):
        ratio = R / amp
        ok = np.abs(ratio) <= 1.0
        phi0 = np.arctan2(Q, P)
        dphi = np.where(ok, np.arccos(np.clip(ratio, -1.0, 1.0)), np.nan)
    return phi0 + dphi, phi0 - dphi


def ewald_project(S, geom, beam=np.array([1.0, 0.0, 0.0]), fibre=np.array([0.0, 0.0, 1.0])):
    """Detector positions (column i, row j, fractional pixel units, pixel centres at
    integers) of the two diffraction-condition rotations of each S: k_out = k_in + S_phi
    (section "Analytical Solution of the Ewald Diffraction Condition") intersected with
    the detector plane.  The plane passes through the beam centre P0 = (SF, 0, 0) with
    horizontal axis u = y and vertical axis v = (-sin d, 0, cos d), d = geom.det_tilt (its
    top leans toward the sample for d > 0; v = z for a detector normal to the beam), so its
    normal is u x v = (cos d, 0, sin d): the ray t k_out meets it at t = (P0.n)/(k_out.n),
    and the point X has detector coordinates X.u and (X - P0).v.  NaN where no rotation
    reaches the sphere."""
    S = np.atleast_2d(np.asarray(S, dtype=np.float64))
    d = float(getattr(geom, "det_tilt", 0.0))
    P0 = np.array([geom.distance, 0.0, 0.0])
    u = np.array([0.0, 1.0, 0.0])
    v = np.array([-math.sin(d), 0.0, math.cos(d)])
    nrm = np.cross(u, v)
    out = []
    for phi in ewald_angles(S, geom.wavelength, beam, fibre):
        Sphi = rodrigues(S, phi, fibre)
        kout = beam / geom.wavelength + Sphi
        t = (P0 @ nrm) / (kout @ nrm)
        X = t[:, None] * kout
        y = X @ u
        z = (X - P0) @ v
        out.append(np.stack([y / geom.pixel + geom.center_x - 0.5, z / geom.pixel + geom.center_y - 0.5], axis=1))
    return out[0], out[1]


def lorentz(R, delta):
    """Regularised Lorentz factor L = delta/(R + delta) (Eq. lorentz)."""
    return delta / (np.asarray(R, dtype=np.float64) + delta)
