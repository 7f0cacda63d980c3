"""torch.autograd wrapper of the forward pattern and its hand-written adjoint.

``PatternFunction`` maps (fractional x, y, z, B, occupancy, globals) to the
detector image through libfdtbx (structure factors, then the profile pattern)
and back through fdtbx_pattern_backward.  globals is a float64 tensor of the
eleven parameters (sigma_theta, gamma_theta, N_base a/b/c, g a/b/c, B_axis a/b/c);
the node grid extent T stays fixed.

``FibreModel`` holds refinement parameters in physical units (Cartesian
coordinates in A, B, occupancy, total angular width sigma and Lorentzian fraction
eta, crystallite sizes in A, Hosemann g, axis damping B_axis) and converts them
with torch ops, so that autograd supplies those chain rules.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np
import torch

from . import binding as B


class PatternEngine:
    """Static part of a model: cell, detector, quadrature, scattering-factor table,
    atom types and the reflection list (enumerated once, with the extinction cull of
    the initial g).  Owns the pattern workspace that the backward reuses."""

    def __init__(self, wl, device="cuda"):
        self.wl = wl
        self.model = B.make_model(wl)
        self.cell = self.model.cell
        self.device = device
        ext = None
        if wl.quad.extinction > 0:
            ext = (wl.dis.g[0], wl.dis.g[1], wl.dis.g[2], wl.quad.extinction)
        self.hkl = B.enumerate_hkl(self.cell, wl.quad.d_min, wl.quad.d_max, extinction=ext, device=device)
        self.n_hkl = int(self.hkl.shape[0])
        self.type = torch.as_tensor(wl.atoms.type, dtype=torch.int32).contiguous().to(device)
        self.ff = torch.as_tensor(wl.atoms.ff, dtype=torch.float32).contiguous().to(device)
        self.plan = B.PatternPlan(self.model, self.n_hkl)
        # forward passes run on this engine; a backward needs the workspace of its own forward
        self.generation = 0

    def set_globals(self, g):
        d = self.model.dis
        d.sigma_theta, d.gamma_theta = float(g[0]), float(g[1])
        for i in range(3):
            d.N_base[i] = float(g[2 + i])
            d.g[i] = float(g[5 + i])
            d.B_axis[i] = float(g[8 + i])

    def globals_of(self, wl=None) -> torch.Tensor:
        d = (wl or self.wl).dis
        return torch.tensor([d.sigma_theta, d.gamma_theta, *d.N_base, *d.g, *d.B_axis], dtype=torch.float64)

    def atoms(self, x, y, z, Bf, occ) -> dict:
        c = lambda t: t.detach().to(self.device, torch.float32).contiguous()
        return {"x": c(x), "y": c(y), "z": c(z), "B": c(Bf), "occ": c(occ), "type": self.type, "ff": self.ff}


class PatternFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, z, Bf, occ, glob, engine: PatternEngine):
        engine.set_globals(glob.detach().cpu().tolist())
        atoms = engine.atoms(x, y, z, Bf, occ)
        F, F2 = B.structure_factors(engine.cell, atoms, engine.hkl)
        img = engine.plan.run(engine.hkl, F2)
        engine.generation += 1
        ctx.generation = engine.generation
        ctx.engine = engine
        ctx.atoms = atoms
        ctx.F = F
        ctx.glob_meta = (glob.dtype, glob.device)
        ctx.atom_meta = [(t.dtype, t.device) for t in (x, y, z, Bf, occ)]
        return img

    @staticmethod
    def backward(ctx, grad):
        engine = ctx.engine
        if engine.generation != ctx.generation:
            # the engine's workspace (records, node table, culling lists) and its model's globals
            # now belong to a later forward: this graph's gradients cannot be formed from them
            raise RuntimeError("PatternFunction.backward: the engine ran another forward pass after this one; "
                               "call backward before the next forward on the same PatternEngine, or use one "
                               "engine per pattern")
        grad = grad.detach().to(torch.float32).contiguous()
        need_atoms = any(ctx.needs_input_grad[:5])
        out, glob, _ = B.pattern_backward(engine.plan, engine.hkl, ctx.F, grad, ctx.atoms if need_atoms else None)
        res = [None] * 7
        if need_atoms:
            for i, k in enumerate(("x", "y", "z", "B", "occ")):
                dt, dev = ctx.atom_meta[i]
                res[i] = out[k].to(dev, dt)
        dt, dev = ctx.glob_meta
        res[5] = glob.to(dev, dt)
        return tuple(res)


def pattern(engine: PatternEngine, x, y, z, Bf, occ, glob):
    return PatternFunction.apply(x, y, z, Bf, occ, glob, engine)


def real_basis(cell) -> np.ndarray:
    """Rows a, b, c of the real basis in the laboratory frame of the tutorial (c along z,
    b in the yz-plane); fractional -> Cartesian is x_cart = frac @ basis."""
    ca, cb, cg = math.cos(cell.alpha), math.cos(cell.beta), math.cos(cell.gamma)
    sa = math.sin(cell.alpha)
    az = cell.a * cb
    ay = cell.a * (cg - ca * cb) / sa
    ax = math.sqrt(cell.a * cell.a - ay * ay - az * az)
    return np.array([[ax, ay, az], [0.0, cell.b * sa, cell.b * ca], [0.0, 0.0, cell.c]])


class FibreModel(torch.nn.Module):
    """Parameters: xyz (Cartesian, A) [n][3], B [n], occ [n], sigma (rad), eta, size (A) [3],
    g [3], B_axis (A^2) [3].  forward() returns the detector image."""

    def __init__(self, wl, engine: Optional[PatternEngine] = None, device="cuda"):
        super().__init__()
        self.engine = engine or PatternEngine(wl, device)
        basis = torch.tensor(real_basis(wl.cell), dtype=torch.float64)
        self.register_buffer("basis", basis)
        self.register_buffer("basis_inv", torch.linalg.inv(basis))
        self.register_buffer("edges", torch.tensor([wl.cell.a, wl.cell.b, wl.cell.c], dtype=torch.float64))
        a = wl.atoms
        frac = torch.tensor(np.stack([a.x, a.y, a.z], 1).astype(np.float64))
        self.xyz = torch.nn.Parameter(frac @ basis)
        self.B = torch.nn.Parameter(torch.tensor(a.B.astype(np.float64)))
        self.occ = torch.nn.Parameter(torch.tensor(a.occ.astype(np.float64)))
        st, gt = wl.dis.sigma_theta, wl.dis.gamma_theta
        self.sigma = torch.nn.Parameter(torch.tensor(st + gt, dtype=torch.float64))
        self.eta = torch.nn.Parameter(torch.tensor(gt / (st + gt), dtype=torch.float64))
        self.size = torch.nn.Parameter(torch.tensor([wl.dis.N_base[i] * [wl.cell.a, wl.cell.b, wl.cell.c][i]
                                                     for i in range(3)], dtype=torch.float64))
        self.g = torch.nn.Parameter(torch.tensor(list(wl.dis.g), dtype=torch.float64))
        self.B_axis = torch.nn.Parameter(torch.tensor(list(wl.dis.B_axis), dtype=torch.float64))

    def globals(self):
        st = (1.0 - self.eta) * self.sigma
        gt = self.eta * self.sigma
        Nb = self.size / self.edges
        return torch.cat([st.reshape(1), gt.reshape(1), Nb, self.g, self.B_axis])

    def forward(self):
        frac = self.xyz @ self.basis_inv
        glob = self.globals()
        return pattern(self.engine, frac[:, 0], frac[:, 1], frac[:, 2], self.B, self.occ, glob)


def weighted_residual(img: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """sum w (I - T)^2 with w = 1/(T + 1e-3 max T), the refinement loss."""
    w = 1.0 / (target + 1e-3 * target.max())
    return torch.sum(w * (img - target) ** 2)
