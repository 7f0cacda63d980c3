"""MI355X (gfx950) implementation of the fibre-diffraction profile-quadrature path.

The compute runs in libfdtbx.so (hand-written HIP kernels behind a C ABI,
include/fdtbx.h); this package holds the ctypes binding and a small pipeline
that strings the entry points together on torch's current stream:

  enumerate_hkl -> structure_factors -> profile pattern (reflection prep, node
  table, pixel map, tile culling, profile kernel)

There is no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import torch

from . import binding as B

__all__ = ["B", "Pipeline", "atoms_to_device", "build"]


def build(verbose: bool = False) -> str:
    from .build import build as _b
    return _b(verbose)


def atoms_to_device(atoms, device="cuda") -> dict:
    t = lambda a, dt: torch.as_tensor(a, dtype=dt).contiguous().to(device)
    return {"x": t(atoms.x, torch.float32), "y": t(atoms.y, torch.float32), "z": t(atoms.z, torch.float32),
            "B": t(atoms.B, torch.float32), "occ": t(atoms.occ, torch.float32), "type": t(atoms.type, torch.int32),
            "ff": t(atoms.ff, torch.float32)}


class Pipeline:
    """Forward pattern of one workload: reflection list (with the extinction cull),
    structure factors and the detector image, all on the device."""

    def __init__(self, wl, device="cuda"):
        self.wl = wl
        self.model = B.make_model(wl)
        self.cell = self.model.cell
        self.atoms = atoms_to_device(wl.atoms, device)
        ext = None
        if wl.quad.extinction > 0:
            ext = (wl.dis.g[0], wl.dis.g[1], wl.dis.g[2], wl.quad.extinction)
        self.hkl = B.enumerate_hkl(self.cell, wl.quad.d_min, wl.quad.d_max, extinction=ext, device=device)
        self.n_hkl = int(self.hkl.shape[0])
        self.plan = B.PatternPlan(self.model, self.n_hkl)

    def structure_factors(self):
        return B.structure_factors(self.cell, self.atoms, self.hkl)

    def pattern(self, F2=None, out=None):
        if F2 is None:
            _, F2 = B.structure_factors(self.cell, self.atoms, self.hkl, want_F=False)
        return self.plan.run(self.hkl, F2, out)
