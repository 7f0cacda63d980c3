"""ctypes binding of libfdtbx.so.

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Device buffers are torch CUDA tensors (torch supplies device memory
and the current stream); the functions below mirror the C ABI names in
include/fdtbx.h.  If the library is missing, importing works but every call
raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libfdtbx.so")

REFL_FLOATS = 64
CULL_DOUBLES = 16
NODE_FLOATS = 8
NODE_BLOCK = 4
TILE = 8

ERRORS = {0: "ok", -1: "invalid argument", -2: "geometry", -3: "buffer too small", -4: "hip", -5: "unsupported"}


class FdtbxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fdtbx error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


class Cell(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("b", ctypes.c_double), ("c", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("gamma", ctypes.c_double)]


class Geometry(ctypes.Structure):
    _fields_ = [("wavelength", ctypes.c_double), ("distance", ctypes.c_double), ("pixel", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("center_x", ctypes.c_double), ("center_y", ctypes.c_double), ("tilt", ctypes.c_double),
                ("tile_w", ctypes.c_int32), ("mirror", ctypes.c_int32), ("tile_waves", ctypes.c_int32),
                ("unit_pairs", ctypes.c_int32), ("det_tilt", ctypes.c_double)]


class Disorder(ctypes.Structure):
    _fields_ = [("sigma_theta", ctypes.c_double), ("gamma_theta", ctypes.c_double),
                ("N_base", ctypes.c_double * 3), ("g", ctypes.c_double * 3), ("intensity_model", ctypes.c_int32),
                ("lineshape", ctypes.c_int32), ("B_axis", ctypes.c_double * 3)]


class Quadrature(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("T", ctypes.c_double), ("sigma_r", ctypes.c_double),
                ("m", ctypes.c_int32), ("delta", ctypes.c_double), ("d_min", ctypes.c_double),
                ("d_max", ctypes.c_double), ("extinction", ctypes.c_double)]


class Model(ctypes.Structure):
    _fields_ = [("cell", Cell), ("geom", Geometry), ("dis", Disorder), ("quad", Quadrature)]


class BatchEntry(ctypes.Structure):
    _fields_ = [("model", Model), ("frame", ctypes.c_double * 19), ("atom_off", ctypes.c_int64),
                ("n_atoms", ctypes.c_int64), ("hkl_off", ctypes.c_int64), ("n_hkl", ctypes.c_int64),
                ("pix_off", ctypes.c_int64), ("tile_off", ctypes.c_int64), ("rowptr_off", ctypes.c_int64),
                ("pair_off", ctypes.c_int64), ("node_off", ctypes.c_int64), ("ff_off", ctypes.c_int64),
                ("n_types", ctypes.c_int32), ("n_tiles", ctypes.c_int32), ("setup_g", ctypes.c_double * 3),
                ("setup_N_base", ctypes.c_double * 3), ("stale", ctypes.c_int32), ("reserved", ctypes.c_int32)]


STATS_STAMPS = 8


class Stats(ctypes.Structure):
    _fields_ = [("n_hkl", ctypes.c_int64), ("n_pairs", ctypes.c_int64), ("pair_cap", ctypes.c_int64),
                ("useful_evals", ctypes.c_int64), ("overflow", ctypes.c_int32), ("n_stamps", ctypes.c_int32),
                ("clock_khz", ctypes.c_int64), ("stamp", ctypes.c_uint64 * STATS_STAMPS)]


STATS_STEPS = ("reflection_prep", "node_table", "pixel_map", "cull", "tile_order", "profile", "count")

_lib = None

_SIGS = {
    "fdtbx_error_string": (ctypes.c_char_p, [ctypes.c_int]),
    "fdtbx_last_hip_error": (ctypes.c_int, []),
    "fdtbx_hkl_capacity": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]),
    "fdtbx_enumerate_workspace": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_double]),
    "fdtbx_enumerate_hkl": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_size_t, ctypes.c_void_p]),
    "fdtbx_sf_workspace": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int64]),
    "fdtbx_structure_factors": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64] + [ctypes.c_void_p] * 7 +
                                [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "fdtbx_node_rows": (ctypes.c_int64, [ctypes.c_int32]),
    "fdtbx_node_table": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fdtbx_reflection_prep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fdtbx_pixel_map": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fdtbx_tile_grid": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fdtbx_launch_waves": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "fdtbx_cull_workspace": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int64]),
    "fdtbx_cull": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_void_p]),
    "fdtbx_stacked_rows": (ctypes.c_int32, [ctypes.c_void_p]),
    "fdtbx_stacked_boxes": (ctypes.c_int, [ctypes.c_void_p] * 4),
    "fdtbx_stacked_cull_workspace": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int64]),
    "fdtbx_stacked_cull": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "fdtbx_profile": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 10),
    "fdtbx_tile_order_size": (ctypes.c_int64, [ctypes.c_void_p]),
    "fdtbx_tile_order_workspace": (ctypes.c_size_t, [ctypes.c_void_p]),
    "fdtbx_tile_order": (ctypes.c_int, [ctypes.c_void_p] * 4 + [ctypes.c_size_t, ctypes.c_void_p]),
    "fdtbx_profile_cyl": (ctypes.c_int, [ctypes.c_void_p] * 7 + [ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                                                   ctypes.c_void_p]),
    "fdtbx_cyl_records": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "fdtbx_profile_points": (ctypes.c_int, [ctypes.c_void_p] * 6 + [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "fdtbx_ewald_project": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "fdtbx_splat": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fdtbx_pattern_workspace": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64]),
    "fdtbx_profile_pattern": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_size_t, ctypes.c_void_p]),
    "fdtbx_profile_pattern_async": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "fdtbx_profile_adjoint": (ctypes.c_int, [ctypes.c_void_p] * 8 + [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                                                      ctypes.c_void_p]),
    "fdtbx_adjoint_finish_workspace": (ctypes.c_size_t, [ctypes.c_int64]),
    "fdtbx_adjoint_finish": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64] + [ctypes.c_void_p] * 6 +
                             [ctypes.c_size_t, ctypes.c_void_p]),
    "fdtbx_sf_adjoint_workspace": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int64]),
    "fdtbx_sf_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64] + [ctypes.c_void_p] * 7 +
                         [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64] + [ctypes.c_void_p] * 8 +
                         [ctypes.c_size_t, ctypes.c_void_p]),
    "fdtbx_backward_workspace": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int64]),
    "fdtbx_pattern_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64,
                                              ctypes.c_int64] + [ctypes.c_void_p] * 7 + [ctypes.c_int32] +
                               [ctypes.c_void_p] * 8 + [ctypes.c_size_t, ctypes.c_void_p]),
    "fdtbx_profile_adjoint_pairs": (ctypes.c_int, [ctypes.c_void_p] * 8 + [ctypes.c_int64, ctypes.c_int64,
                                                                            ctypes.c_void_p, ctypes.c_void_p,
                                                                            ctypes.c_void_p]),
    "fdtbx_pair_transpose_workspace": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int64]),
    "fdtbx_pair_transpose": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                            ctypes.c_void_p]),
    "fdtbx_pair_reduce": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "fdtbx_backward_deterministic_workspace": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]),
    "fdtbx_pattern_backward_deterministic": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                            ctypes.c_size_t, ctypes.c_int64, ctypes.c_int64] +
                                             [ctypes.c_void_p] * 7 + [ctypes.c_int32] + [ctypes.c_void_p] * 8 +
                                             [ctypes.c_size_t, ctypes.c_void_p]),
    "fdtbx_unit_pairs": (ctypes.c_int64, [ctypes.c_int64]),
    "fdtbx_profile_balanced_workspace": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int64]),
    "fdtbx_profile_balanced": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 7 +
                               [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "fdtbx_profile_adjoint_balanced": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 7 +
                                       [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "fdtbx_pattern_backward_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                       ctypes.c_size_t, ctypes.c_int64, ctypes.c_int64] +
                                       [ctypes.c_void_p] * 7 + [ctypes.c_int32] + [ctypes.c_void_p] * 8),
    "fdtbx_batch_backward_deterministic": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                                          ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                                          ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                                          ctypes.c_int64] + [ctypes.c_void_p] * 16 +
                                           [ctypes.c_int64] + [ctypes.c_void_p] * 15),
    "fdtbx_batch_entry_init": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "fdtbx_batch_entry_size": (ctypes.c_size_t, []),
    "fdtbx_batch_entries_check": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "fdtbx_batch_set_globals": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "fdtbx_batch_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64] +
                            [ctypes.c_void_p] * 18 + [ctypes.c_void_p]),
    "fdtbx_batch_profile_stacked": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_int64] + [ctypes.c_void_p] * 10),
    "fdtbx_batch_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                            ctypes.c_int64, ctypes.c_int64] + [ctypes.c_void_p] * 26 + [ctypes.c_void_p]),
}


def exported_symbols():
    return list(_SIGS.keys())


def lib():
    """Load libfdtbx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        msg = lib().fdtbx_error_string(rc).decode()
        raise FdtbxError(rc, msg)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, dtype, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ----------------------------------------------------------------------------- struct builders
def make_cell(c) -> Cell:
    return Cell(c.a, c.b, c.c, c.alpha, c.beta, c.gamma)


def make_model(wl) -> Model:
    g, d, q = wl.geom, wl.dis, wl.quad
    return Model(make_cell(wl.cell),
                 Geometry(g.wavelength, g.distance, g.pixel, g.width, g.height, g.center_x, g.center_y,
                          float(getattr(g, "tilt", 0.0)), int(getattr(g, "tile_w", 0)), int(getattr(g, "mirror", 0)),
                          int(getattr(g, "tile_waves", 0)), int(getattr(g, "unit_pairs", 0)),
                          float(getattr(g, "det_tilt", 0.0))),
                 Disorder(d.sigma_theta, d.gamma_theta, (ctypes.c_double * 3)(*d.N_base),
                          (ctypes.c_double * 3)(*d.g), d.intensity_model, int(getattr(d, "lineshape", 0)),
                          (ctypes.c_double * 3)(*getattr(d, "B_axis", (0.0, 0.0, 0.0)))),
                 Quadrature(q.n_nodes, q.T, q.sigma_r, q.m, q.delta, q.d_min, q.d_max, q.extinction))


def launch_waves(geom: Geometry) -> int:
    """fdtbx_launch_waves: waves per tile of the profile and adjoint launches."""
    w = ctypes.c_int32(0)
    _check(lib().fdtbx_launch_waves(ctypes.byref(geom), ctypes.byref(w)))
    return int(w.value)


def tile_grid(geom: Geometry):
    """fdtbx_tile_grid: (tiles_x, tiles_y) of the geometry's pixel tiles."""
    tx, ty = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().fdtbx_tile_grid(ctypes.byref(geom), ctypes.byref(tx), ctypes.byref(ty)))
    return int(tx.value), int(ty.value)


# ----------------------------------------------------------------------------- entry points
def hkl_capacity(cell: Cell, d_min: float) -> int:
    cap = ctypes.c_int64(0)
    _check(lib().fdtbx_hkl_capacity(ctypes.byref(cell), d_min, ctypes.byref(cap)))
    return int(cap.value)


def enumerate_hkl(cell: Cell, d_min: float, d_max: float, extinction=None, device="cuda") -> torch.Tensor:
    """fdtbx_enumerate_hkl; returns int32 [n][3] on the device (one synchronisation to read n)."""
    L = lib()
    cap = hkl_capacity(cell, d_min)
    out = torch.empty((cap, 3), dtype=torch.int32, device=device)
    n = torch.zeros(1, dtype=torch.int64, device=device)
    wsb = L.fdtbx_enumerate_workspace(ctypes.byref(cell), d_min)
    ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device=device)
    ext = None
    if extinction is not None:
        ext = (ctypes.c_double * 4)(*extinction)
    _check(L.fdtbx_enumerate_hkl(ctypes.byref(cell), d_min, d_max, ext, _ptr(out), cap, _ptr(n), _ptr(ws), wsb,
                                 _stream()))
    return out[: int(n.item())]


def structure_factors(cell: Cell, atoms: dict, hkl: torch.Tensor, want_F=True, want_F2=True):
    """fdtbx_structure_factors.  atoms: dict of device tensors x, y, z, B, occ (float32), type (int32),
    ff (float32 [n_types][9]).  Returns (F [n][2] or None, F2 [n] or None)."""
    L = lib()
    n_hkl = int(hkl.shape[0])
    n_atoms = int(atoms["x"].shape[0])
    for k in ("x", "y", "z", "B", "occ", "ff"):
        _dev(atoms[k], torch.float32, k)
    _dev(atoms["type"], torch.int32, "type")
    _dev(hkl, torch.int32, "hkl")
    dev = hkl.device
    F = torch.empty((n_hkl, 2), dtype=torch.float32, device=dev) if want_F else None
    F2 = torch.empty(n_hkl, dtype=torch.float32, device=dev) if want_F2 else None
    wsb = L.fdtbx_sf_workspace(n_hkl, n_atoms)
    ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device=dev)
    _check(L.fdtbx_structure_factors(ctypes.byref(cell), n_atoms, _ptr(atoms["x"]), _ptr(atoms["y"]), _ptr(atoms["z"]),
                                     _ptr(atoms["B"]), _ptr(atoms["occ"]), _ptr(atoms["type"]), _ptr(atoms["ff"]),
                                     int(atoms["ff"].shape[0]), _ptr(hkl), n_hkl, _ptr(F), _ptr(F2), _ptr(ws), wsb,
                                     _stream()))
    return F, F2


def node_rows(n_nodes: int) -> int:
    """Rows of the node table: n^2 node records followed by the node-block records."""
    rows = int(lib().fdtbx_node_rows(int(n_nodes)))
    if rows <= 0:
        raise FdtbxError(-1, f"n_nodes {n_nodes} outside 1..256")
    return rows


def node_table(model: Model) -> torch.Tensor:
    """Node table [node_rows(n)][NODE_FLOATS]; the first n^2 rows are the node records."""
    out = torch.empty((node_rows(model.quad.n_nodes), NODE_FLOATS), dtype=torch.float32, device="cuda")
    _check(lib().fdtbx_node_table(ctypes.byref(model.dis), ctypes.byref(model.quad), _ptr(out), _stream()))
    return out


def reflection_prep(model: Model, hkl: torch.Tensor, F2: torch.Tensor):
    n = int(hkl.shape[0])
    _dev(hkl, torch.int32, "hkl")
    _dev(F2, torch.float32, "F2")
    refl = torch.empty((n, REFL_FLOATS), dtype=torch.float32, device=hkl.device)
    cull = torch.empty((n, CULL_DOUBLES), dtype=torch.float64, device=hkl.device)
    _check(lib().fdtbx_reflection_prep(ctypes.byref(model), _ptr(hkl), n, _ptr(F2), _ptr(refl), _ptr(cull), _stream()))
    return refl, cull


def pixel_map(geom: Geometry):
    tx, ty = tile_grid(geom)
    pix = torch.empty((geom.height, geom.width, 2), dtype=torch.float64, device="cuda")
    tile = torch.empty((tx * ty, 8), dtype=torch.float64, device="cuda")
    _check(lib().fdtbx_pixel_map(ctypes.byref(geom), _ptr(pix), _ptr(tile), _stream()))
    return pix, tile


def cull(geom: Geometry, tile: torch.Tensor, cull_rec: torch.Tensor, cap: Optional[int] = None):
    """fdtbx_cull; returns (offsets int64 [n_tiles+1], idx int32 [n_pairs]).  Retries once with the
    exact capacity when cap is too small."""
    L = lib()
    n_hkl = int(cull_rec.shape[0])
    n_tiles = int(tile.shape[0])
    offsets = torch.empty(n_tiles + 1, dtype=torch.int64, device=tile.device)
    wsb = L.fdtbx_cull_workspace(ctypes.byref(geom), n_hkl)
    ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device=tile.device)
    if cap is None:
        cap = 1 << 20
    for _ in range(2):
        idx = torch.empty(max(cap, 1), dtype=torch.int32, device=tile.device)
        n_pairs = ctypes.c_int64(0)
        rc = L.fdtbx_cull(ctypes.byref(geom), _ptr(tile), n_hkl, _ptr(cull_rec), _ptr(offsets), _ptr(idx), cap,
                          ctypes.byref(n_pairs), _ptr(ws), wsb, _stream())
        if rc == -3 and n_pairs.value > cap:
            cap = int(n_pairs.value)
            continue
        _check(rc)
        return offsets, idx[: int(n_pairs.value)]
    raise FdtbxError(-3, "culling capacity")


def stacked_cull(geom: Geometry, tile: torch.Tensor, cull_rec: torch.Tensor, cap: Optional[int] = None):
    """fdtbx_stacked_boxes and fdtbx_stacked_cull; returns (boxes float64 [n_stacked][8], offsets
    int64 [n_stacked + 1], idx int32 [n_pairs]) of the stacked tiles (pairs of launched tile rows)."""
    L = lib()
    n_rows = int(L.fdtbx_stacked_rows(ctypes.byref(geom)))
    if n_rows <= 0:
        raise FdtbxError(-1, "fdtbx_stacked_rows rejected the geometry")
    tx, _ = tile_grid(geom)
    n = tx * n_rows
    _dev(tile, torch.float64, "tile")
    boxes = torch.empty((n, 8), dtype=torch.float64, device=tile.device)
    _check(L.fdtbx_stacked_boxes(ctypes.byref(geom), _ptr(tile), _ptr(boxes), _stream()))
    n_hkl = int(cull_rec.shape[0])
    offsets = torch.empty(n + 1, dtype=torch.int64, device=tile.device)
    wsb = L.fdtbx_stacked_cull_workspace(ctypes.byref(geom), n_hkl)
    ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device=tile.device)
    cap = 1 << 20 if cap is None else cap
    for _ in range(2):
        idx = torch.empty(max(cap, 1), dtype=torch.int32, device=tile.device)
        n_pairs = ctypes.c_int64(0)
        rc = L.fdtbx_stacked_cull(ctypes.byref(geom), _ptr(boxes), n_hkl, _ptr(cull_rec), _ptr(offsets), _ptr(idx),
                                  cap, ctypes.byref(n_pairs), _ptr(ws), wsb, _stream())
        if rc == -3 and n_pairs.value > cap:
            cap = int(n_pairs.value)
            continue
        _check(rc)
        return boxes, offsets, idx[: int(n_pairs.value)]
    raise FdtbxError(-3, "culling capacity")


def tile_order(geom: Geometry, offsets: torch.Tensor) -> torch.Tensor:
    """fdtbx_tile_order: launch order (int32, -1 for padding) of the per-tile kernels."""
    L = lib()
    n = int(L.fdtbx_tile_order_size(ctypes.byref(geom)))
    if n <= 0:
        raise FdtbxError(-1, "fdtbx_tile_order_size rejected the geometry")
    _dev(offsets, torch.int64, "offsets")
    order = torch.empty(n, dtype=torch.int32, device=offsets.device)
    wsb = L.fdtbx_tile_order_workspace(ctypes.byref(geom))
    ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device=offsets.device)
    _check(L.fdtbx_tile_order(ctypes.byref(geom), _ptr(offsets), _ptr(order), _ptr(ws), wsb, _stream()))
    return order


def profile(model: Model, refl, nodes, pix, tile, offsets, idx, count=False, order=None):
    """fdtbx_profile: the image [H][W] float32, or (count=True) the number of support-passing
    evaluations.  order: fdtbx_tile_order of the lists, or None."""
    g = model.geom
    if count:
        c = torch.zeros(1, dtype=torch.int64, device="cuda")
        _check(lib().fdtbx_profile(ctypes.byref(model), _ptr(refl), _ptr(nodes), _ptr(pix), _ptr(tile), _ptr(offsets),
                                   _ptr(idx), _ptr(order), None, _ptr(c), _stream()))
        return int(c.item())
    img = torch.empty((g.height, g.width), dtype=torch.float32, device="cuda")
    _check(lib().fdtbx_profile(ctypes.byref(model), _ptr(refl), _ptr(nodes), _ptr(pix), _ptr(tile), _ptr(offsets),
                               _ptr(idx), _ptr(order), _ptr(img), None, _stream()))
    return img


def unit_pairs(n_pairs: int) -> int:
    """fdtbx_unit_pairs: the library's pairs per work unit of the balanced launch."""
    return int(lib().fdtbx_unit_pairs(int(n_pairs)))


def profile_balanced(model: Model, refl, nodes, pix, tile, offsets, idx, order=None, pair_cap=None, ws=None):
    """fdtbx_profile_balanced: the image [H][W] float32 from the launch balanced over the
    compute units (model.geom.unit_pairs pairs per work unit, 0: the library's choice).
    pair_cap: capacity of idx (default: its length).  ws: a uint8 device tensor of at least
    fdtbx_profile_balanced_workspace bytes to use (and keep the unit tables in, for
    profile_adjoint_balanced), or None."""
    g = model.geom
    cap = int(idx.shape[0]) if pair_cap is None else int(pair_cap)
    if idx.numel() == 0:  # empty lists: any valid pointer
        idx = torch.zeros(1, dtype=torch.int32, device="cuda")
    wsb = lib().fdtbx_profile_balanced_workspace(ctypes.byref(model), cap)
    if wsb == 0:
        raise FdtbxError(-1, "fdtbx_profile_balanced_workspace: invalid model or capacity")
    if ws is None:
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    img = torch.empty((g.height, g.width), dtype=torch.float32, device="cuda")
    _check(lib().fdtbx_profile_balanced(ctypes.byref(model), _ptr(refl), _ptr(nodes), _ptr(pix), _ptr(tile),
                                        _ptr(offsets), _ptr(idx), _ptr(order), cap, _ptr(img), _ptr(ws),
                                        int(ws.numel()), _stream()))
    return img


def balanced_workspace(model: Model, pair_cap: int) -> torch.Tensor:
    """A device workspace for profile_balanced and profile_adjoint_balanced."""
    wsb = lib().fdtbx_profile_balanced_workspace(ctypes.byref(model), int(pair_cap))
    if wsb == 0:
        raise FdtbxError(-1, "fdtbx_profile_balanced_workspace: invalid model or capacity")
    return torch.empty(wsb, dtype=torch.uint8, device="cuda")


def profile_adjoint_balanced(model: Model, refl, nodes, pix, tile, offsets, idx, grad_image: torch.Tensor, ws,
                             order=None, pair_cap=None) -> torch.Tensor:
    """fdtbx_profile_adjoint_balanced: per-reflection sums float64 [n_hkl][6] over the work
    units of the profile_balanced call that used ws (same model, lists, order and pair_cap)."""
    n = int(refl.shape[0])
    _dev(grad_image, torch.float32, "grad_image")
    cap = int(idx.shape[0]) if pair_cap is None else int(pair_cap)
    if idx.numel() == 0:
        idx = torch.zeros(1, dtype=torch.int32, device="cuda")
    sums = torch.empty((n, 6), dtype=torch.float64, device=refl.device)
    _check(lib().fdtbx_profile_adjoint_balanced(ctypes.byref(model), _ptr(refl), _ptr(nodes), _ptr(pix), _ptr(tile),
                                                _ptr(offsets), _ptr(idx), _ptr(order), cap, n, _ptr(grad_image),
                                                _ptr(sums), _ptr(ws), int(ws.numel()), _stream()))
    return sums


def cyl_records(model: Model, hkl) -> torch.Tensor:
    """fdtbx_cyl_records: culling records float64 [n][CULL_DOUBLES] for the cylindrical average."""
    n = int(hkl.shape[0])
    out = torch.empty((n, CULL_DOUBLES), dtype=torch.float64, device=hkl.device)
    _check(lib().fdtbx_cyl_records(ctypes.byref(model), _ptr(hkl), n, _ptr(out), _stream()))
    return out


def profile_cyl(model: Model, refl, nodes, pix, offsets, idx, arc: float, count=False, order=None):
    """fdtbx_profile_cyl: the cylindrically averaged image [H][W] float32, or (count=True) the
    number of support-passing evaluations.  order: fdtbx_tile_order of the lists, or None."""
    g = model.geom
    if count:
        c = torch.zeros(1, dtype=torch.int64, device="cuda")
        _check(lib().fdtbx_profile_cyl(ctypes.byref(model), _ptr(refl), _ptr(nodes), _ptr(pix), _ptr(offsets), _ptr(idx),
                                       _ptr(order), float(arc), None, _ptr(c), _stream()))
        return int(c.item())
    img = torch.empty((g.height, g.width), dtype=torch.float32, device="cuda")
    _check(lib().fdtbx_profile_cyl(ctypes.byref(model), _ptr(refl), _ptr(nodes), _ptr(pix), _ptr(offsets), _ptr(idx),
                                   _ptr(order), float(arc), _ptr(img), None, _stream()))
    return img


def profile_points(model: Model, hkl, refl, nodes, ridx, points) -> torch.Tensor:
    """fdtbx_profile_points: W_h I_h(p) float32 [n] for reflection ridx[k] at points[k]."""
    n = int(points.shape[0])
    _dev(ridx, torch.int32, "ridx")
    _dev(points, torch.float64, "points")
    out = torch.empty(n, dtype=torch.float32, device=points.device)
    _check(lib().fdtbx_profile_points(ctypes.byref(model), _ptr(hkl), _ptr(refl), _ptr(nodes), _ptr(ridx), _ptr(points), n,
                                      _ptr(out), _stream()))
    return out


def ewald_project(geom: Geometry, S) -> torch.Tensor:
    """fdtbx_ewald_project: float64 [n][4] detector positions of both rotations (NaN if none)."""
    n = int(S.shape[0])
    _dev(S, torch.float64, "S")
    out = torch.empty((n, 4), dtype=torch.float64, device=S.device)
    _check(lib().fdtbx_ewald_project(ctypes.byref(geom), _ptr(S), n, _ptr(out), _stream()))
    return out


def splat(model: Model, hkl, refl, nodes, n_r: int, n_s: int, count=False):
    """fdtbx_splat: the forward-splat image [H][W] float32, or (count=True) the number of
    (sample, node) pairs inside the support."""
    g = model.geom
    n = int(hkl.shape[0])
    if count:
        c = torch.zeros(1, dtype=torch.int64, device="cuda")
        _check(lib().fdtbx_splat(ctypes.byref(model), _ptr(hkl), n, _ptr(refl), _ptr(nodes), int(n_r), int(n_s), None,
                                 _ptr(c), _stream()))
        return int(c.item())
    img = torch.empty((g.height, g.width), dtype=torch.float32, device="cuda")
    _check(lib().fdtbx_splat(ctypes.byref(model), _ptr(hkl), n, _ptr(refl), _ptr(nodes), int(n_r), int(n_s), _ptr(img),
                             None, _stream()))
    return img


class PatternPlan:
    """Workspace holder for fdtbx_profile_pattern; grows its culling capacity on demand."""

    def __init__(self, model: Model, n_hkl: int, pair_cap: int = 1 << 20):
        self.model = model
        self.n_hkl = n_hkl
        self.pair_cap = pair_cap
        self._alloc()

    def _alloc(self):
        wsb = lib().fdtbx_pattern_workspace(ctypes.byref(self.model), self.n_hkl, self.pair_cap)
        if wsb == 0:
            raise FdtbxError(-1, "fdtbx_pattern_workspace rejected the model")
        self.ws_bytes = wsb
        self.ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")

    def run(self, hkl: torch.Tensor, F2: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        g = self.model.geom
        if out is None:
            out = torch.empty((g.height, g.width), dtype=torch.float32, device="cuda")
        for _ in range(2):
            need = ctypes.c_int64(0)
            rc = lib().fdtbx_profile_pattern(ctypes.byref(self.model), _ptr(hkl), self.n_hkl, _ptr(F2), _ptr(out),
                                             self.pair_cap, ctypes.byref(need), _ptr(self.ws), self.ws_bytes, _stream())
            if rc == -3 and need.value > self.pair_cap:
                self.pair_cap = int(need.value * 1.05) + 1024
                self._alloc()
                continue
            _check(rc)
            self.pairs = int(need.value)
            return out
        raise FdtbxError(-3, "pattern workspace")

    def run_async(self, hkl: torch.Tensor, F2: torch.Tensor, out: torch.Tensor, stats: torch.Tensor,
                  count: bool = False) -> torch.Tensor:
        """fdtbx_profile_pattern_async into out with the plan's current capacity: no host round
        trip, so it can be captured in a graph.  stats: a device buffer of sizeof(fdtbx_stats)
        bytes (new_stats()); read it after the stream with read_stats() and, on overflow,
        grow(n_pairs) and run again."""
        _check(lib().fdtbx_profile_pattern_async(ctypes.byref(self.model), _ptr(hkl), self.n_hkl, _ptr(F2), _ptr(out),
                                                 self.pair_cap, 1 if count else 0, _ptr(stats), _ptr(self.ws),
                                                 self.ws_bytes, _stream()))
        return out

    def grow(self, n_pairs: int):
        """Capacity for at least n_pairs culling-list entries (reallocates the workspace)."""
        if n_pairs > self.pair_cap:
            self.pair_cap = int(n_pairs * 1.05) + 1024
            self._alloc()


def new_stats(device="cuda") -> torch.Tensor:
    """A device buffer for one fdtbx_stats."""
    return torch.zeros(ctypes.sizeof(Stats), dtype=torch.uint8, device=device)


def read_stats(stats: torch.Tensor) -> dict:
    """The fdtbx_stats in a device buffer (synchronises), with per-step milliseconds."""
    raw = bytes(stats.cpu().numpy().tobytes())
    st = Stats.from_buffer_copy(raw)
    khz = max(int(st.clock_khz), 1)
    stamps = [int(v) for v in st.stamp]
    ms = {name: (stamps[k + 1] - stamps[k]) / khz for k, name in enumerate(STATS_STEPS)}
    return {"n_hkl": int(st.n_hkl), "n_pairs": int(st.n_pairs), "pair_cap": int(st.pair_cap),
            "useful_evals": int(st.useful_evals), "overflow": bool(st.overflow), "clock_khz": int(st.clock_khz),
            "ms": ms, "total_ms": (stamps[-1] - stamps[0]) / khz}


# ----------------------------------------------------------------------------- adjoint
GLOBAL_NAMES = ("sigma_theta", "gamma_theta", "N_base_a", "N_base_b", "N_base_c", "g_a", "g_b", "g_c",
                "B_a", "B_b", "B_c")
N_GLOBALS = len(GLOBAL_NAMES)
NOALLOC_SCRATCH_BYTES = 64 << 20  # FDTBX_NOALLOC_SCRATCH_BYTES of include/fdtbx.h
LINESHAPES = {"laue": 0, "gaussian": 1, "hosemann": 2}


def profile_adjoint(model: Model, refl, nodes, pix, tile, offsets, idx, grad_image: torch.Tensor, order=None) -> torch.Tensor:
    """fdtbx_profile_adjoint: per-reflection sums float64 [n_hkl][6]."""
    n = int(refl.shape[0])
    _dev(grad_image, torch.float32, "grad_image")
    sums = torch.empty((n, 6), dtype=torch.float64, device=refl.device)
    _check(lib().fdtbx_profile_adjoint(ctypes.byref(model), _ptr(refl), _ptr(nodes), _ptr(pix), _ptr(tile), _ptr(offsets),
                                       _ptr(idx), _ptr(order), n, _ptr(grad_image), _ptr(sums), _stream()))
    return sums


def profile_adjoint_pairs(model: Model, refl, nodes, pix, tile, offsets, idx, grad_image: torch.Tensor,
                          order=None) -> torch.Tensor:
    """fdtbx_profile_adjoint_pairs: per-pair partial sums float32 [n_pairs][12] (the pair's
    reflection's six, then its Friedel mate's six)."""
    n = int(refl.shape[0])
    _dev(grad_image, torch.float32, "grad_image")
    cap = int(idx.shape[0])
    partials = torch.empty((max(cap, 1), 12), dtype=torch.float32, device=refl.device)
    _check(lib().fdtbx_profile_adjoint_pairs(ctypes.byref(model), _ptr(refl), _ptr(nodes), _ptr(pix), _ptr(tile),
                                             _ptr(offsets), _ptr(idx), _ptr(order), n, cap, _ptr(grad_image),
                                             _ptr(partials), _stream()))
    return partials[:cap]


def pair_transpose(n_hkl: int, idx: torch.Tensor, n_pairs_dev: Optional[torch.Tensor] = None):
    """fdtbx_pair_transpose: (refl_ptr int64 [n_hkl+1], refl_pairs int32 [len(idx)])."""
    L = lib()
    cap = int(idx.shape[0])
    dev = idx.device
    refl_ptr = torch.empty(n_hkl + 1, dtype=torch.int64, device=dev)
    refl_pairs = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    wsb = L.fdtbx_pair_transpose_workspace(n_hkl, cap)
    if wsb == 0:
        raise FdtbxError(-5, "fdtbx_pair_transpose_workspace: sizes out of range")
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    _check(L.fdtbx_pair_transpose(n_hkl, _ptr(idx), cap, _ptr(n_pairs_dev), _ptr(refl_ptr), _ptr(refl_pairs), _ptr(ws),
                                  wsb, _stream()))
    return refl_ptr, refl_pairs[:cap]


def pair_reduce(n_hkl: int, refl_ptr, refl_pairs, partials, mate=None, updown: bool = False) -> torch.Tensor:
    """fdtbx_pair_reduce: per-reflection sums float64 [n_hkl][6] in a fixed order."""
    sums = torch.empty((n_hkl, 6), dtype=torch.float64, device=refl_ptr.device)
    _check(lib().fdtbx_pair_reduce(n_hkl, _ptr(refl_ptr), _ptr(refl_pairs), _ptr(partials), _ptr(mate),
                                   1 if updown else 0, _ptr(sums), _stream()))
    return sums


def adjoint_finish(model: Model, hkl, refl, sums, F):
    """fdtbx_adjoint_finish: (dF2 float32 [n], d_globals float64 [N_GLOBALS])."""
    L = lib()
    n = int(hkl.shape[0])
    dF2 = torch.empty(n, dtype=torch.float32, device=hkl.device)
    glob = torch.empty(N_GLOBALS, dtype=torch.float64, device=hkl.device)
    wsb = L.fdtbx_adjoint_finish_workspace(n)
    ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device=hkl.device)
    _check(L.fdtbx_adjoint_finish(ctypes.byref(model), _ptr(hkl), n, _ptr(refl), _ptr(sums), _ptr(F), _ptr(dF2), _ptr(glob),
                                  _ptr(ws), wsb, _stream()))
    return dF2, glob


def sf_adjoint(cell: Cell, atoms: dict, hkl, F, dF2):
    """fdtbx_sf_adjoint: dict of float32 [n_atoms] gradients x, y, z (fractional), B, occ."""
    L = lib()
    n_hkl = int(hkl.shape[0])
    n_atoms = int(atoms["x"].shape[0])
    dev = hkl.device
    out = {k: torch.empty(n_atoms, dtype=torch.float32, device=dev) for k in ("x", "y", "z", "B", "occ")}
    wsb = L.fdtbx_sf_adjoint_workspace(n_hkl, n_atoms)
    ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device=dev)
    _check(L.fdtbx_sf_adjoint(ctypes.byref(cell), n_atoms, _ptr(atoms["x"]), _ptr(atoms["y"]), _ptr(atoms["z"]),
                              _ptr(atoms["B"]), _ptr(atoms["occ"]), _ptr(atoms["type"]), _ptr(atoms["ff"]),
                              int(atoms["ff"].shape[0]), _ptr(hkl), n_hkl, _ptr(F), _ptr(dF2), _ptr(out["x"]),
                              _ptr(out["y"]), _ptr(out["z"]), _ptr(out["B"]), _ptr(out["occ"]), _ptr(ws), wsb,
                              _stream()))
    return out


def _backward_outputs(n_hkl, atoms, dev):
    glob = torch.empty(N_GLOBALS, dtype=torch.float64, device=dev)
    dF2 = torch.empty(n_hkl, dtype=torch.float32, device=dev)
    out, a, d, nt = None, [None] * 7, [None] * 5, 1
    if atoms is not None:
        n_atoms = int(atoms["x"].shape[0])
        out = {k: torch.empty(n_atoms, dtype=torch.float32, device=dev) for k in ("x", "y", "z", "B", "occ")}
        a = [_ptr(atoms[k]) for k in ("x", "y", "z", "B", "occ", "type", "ff")]
        d = [_ptr(out[k]) for k in ("x", "y", "z", "B", "occ")]
        nt = int(atoms["ff"].shape[0])
    return out, glob, dF2, a, d, nt


def pattern_backward_noalloc(plan: "PatternPlan", hkl, F, grad_image, atoms: Optional[dict]):
    """fdtbx_pattern_backward_noalloc: fdtbx_pattern_backward with the library's own device
    scratch array as its workspace (the call allocates nothing; the output tensors here are
    the caller's).  Raises FdtbxError when the problem's workspace exceeds
    NOALLOC_SCRATCH_BYTES."""
    L = lib()
    n_atoms = int(atoms["x"].shape[0]) if atoms is not None else 0
    out, glob, dF2, a, d, nt = _backward_outputs(plan.n_hkl, atoms, hkl.device)
    _check(L.fdtbx_pattern_backward_noalloc(ctypes.byref(plan.model), _ptr(hkl), plan.n_hkl, _ptr(F), _ptr(grad_image),
                                            _ptr(plan.ws), plan.ws_bytes, plan.pair_cap, n_atoms, *a, nt, *d, _ptr(glob),
                                            _ptr(dF2), _stream()))
    return out, glob, dF2


def pattern_backward(plan: "PatternPlan", hkl, F, grad_image, atoms: Optional[dict], deterministic: bool = False):
    """fdtbx_pattern_backward (or, with deterministic, fdtbx_pattern_backward_deterministic:
    fixed-order sums, the same bits on every run) after plan.run(hkl, |F|^2): (atom gradients
    dict or None, d_globals float64 [N_GLOBALS], dF2 float32 [n_hkl])."""
    L = lib()
    n_hkl = plan.n_hkl
    dev = hkl.device
    n_atoms = int(atoms["x"].shape[0]) if atoms is not None else 0
    if deterministic:
        wsb = L.fdtbx_backward_deterministic_workspace(n_hkl, n_atoms, plan.pair_cap)
        if wsb == 0:
            raise FdtbxError(-5, "fdtbx_backward_deterministic_workspace: sizes out of range")
        entry = L.fdtbx_pattern_backward_deterministic
    else:
        wsb = L.fdtbx_backward_workspace(n_hkl, n_atoms)
        entry = L.fdtbx_pattern_backward
    ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device=dev)
    out, glob, dF2, a, d, nt = _backward_outputs(n_hkl, atoms, dev)
    _check(entry(ctypes.byref(plan.model), _ptr(hkl), n_hkl, _ptr(F), _ptr(grad_image), _ptr(plan.ws), plan.ws_bytes,
                 plan.pair_cap, n_atoms, *a, nt, *d, _ptr(glob), _ptr(dF2), _ptr(ws), wsb, _stream()))
    return out, glob, dF2
