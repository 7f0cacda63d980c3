"""Batched models: many workloads of different cells, atom counts, reflection lists
and detectors, stepped together by fdtbx_batch_forward / fdtbx_batch_backward.

Set-up runs the single-model entry points once per model (reflection list with the
extinction cull of its initial g, pixel map, tile boxes, culling lists) and
concatenates the results; the per-model descriptors (fdtbx_batch_entry) live in
device memory, so the refinable parameters of every model can be updated in place
(set_globals) between steps.  The step itself allocates nothing, copies nothing to
the host and never synchronises, so it can be captured in a HIP graph
(``GraphStep``).

Each model's tiles run in its own shape (its geometry's tile_w); ``autotune.tune_batch``
picks the shape of a whole batch by timing the batched forward in each candidate shape.
The forward walks stacked tiles (two launched tile rows per wave, one culling list for
both, fdtbx_batch_profile_stacked) unless the engine is built with stacked=False; the
backward walks the single tiles.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional

import numpy as np
import torch

from . import binding as B

RB = 256  # reflections / atoms / node-table rows per block of the work tables


def _pack(model: int, first: int) -> int:
    return (model << 40) | first


class StaleListsError(RuntimeError):
    """The globals of some model widen a lineshape support beyond its set-up culling lists."""


class BatchEngine:
    def __init__(self, workloads: List, device="cuda", deterministic: bool = False, stacked: bool = True):
        L = B.lib()
        if L.fdtbx_batch_entry_size() != ctypes.sizeof(B.BatchEntry):
            raise RuntimeError("fdtbx_batch_entry layout differs between the library and the binding")
        self.workloads = workloads
        self.n = n = len(workloads)
        self.device = device
        self.models = [B.make_model(wl) for wl in workloads]
        ents = (B.BatchEntry * n)()
        hkls, pixs, tiles, rowptrs, idxs = [], [], [], [], []
        ax, ay, az, aB, aocc, atype, ffs = [], [], [], [], [], [], []
        self.shapes = []
        off = dict(atom=0, hkl=0, pix=0, tile=0, rowptr=0, pair=0, node=0, ff=0)
        refl_blocks, model_rb, atom_blocks, node_blocks, items, costs = [], [], [], [], [], []
        # the forward's stacked tiles (fdtbx_batch_profile_stacked): two launched tile rows per
        # wave, one culling list for both (the backward keeps the per-tile lists)
        self.stacked = bool(stacked)
        sboxes, srowptrs, sidxs, s_items, s_costs, stack_off = [], [], [], [], [], []
        soff = dict(box=0, rowptr=0, pair=0)
        self.list_len = []
        self.tile_w = []
        for m, (wl, mod) in enumerate(zip(workloads, self.models)):
            e = ents[m]
            ext = (wl.dis.g[0], wl.dis.g[1], wl.dis.g[2], wl.quad.extinction) if wl.quad.extinction > 0 else None
            hkl = B.enumerate_hkl(mod.cell, wl.quad.d_min, wl.quad.d_max, extinction=ext, device=device)
            n_hkl = int(hkl.shape[0])
            if n_hkl == 0:
                raise ValueError(f"model {m} has no reflections")
            _, cull = B.reflection_prep(mod, hkl, torch.ones(n_hkl, dtype=torch.float32, device=device))
            self.tile_w.append(mod.geom.tile_w or B.TILE)
            B._check(L.fdtbx_batch_entry_init(ctypes.byref(mod), ctypes.byref(e)))
            pix, tile = B.pixel_map(mod.geom)
            rowptr, idx = B.cull(mod.geom, tile, cull)
            n_tiles = int(tile.shape[0])
            a = wl.atoms
            e.atom_off, e.n_atoms = off["atom"], a.n
            e.hkl_off, e.n_hkl = off["hkl"], n_hkl
            e.pix_off = off["pix"]
            e.tile_off = off["tile"]
            e.rowptr_off = off["rowptr"]
            e.pair_off = off["pair"]
            e.node_off = off["node"]
            e.ff_off = off["ff"]
            e.n_types = int(a.ff.shape[0])
            e.n_tiles = n_tiles
            model_rb.append(len(refl_blocks))
            refl_blocks += [_pack(m, r) for r in range(0, n_hkl, RB)]
            atom_blocks += [_pack(m, r) for r in range(0, a.n, RB)]
            n_rows = B.node_rows(wl.quad.n_nodes)
            node_blocks += [_pack(m, r) for r in range(0, n_rows, RB)]
            lens = (rowptr[1:] - rowptr[:-1]).cpu().numpy()
            # under the mirror folds only the left tile columns (bit 0) and the top tile rows
            # (bit 1) run; their values serve the mirror pixels
            tx_n, ty_n = B.tile_grid(mod.geom)
            lcols = (tx_n + 1) // 2 if mod.geom.mirror & 1 else tx_n
            lrows = (ty_n + 1) // 2 if mod.geom.mirror & 2 else ty_n
            t_all = np.arange(n_tiles)
            keep = np.nonzero((t_all % tx_n < lcols) & (t_all // tx_n < lrows))[0]
            items += [_pack(m, int(t)) for t in keep]
            costs.append(lens[keep])
            if self.stacked:
                sbox, srowptr, sidx = B.stacked_cull(mod.geom, tile, cull)
                n_st = int(sbox.shape[0])
                slens = (srowptr[1:] - srowptr[:-1]).cpu().numpy()
                s_all = np.arange(n_st)
                skeep = np.nonzero(s_all % tx_n < lcols)[0]  # every stacked row holds launched rows
                s_items += [_pack(m, int(t)) for t in skeep]
                s_costs.append(slens[skeep])
                stack_off += [soff["box"], soff["rowptr"], soff["pair"]]
                sboxes.append(sbox)
                srowptrs.append(srowptr)
                sidxs.append(sidx)
                soff["box"] += n_st
                soff["rowptr"] += n_st + 1
                soff["pair"] += int(sidx.shape[0])
            self.list_len.append(int(idx.shape[0]))
            hkls.append(hkl)
            pixs.append(pix.reshape(-1, 2))
            tiles.append(tile)
            rowptrs.append(rowptr)
            idxs.append(idx)
            ax.append(a.x), ay.append(a.y), az.append(a.z), aB.append(a.B), aocc.append(a.occ)
            atype.append(a.type), ffs.append(a.ff)
            self.shapes.append((wl.geom.height, wl.geom.width))
            off["atom"] += a.n
            off["hkl"] += n_hkl
            off["pix"] += wl.geom.width * wl.geom.height
            off["tile"] += n_tiles
            off["rowptr"] += n_tiles + 1
            off["pair"] += int(idx.shape[0])
            off["node"] += n_rows
            off["ff"] += int(a.ff.shape[0])
        model_rb.append(len(refl_blocks))
        self.totals = dict(off)
        dev = lambda arr, dt: torch.as_tensor(np.ascontiguousarray(arr), dtype=dt).to(device)
        self.hkl = torch.cat(hkls).contiguous()
        self.pix = torch.cat(pixs).contiguous()
        self.tile = torch.cat(tiles).contiguous()
        self.rowptr = torch.cat(rowptrs).contiguous()
        self.idx = torch.cat(idxs).contiguous() if off["pair"] > 0 else torch.zeros(1, dtype=torch.int32, device=device)
        self.atoms = {"x": dev(np.concatenate(ax), torch.float32), "y": dev(np.concatenate(ay), torch.float32),
                      "z": dev(np.concatenate(az), torch.float32), "B": dev(np.concatenate(aB), torch.float32),
                      "occ": dev(np.concatenate(aocc), torch.float32), "type": dev(np.concatenate(atype), torch.int32),
                      "ff": dev(np.concatenate(ffs), torch.float32)}
        # longest culling list first: the persistent kernels take items in this order
        cost = np.concatenate(costs)
        order = np.argsort(-cost, kind="stable")
        self.items = dev(np.asarray(items, dtype=np.int64)[order], torch.int64)
        if self.stacked:
            s_order = np.argsort(-np.concatenate(s_costs), kind="stable")
            self.stack_items = dev(np.asarray(s_items, dtype=np.int64)[s_order], torch.int64)
            self.stack_off = dev(np.asarray(stack_off, dtype=np.int64), torch.int64)
            self.stile = torch.cat(sboxes).contiguous()
            self.srowptr = torch.cat(srowptrs).contiguous()
            self.sidx = torch.cat(sidxs).contiguous() if soff["pair"] > 0 else \
                torch.zeros(1, dtype=torch.int32, device=device)
            self.totals["stacked_pair"] = soff["pair"]
        self.refl_blocks = dev(np.asarray(refl_blocks, dtype=np.int64), torch.int64)
        self.model_rb = dev(np.asarray(model_rb, dtype=np.int64), torch.int64)
        self.atom_blocks = dev(np.asarray(atom_blocks, dtype=np.int64), torch.int64)
        self.node_blocks = dev(np.asarray(node_blocks, dtype=np.int64), torch.int64)
        B._check(L.fdtbx_batch_entries_check(ctypes.byref(ents), n))
        raw = bytes(ctypes.string_at(ctypes.addressof(ents), ctypes.sizeof(ents)))
        self.entries = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)
        self._host_entries = ents
        H = off["hkl"]
        self.F = torch.empty((H, 2), dtype=torch.float32, device=device)
        self.F2 = torch.empty(H, dtype=torch.float32, device=device)
        self.refl = torch.empty((H, B.REFL_FLOATS), dtype=torch.float32, device=device)
        self.nodes = torch.empty((off["node"], B.NODE_FLOATS), dtype=torch.float32, device=device)
        self.image = torch.empty(off["pix"], dtype=torch.float32, device=device)
        self.counter = torch.zeros(2, dtype=torch.int64, device=device)
        self.sums = torch.empty((H, 6), dtype=torch.float64, device=device)
        self.part = torch.empty((max(len(refl_blocks), 1), B.N_GLOBALS), dtype=torch.float64, device=device)
        self.dF2 = torch.empty(H, dtype=torch.float32, device=device)
        self.grads = {k: torch.empty(off["atom"], dtype=torch.float32, device=device) for k in ("x", "y", "z", "B", "occ")}
        self.d_globals = torch.empty((n, B.N_GLOBALS), dtype=torch.float64, device=device)
        pix_off = [0]
        for h, w in self.shapes:
            pix_off.append(pix_off[-1] + h * w)
        self.pix_off = pix_off
        self.hkl_off = [ents[m].hkl_off for m in range(n)] + [H]
        self.atom_off = [ents[m].atom_off for m in range(n)] + [off["atom"]]
        # fixed-order adjoint sums: the batch's pairs by reflection (global indices), once
        self.deterministic = bool(deterministic)
        if self.deterministic:
            keys = np.concatenate([idxs[m].cpu().numpy().astype(np.int64) + ents[m].hkl_off for m in range(n)]) \
                if off["pair"] > 0 else np.zeros(0, dtype=np.int64)
            perm = np.argsort(keys, kind="stable")
            ptr = np.searchsorted(keys[perm], np.arange(H + 1), side="left")
            mate = np.full(H, -1, dtype=np.int64)
            for m, mod in enumerate(self.models):
                if mod.geom.mirror & 2:
                    h0, nh = ents[m].hkl_off, ents[m].n_hkl
                    mate[h0:h0 + nh] = h0 + nh - 1 - np.arange(nh)
            self.refl_ptr = dev(ptr, torch.int64)
            self.refl_pairs = dev(perm, torch.int32) if perm.size else torch.zeros(1, dtype=torch.int32, device=device)
            self.mate = dev(mate, torch.int64)
            self.partials = torch.empty((max(off["pair"], 1), 12), dtype=torch.float32, device=device)

    # ------------------------------------------------------------------ views
    def image_of(self, m: int) -> torch.Tensor:
        h, w = self.shapes[m]
        return self.image[self.pix_off[m]:self.pix_off[m + 1]].view(h, w)

    def globals(self) -> torch.Tensor:
        g = [[wl.dis.sigma_theta, wl.dis.gamma_theta, *wl.dis.N_base, *wl.dis.g, *wl.dis.B_axis] for wl in self.workloads]
        return torch.tensor(g, dtype=torch.float64, device=self.device)

    # ------------------------------------------------------------------ step
    def set_globals(self, glob: torch.Tensor, on_stale: str = "raise"):
        """Write every model's globals on the device.  The culling lists were built for the
        set-up g and N_base; a larger g or a smaller N_base widens a support past them, which
        fdtbx_batch_set_globals flags per model.  The flags are read back here (one small copy;
        keep this call outside a captured graph), and such a move either raises
        (on_stale="raise") or rebuilds the batch's static data for the new globals
        (on_stale="rebuild"; the atoms keep their current device values)."""
        if on_stale not in ("raise", "rebuild"):
            raise ValueError("on_stale must be 'raise' or 'rebuild'")
        glob = glob.to(self.device, torch.float64).contiguous()
        B._check(B.lib().fdtbx_batch_set_globals(B._ptr(self.entries), self.n, B._ptr(glob), B._stream()))
        stale = self.stale_models()
        if not stale:
            return
        if on_stale == "raise":
            raise StaleListsError(f"models {stale} widen a support beyond their culling lists (larger g or smaller "
                                  "N_base than at set-up); rebuild the batch")
        self._rebuild(glob)

    def stale_models(self) -> List[int]:
        """Models whose current globals widen a support beyond their set-up culling lists."""
        size = ctypes.sizeof(B.BatchEntry)
        off = B.BatchEntry.stale.offset
        raw = self.entries.view(self.n, size)[:, off:off + 4].cpu().numpy().copy().view(np.int32).ravel()
        return [int(m) for m in np.nonzero(raw)[0]]

    def _rebuild(self, glob: torch.Tensor):
        import dataclasses
        g = glob.cpu().numpy()
        wls = []
        for m, wl in enumerate(self.workloads):
            d = dataclasses.replace(wl.dis, sigma_theta=float(g[m, 0]), gamma_theta=float(g[m, 1]),
                                    N_base=tuple(float(v) for v in g[m, 2:5]), g=tuple(float(v) for v in g[m, 5:8]),
                                    B_axis=tuple(float(v) for v in g[m, 8:11]))
            wls.append(dataclasses.replace(wl, dis=d))
        atoms = {k: v.clone() for k, v in self.atoms.items()}
        self.__init__(wls, device=self.device, deterministic=self.deterministic, stacked=self.stacked)
        for k, v in atoms.items():
            self.atoms[k].copy_(v)

    def forward(self) -> torch.Tensor:
        a = self.atoms
        n_items = 0 if self.stacked else int(self.items.shape[0])
        B._check(B.lib().fdtbx_batch_forward(
            B._ptr(self.entries), self.n, B._ptr(self.refl_blocks), int(self.refl_blocks.shape[0]),
            B._ptr(self.node_blocks), int(self.node_blocks.shape[0]), B._ptr(self.items), n_items,
            B._ptr(self.hkl), B._ptr(a["x"]), B._ptr(a["y"]), B._ptr(a["z"]), B._ptr(a["B"]), B._ptr(a["occ"]),
            B._ptr(a["type"]), B._ptr(a["ff"]), B._ptr(self.pix), B._ptr(self.tile), B._ptr(self.rowptr),
            B._ptr(self.idx), B._ptr(self.F), B._ptr(self.F2), B._ptr(self.refl), B._ptr(self.nodes),
            B._ptr(self.image), B._ptr(self.counter), B._stream()))
        if self.stacked:
            B._check(B.lib().fdtbx_batch_profile_stacked(
                B._ptr(self.entries), self.n, B._ptr(self.stack_off), B._ptr(self.stack_items),
                int(self.stack_items.shape[0]), B._ptr(self.refl), B._ptr(self.nodes), B._ptr(self.pix),
                B._ptr(self.tile), B._ptr(self.stile), B._ptr(self.srowptr), B._ptr(self.sidx), B._ptr(self.image),
                B._ptr(self.counter), B._stream()))
        return self.image

    def backward(self, grad_image: torch.Tensor, atoms: bool = True):
        a = self.atoms
        g = self.grads
        d = [B._ptr(g[k]) if atoms else None for k in ("x", "y", "z", "B", "occ")]
        if self.deterministic:
            B._check(B.lib().fdtbx_batch_backward_deterministic(
                B._ptr(self.entries), self.n, B._ptr(self.refl_blocks), int(self.refl_blocks.shape[0]),
                B._ptr(self.model_rb), B._ptr(self.atom_blocks), int(self.atom_blocks.shape[0]), B._ptr(self.items),
                int(self.items.shape[0]), int(self.totals["hkl"]), B._ptr(self.hkl), B._ptr(a["x"]), B._ptr(a["y"]),
                B._ptr(a["z"]), B._ptr(a["B"]), B._ptr(a["occ"]), B._ptr(a["type"]), B._ptr(a["ff"]), B._ptr(self.pix),
                B._ptr(self.tile), B._ptr(self.rowptr), B._ptr(self.idx), B._ptr(self.F), B._ptr(self.refl),
                B._ptr(self.nodes), B._ptr(grad_image), int(self.totals["pair"]), B._ptr(self.refl_ptr),
                B._ptr(self.refl_pairs), B._ptr(self.mate), B._ptr(self.partials), B._ptr(self.sums), B._ptr(self.part),
                B._ptr(self.dF2), *d, B._ptr(self.d_globals), B._ptr(self.counter), B._stream()))
            return g, self.d_globals
        B._check(B.lib().fdtbx_batch_backward(
            B._ptr(self.entries), self.n, B._ptr(self.refl_blocks), int(self.refl_blocks.shape[0]),
            B._ptr(self.model_rb), B._ptr(self.atom_blocks), int(self.atom_blocks.shape[0]), B._ptr(self.items),
            int(self.items.shape[0]), int(self.totals["hkl"]), B._ptr(self.hkl), B._ptr(a["x"]), B._ptr(a["y"]),
            B._ptr(a["z"]), B._ptr(a["B"]), B._ptr(a["occ"]), B._ptr(a["type"]), B._ptr(a["ff"]), B._ptr(self.pix),
            B._ptr(self.tile), B._ptr(self.rowptr), B._ptr(self.idx), B._ptr(self.F), B._ptr(self.refl),
            B._ptr(self.nodes), B._ptr(grad_image), B._ptr(self.sums), B._ptr(self.part), B._ptr(self.dF2), *d,
            B._ptr(self.d_globals), B._ptr(self.counter), B._stream()))
        return g, self.d_globals


class GraphStep:
    """One refinement step of every model captured in a HIP graph: forward, pixel weights of
    the weighted residual, G = 2 w (I - T) with w = 1/(T + 1e-3 max T), and backward.  The
    targets and their weights are fixed inputs; replay() recomputes images and gradients
    for the parameters currently in the engine (set_globals / atom tensors updated in
    place).  The graph holds no memset nodes: every scratch buffer is cleared by a kernel."""

    def __init__(self, engine: BatchEngine, target: torch.Tensor):
        self.engine = engine
        self.target = target.contiguous()
        w = torch.empty_like(self.target)
        for m in range(engine.n):
            s = slice(engine.pix_off[m], engine.pix_off[m + 1])
            t = self.target[s]
            w[s] = 1.0 / (t + 1e-3 * t.max())
        self.weight = w
        self.G = torch.empty_like(self.target)
        self.graph = None

    def _body(self):
        img = self.engine.forward()
        torch.sub(img, self.target, out=self.G)
        self.G.mul_(self.weight).mul_(2.0)
        self.engine.backward(self.G)

    def eager(self):
        self._body()

    def capture(self):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self._body()  # warm-up outside the graph
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._body()
        torch.cuda.synchronize()

    def replay(self):
        self.graph.replay()
