"""Per-model choice of the pixel-tile shape of the per-tile launches.

Every per-tile kernel runs one to four 64-lane waves per tile of tile_w x (64 / tile_w)
pixels (fdtbx_geometry.tile_w; the waves per tile follow tile_waves, which the tuner leaves
as the model has it).  The shape changes how many (tile, reflection) pairs the culling
lists hold, how large each pair's node window and alpha box are, and how many of a queued
node's 64 lanes fall inside their supports; which shape is fastest depends on the detector
geometry and on the size of the reflections' supports in pixels.  The image does not depend
on the shape beyond float32 summation order.

TileTuner builds the pixel map, culling lists and launch order of each candidate shape,
times the model's whole profile launch (HIP events on the current stream; one warm-up
launch, then the fastest of `reps`), and keeps the fastest shape.  A candidate other than
the default 8 x 8 must beat it by more than `margin`.  Timing the whole launch matters: a
launch of this size holds only a few rounds of workgroups, so its time is set by how the
long tiles and the L2 sharing of neighbouring tiles play out, which no sample of tiles
reproduces.  Models with fewer than `min_tiles` tiles keep the default shape untimed (their
launch is too short for its time to say anything about their work).  Choices are cached per
model (every model field except tile_w, and the reflection count) behind a lock, so a
refinement loop tunes once.

A batch (batch.py) runs the tiles of all its models in one persistent launch, so the
quantity to tune there is the batched forward's time, not each model's own launch:
tune_batch builds the batch in each candidate shape and keeps the fastest engine.

Tuning launches kernels and synchronises; it is set-up work, never part of a step.
"""
from __future__ import annotations

import ctypes
import dataclasses
import threading
from typing import Dict, Optional, Tuple

import torch

from . import binding as B

CANDIDATES = (4, 8, 16)
DEFAULT = 8


def model_key(model: B.Model, n_hkl: int) -> tuple:
    """Every field of the model except geom.tile_w, and the reflection count."""
    flat = []

    def walk(s):
        for name, _ in s._fields_:
            if name == "tile_w":
                continue
            v = getattr(s, name)
            if isinstance(v, ctypes.Structure):
                walk(v)
            elif isinstance(v, ctypes.Array):
                flat.extend(list(v))
            else:
                flat.append(v)

    walk(model)
    return tuple(flat), int(n_hkl)


def with_tile_w(model: B.Model, tile_w: int) -> B.Model:
    m = B.Model.from_buffer_copy(model)
    m.geom.tile_w = int(tile_w)
    return m


def shape_allowed(geom: B.Geometry) -> bool:
    """The library accepts this tile width for this geometry (under the left-right fold the
    width must be a multiple of it, under the up-down fold the height a multiple of the tile
    height 64 / tile_w)."""
    try:
        B.tile_grid(geom)
        return True
    except B.FdtbxError:
        return False


class TileTuner:
    def __init__(self, candidates=CANDIDATES, reps: int = 2, margin: float = 0.02, min_tiles: int = 0):
        if DEFAULT not in candidates:
            raise ValueError("the candidates must include the default tile width 8")
        self.candidates = tuple(int(c) for c in candidates)
        self.reps, self.margin, self.min_tiles = int(reps), float(margin), int(min_tiles)
        self._cache: Dict[tuple, Tuple[int, Dict[int, float]]] = {}
        self._lock = threading.Lock()

    def cached(self, model: B.Model, n_hkl: int) -> Optional[Tuple[int, Dict[int, float]]]:
        with self._lock:
            return self._cache.get(model_key(model, n_hkl))

    def _time(self, model, refl, nodes, cull_rec) -> float:
        pix, tile = B.pixel_map(model.geom)
        off, idx = B.cull(model.geom, tile, cull_rec)
        order = B.tile_order(model.geom, off)
        if idx.numel() == 0:
            idx = torch.zeros(1, dtype=torch.int32, device=refl.device)
        B.profile_balanced(model, refl, nodes, pix, tile, off, idx, order=order)  # warm-up
        best = float("inf")
        for _ in range(self.reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            B.profile_balanced(model, refl, nodes, pix, tile, off, idx, order=order)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    def choose(self, model: B.Model, refl: torch.Tensor, nodes: torch.Tensor, cull_rec: torch.Tensor) -> int:
        """Tile width for this model (from the cache when an equal model was tuned).
        refl, cull_rec: fdtbx_reflection_prep of the model's reflections (the timing does not
        depend on |F|^2); nodes: its fdtbx_node_table."""
        n_hkl = int(refl.shape[0])
        hit = self.cached(model, n_hkl)
        if hit is not None:
            return hit[0]
        tx, ty = B.tile_grid(with_tile_w(model, DEFAULT).geom)
        if n_hkl == 0 or tx * ty < self.min_tiles:
            times = {}
        else:
            times = {tw: self._time(with_tile_w(model, tw), refl, nodes, cull_rec) for tw in self.candidates
                     if shape_allowed(with_tile_w(model, tw).geom)}
        if not times:
            own = model.geom.tile_w or DEFAULT
            with self._lock:
                self._cache[model_key(model, n_hkl)] = (own, times)
            return own
        best = min(times, key=times.get)
        if DEFAULT in times and times[best] > (1.0 - self.margin) * times[DEFAULT]:
            best = DEFAULT
        with self._lock:
            self._cache[model_key(model, n_hkl)] = (best, times)
        return best

    def choices(self) -> Dict[tuple, Tuple[int, Dict[int, float]]]:
        with self._lock:
            return dict(self._cache)


def tune_batch(workloads, candidates=(8, 16, 4), reps: int = 1, margin: float = 0.02, device="cuda"):
    """Build the batch with every model in each candidate tile shape, time its forward (one
    warm-up, then the fastest of reps) and return (the fastest engine, {tile_w: ms}).  A shape
    other than the default must beat it by more than margin.  At most two engines are alive
    at a time (the best so far and the one being timed)."""
    from .batch import BatchEngine

    order = [DEFAULT] + [int(c) for c in candidates if int(c) != DEFAULT]
    if DEFAULT not in candidates:
        raise ValueError("the candidates must include the default tile width 8")
    best_tw, best_t, best_be, times = None, float("inf"), None, {}
    for tw in order:
        if not all(shape_allowed(with_tile_w(B.make_model(w), tw).geom) for w in workloads):
            continue
        be = BatchEngine([dataclasses.replace(w, geom=dataclasses.replace(w.geom, tile_w=tw)) for w in workloads],
                         device=device)
        be.forward()
        torch.cuda.synchronize()
        t = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            be.forward()
            e1.record()
            torch.cuda.synchronize()
            t = min(t, e0.elapsed_time(e1))
        times[tw] = t
        threshold = best_t * (1.0 - margin) if best_tw == DEFAULT else best_t
        if best_be is None or t < threshold:
            best_tw, best_t, best_be = tw, t, be
        else:
            del be
        torch.cuda.empty_cache()
    if best_be is None:
        raise ValueError("no candidate tile shape is allowed for every model of the batch")
    return best_be, times
