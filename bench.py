"""Benchmark of the fibre-diffraction profile-quadrature path on one MI355X.

A step is one pass of the whole forward path over the large workload (100x100x120 A
cell, 50,000 atoms, reflections to 1.5 A: 293,298 after the extinction cull, 2048x2048
detector, Lorentzian 2 deg, Hosemann g .05 lateral, 96x96 nodes), the largest
configuration that one GPU holds: reflection enumeration, structure factors, reflection
preparation, node table, pixel map, tile culling and the profile kernel.  Inputs are
seeded and synthetic and resident in device memory before the timed region.

Prints one JSON line.  value = useful profile evaluations per second of the whole step
(evaluations = (pixel, reflection, node) triples inside the kernel support, counted once
by a counting pass of the same kernel).  The roofline object refers to the profile
kernel, timed with HIP events on the stream it is launched on; cpu_baseline is the FP64
oracle on a bounded pixel sample of the same workload, on all host cores and on one.
The medium workload's forward step, the tilted fibre, the other lineshapes, the exact
cylindrical average, the forward splat, the refinement step (forward + adjoint) and the
batch of 256 ragged models are reported as further keys.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Per useful evaluation, the issue slots of the arithmetic the method needs in
# this formulation: 3 subtractions (lattice coordinates relative to the node),
# 1 three-way max and 1 compare (support), 4 multiplies (sine and coordinate
# products), 1 multiply and 1 square (ratio), 1 fused multiply-add (weighted
# accumulate), plus 3 sines and 1 reciprocal.  A transcendental takes one issue
# slot: a stream of nothing but v_sin_f32 or v_rcp_f32 runs at half the v_fma_f32
# rate, but mixed with other arithmetic (here one per four) it runs beside it; the
# profile kernel's counters show one VALU instruction issued per SIMD cycle with the
# transcendentals counted once.
TRANS_SLOTS = 1
SLOTS_PER_EVAL = 12 + 4 * TRANS_SLOTS
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = VALU lane issue slots per second.
PEAK_SLOTS = 256 * 4 * 16 * 2.4e9


def log(msg):
    """Progress line on stderr (the JSON result is the only line on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def profile_source_sha():
    """sha256 prefix over the sources the forward profile kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for f in ("profile.hip", "profile_tile.h", "profile_common.h"):
        with open(os.path.join(ROOT, "paper_2608_23245_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload="large"):
    """HBM bytes per launch of the profile kernel on a workload from the committed counter
    summary, or None when the kernel source has changed since the counters were taken."""
    import re
    summ = os.path.join(ROOT, "profiles", f"k_profile_{workload}_traffic.md")
    try:
        text = open(summ).read()
        sha = profile_source_sha()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch: ([0-9.eE+]+)", text)
    h = re.search(r"profile kernel sources sha256 prefix at measurement: ([0-9a-f]+)", text)
    if not m or not h or h.group(1) != sha:
        return None
    return float(m.group(1))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--cpu-block", type=int, default=8, help="side of the pixel block the CPU baseline times")
    ap.add_argument("--cpu-one-core-pixels", type=int, default=8,
                    help="pixels of the block the one-core CPU baseline times")
    ap.add_argument("--no-bwd", action="store_true", help="skip the forward+backward leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 256-model leg")
    ap.add_argument("--no-tilt", action="store_true", help="skip the tilted-fibre forward leg")
    ap.add_argument("--no-medium", action="store_true", help="skip the medium-workload forward leg")
    ap.add_argument("--no-lineshapes", action="store_true", help="skip the Gaussian/Hosemann lineshape legs")
    ap.add_argument("--no-splat", action="store_true", help="skip the forward-splat leg")
    ap.add_argument("--no-cyl", action="store_true", help="skip the exact cylindrical-average leg")
    ap.add_argument("--tile-w", type=int, default=0, choices=(0, 2, 4, 8, 16, 32),
                    help="pixel-tile width of the large (headline) forward (0: chosen by the tile tuner)")
    ap.add_argument("--medium-tile-w", type=int, default=0, choices=(0, 2, 4, 8, 16, 32),
                    help="pixel-tile width of the medium forward (0: chosen by the tile tuner)")
    ap.add_argument("--only-headline", action="store_true", help="run the large forward leg alone (profiler runs)")
    ap.add_argument("--no-mirror", action="store_true", help="run every tile (no mirror fold)")
    ap.add_argument("--no-updown", action="store_true", help="fold the left-right mirror only (not the up-down one)")
    ap.add_argument("--no-unfolded", action="store_true", help="skip the unfolded reference forward")
    ap.add_argument("--only-batch", action="store_true",
                    help="run the batched forward alone, at --batch-tile-w, --steps times (profiler runs)")
    ap.add_argument("--batch-tile-w", type=int, default=16, choices=(4, 8, 16, 32),
                    help="tile width of every model of the batch with --only-batch")
    ap.add_argument("--batch-per-tile", action="store_true",
                    help="with --only-batch, walk the per-tile culling lists instead of the stacked tiles")
    ap.add_argument("--batch-models", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="also run one device-to-device copy of this many MiB (reference kernel for the "
                         "FETCH_SIZE/WRITE_SIZE counters)")
    return ap.parse_args()


def forward_leg(wl, steps, warmup):
    """Times the whole forward step (enumeration, structure factors, reflection prep, node
    table, pixel map, culling, profile kernel) on workload wl.  Returns the wall time per
    step, the profile kernel's mean HIP-event time, the useful evaluations of one step
    (counting pass after the timed region) and the buffers of the last step."""
    import numpy as np
    import torch

    from paper_2608_23245_amd import atoms_to_device
    from paper_2608_23245_amd import binding as B

    model = B.make_model(wl)
    cell = model.cell
    atoms = atoms_to_device(wl.atoms)
    ext = (wl.dis.g[0], wl.dis.g[1], wl.dis.g[2], wl.quad.extinction)
    stream = torch.cuda.current_stream()
    state = {}

    def step(timed_events=None):
        hkl = B.enumerate_hkl(cell, wl.quad.d_min, wl.quad.d_max, extinction=ext)
        _, F2 = B.structure_factors(cell, atoms, hkl, want_F=False)
        refl, cull = B.reflection_prep(model, hkl, F2)
        nodes = B.node_table(model)
        pix, tile = B.pixel_map(model.geom)
        off, idx = B.cull(model.geom, tile, cull, cap=state.get("cap", 1 << 24))
        state["cap"] = int(idx.shape[0]) + 1024
        order = B.tile_order(model.geom, off)
        if timed_events is not None:
            timed_events[0].record(stream)
        img = B.profile_balanced(model, refl, nodes, pix, tile, off, idx, order=order)
        if timed_events is not None:
            timed_events[1].record(stream)
        state.update(hkl=hkl, refl=refl, nodes=nodes, pix=pix, tile=tile, off=off, idx=idx, order=order, img=img)
        return img

    log(f"forward: {wl.name}, {warmup} warm-up steps")
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    log(f"forward: {steps} timed steps")
    events = [[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(events[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / steps
    prof_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    img = state["img"]
    assert torch.isfinite(img).all()
    n_evals = B.profile(model, state["refl"], state["nodes"], state["pix"], state["tile"], state["off"], state["idx"],
                        count=True, order=state["order"])
    return ms_step, prof_ms, n_evals, state


MIRROR = {"on": True, "updown": True}


def fold(wl):
    """wl with the mirror folds its geometry allows, unless --no-mirror was given: left-right
    (bit 0) with the beam centre at width/2 and the width a multiple of the tile width (the
    image is bit-identical); up-down (bit 1, unless --no-updown) with the fibre normal to the
    beam, the beam centre at height/2 and the height a multiple of the tile height (the pattern's
    Friedel symmetry: the mirrored rows agree with an unfolded run to float32 rounding).  The
    per-tile launches run the left columns and top rows and write each value to its mirror
    images; the evaluations counted are the ones performed."""
    g = wl.geom
    tw = g.tile_w or 8
    bits = 0
    if MIRROR["on"] and g.center_x == 0.5 * g.width and g.width % tw == 0:
        bits |= 1
    if MIRROR["on"] and MIRROR["updown"] and g.tilt == 0.0 and g.center_y == 0.5 * g.height and g.height % (64 // tw) == 0:
        bits |= 2
    return dataclasses.replace(wl, geom=dataclasses.replace(g, mirror=bits))


def fold_name(wl):
    m = wl.geom.mirror
    return {0: "none", 1: "left-right", 2: "up-down", 3: "left-right and up-down"}[m]


def compare_unfolded(wl, img, img0):
    """A folded image against the unfolded one of the same waves per tile: the pixels the folded
    launches compute are bit-identical, the left-right mirror pixels too; the up-down mirror rows
    agree to float32 rounding (Friedel mates summed in another order).  Asserts the first and
    returns the relative L2 and largest per-pixel differences of the whole image."""
    import torch
    g = wl.geom
    th = 64 // (g.tile_w or 8)
    tiles_y = -(-g.height // th)
    top = ((tiles_y + 1) // 2) * th if g.mirror & 2 else g.height
    assert torch.equal(img[:top], img0[:top]), "the folded image's computed rows differ from the unfolded ones"
    if g.mirror & 2:
        low = g.height - top  # rows written from their up-down mirrors
        assert torch.equal(img[g.height - low:], torch.flip(img[:low], [0]))
    a, b = img.double(), img0.double()
    big = b > 1e-3 * b.max()
    return {"computed_rows_bit_identical": True, "image_bit_identical": bool(torch.equal(img, img0)),
            "rel_l2": float(torch.linalg.norm(a - b) / torch.linalg.norm(b)),
            "max_rel_pixel": float(((a - b).abs()[big] / b[big]).max())}


def other_rates(kernel_evals_per_s, prof_ms):
    """The profile kernel's rate against the other peaks: the transcendental unit at a quarter
    of the lane rate (3 sines and 1 reciprocal per evaluation), FP32 FLOPs against the 157.3
    TFLOP/s vector peak (13 FLOPs per evaluation: the FMA counts two, compare and max3 one each,
    the transcendentals none), and HBM bandwidth from the committed counters."""
    trans = 4 * kernel_evals_per_s
    flops = 13 * kernel_evals_per_s
    tr = measured_traffic()
    return {"transcendental_lane_ops_per_s": trans, "transcendental_frac_of_quarter_rate": trans / (PEAK_SLOTS / 4),
            "fp32_flop_per_s": flops, "fp32_flop_frac_of_157.3T": flops / 157.3e12,
            "hbm_GBps": None if tr is None else tr / (prof_ms * 1e-3) / 1e9}


def tune_tiles(wl):
    """Tile shape of workload wl chosen by the tuner (set-up, outside every timed region)."""
    import dataclasses

    import torch

    from paper_2608_23245_amd import atoms_to_device
    from paper_2608_23245_amd import binding as B
    from paper_2608_23245_amd.autotune import TileTuner

    t0 = time.perf_counter()
    model = B.make_model(wl)
    ext = (wl.dis.g[0], wl.dis.g[1], wl.dis.g[2], wl.quad.extinction)
    hkl = B.enumerate_hkl(model.cell, wl.quad.d_min, wl.quad.d_max, extinction=ext)
    _, F2 = B.structure_factors(model.cell, atoms_to_device(wl.atoms), hkl, want_F=False)
    refl, cull = B.reflection_prep(model, hkl, F2)
    tuner = TileTuner()
    tw = tuner.choose(model, refl, B.node_table(model), cull)
    times = tuner.cached(model, int(hkl.shape[0]))[1]
    torch.cuda.synchronize()
    info = {"tile": f"{tw}x{64 // tw}", "profile_ms": {f"{c}x{64 // c}": round(v, 3) for c, v in times.items()},
            "tuned": True, "tuning_s": time.perf_counter() - t0}
    log(f"tile tuner: {info['profile_ms']} -> {info['tile']}")
    return dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, tile_w=tw)), info


def bench_medium(args):
    """The medium workload's forward step (40x40x60 A cell, beta 95 deg, 5000 atoms,
    reflections to 2 A, 1024^2 detector, Voigt 3 deg eta .5, Hosemann g .03 lateral, 64x64
    nodes), folded, in the tile shape the tuner picks (or --medium-tile-w), the library's
    waves per tile; the same step unfolded beside it."""
    import workloads as W
    from paper_2608_23245_amd import binding as B
    wl = W.config1()
    if args.medium_tile_w:
        wl = dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, tile_w=args.medium_tile_w))
        tiles = {"tile": f"{args.medium_tile_w}x{64 // args.medium_tile_w}", "tuned": False}
    else:
        wl, tiles = tune_tiles(fold(wl))
    wl = fold(wl)
    ms_step, prof_ms, n_evals, state = forward_leg(wl, max(1, min(args.steps, 5)), 1)
    waves = B.launch_waves(B.make_model(wl).geom)
    ach = n_evals * SLOTS_PER_EVAL / (prof_ms * 1e-3)
    out = {"workload": wl.name, "n_hkl": int(state["hkl"].shape[0]), "culled_pairs": int(state["idx"].shape[0]),
           "useful_evals_per_step": int(n_evals), "ms_per_pattern": ms_step, "profile_kernel_ms": prof_ms,
           "evals_per_s": n_evals / (ms_step * 1e-3), "profile_kernel_evals_per_s": n_evals / (prof_ms * 1e-3),
           "issue_frac": ach / PEAK_SLOTS, "mirror_fold": fold_name(wl), "tile_tuning": tiles,
           "waves_per_tile": waves, "pass": "forward"}
    if wl.geom.mirror and not args.no_unfolded:
        # the folded launch's pairs per work unit, so that the computed rows can be compared bit for bit
        u = B.unit_pairs(int(state["idx"].shape[0]))
        wl0 = dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, mirror=0, tile_waves=waves, unit_pairs=u))
        ms0, prof0, n0, st0 = forward_leg(wl0, max(1, min(args.steps, 3)), 1)
        out["unfolded"] = {"ms_per_pattern": ms0, "profile_kernel_ms": prof0, "useful_evals_per_step": int(n0),
                           "waves_per_tile": waves, "profile_kernel_evals_per_s": n0 / (prof0 * 1e-3),
                           **compare_unfolded(wl, state["img"], st0["img"])}
        del st0
    del state
    return out


def bench_tilted(args):
    """The medium forward step with the fibre tilted 22 degrees toward the beam."""
    import workloads as W
    wl = fold(W.with_tilt(W.config1(), math.radians(22.0)))
    ms_step, prof_ms, n_evals, state = forward_leg(wl, max(1, min(args.steps, 3)), 1)
    return {"workload": wl.name, "culled_pairs": int(state["idx"].shape[0]), "useful_evals_per_step": int(n_evals),
            "ms_per_pattern": ms_step, "profile_kernel_ms": prof_ms, "evals_per_s": n_evals / (ms_step * 1e-3),
            "profile_kernel_evals_per_s": n_evals / (prof_ms * 1e-3), "pass": "forward"}


# Issue slots per useful evaluation of the other lineshapes (same accounting as above):
# Gaussian: 3 subtractions, max3, compare, sum of squares (3), scale (1), accumulate (1)
# and one exp2; Hosemann: 3 subtractions, max3, compare, 3 denominators, 2 products,
# accumulate and three cosines and one reciprocal.
# issue slots per useful evaluation of the adjoint kernel (k_profile_adj, Laue), the |y| + tiny
# guards not credited as in the forward: 39 full-rate operations (support test 5, the product
# of the y 2, the three sinc factors 8, their squares and product 5, G P and the three weighted
# sums 4, the three d/dN_i terms 15) and 3 sin + 3 cos + 1 rcp
ADJ_SLOTS_PER_EVAL = 39 + 7 * TRANS_SLOTS
SLOTS_PER_EVAL_LS = {"gaussian": 10 + 1 * TRANS_SLOTS, "hosemann": 11 + 4 * TRANS_SLOTS}


def bench_lineshapes(args):
    """The medium forward step with the Gaussian and the Hosemann lineshapes and the
    tutorial's axis damping B = (10, 10, 10) A^2."""
    import workloads as W
    out = {}
    for name, code in (("gaussian", 1), ("hosemann", 2)):
        wl = fold(W.with_disorder(W.config1(), lineshape=code, B_axis=(10.0, 10.0, 10.0)))
        ms_step, prof_ms, n_evals, state = forward_leg(wl, max(1, min(args.steps, 3)), 1)
        ach = n_evals * SLOTS_PER_EVAL_LS[name] / (prof_ms * 1e-3)
        out[name] = {"ms_per_pattern": ms_step, "profile_kernel_ms": prof_ms, "useful_evals_per_step": int(n_evals),
                     "evals_per_s": n_evals / (ms_step * 1e-3), "profile_kernel_evals_per_s": n_evals / (prof_ms * 1e-3),
                     "slots_per_eval": SLOTS_PER_EVAL_LS[name], "issue_frac": ach / PEAK_SLOTS}
        del state
    out["workload"] = "medium (as value), lineshape varied, axis damping B = (10, 10, 10) A^2"
    return out


def bench_splat(args, n_r=8, n_s=64):
    """Deterministic forward splat of the medium workload: n_r x n_s^2 shell samples per
    reflection, each evaluated by the direct sum and deposited at both diffraction-condition
    rotations."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2608_23245_amd import atoms_to_device
    from paper_2608_23245_amd import binding as B

    wl = W.config1()
    model = B.make_model(wl)
    ext = (wl.dis.g[0], wl.dis.g[1], wl.dis.g[2], wl.quad.extinction)
    hkl = B.enumerate_hkl(model.cell, wl.quad.d_min, wl.quad.d_max, extinction=ext)
    _, F2 = B.structure_factors(model.cell, atoms_to_device(wl.atoms), hkl, want_F=False)
    refl, _ = B.reflection_prep(model, hkl, F2)
    nodes = B.node_table(model)
    B.splat(model, hkl, refl, nodes, n_r, n_s)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(2)]
    for e0, e1 in evs:
        e0.record(stream)
        img = B.splat(model, hkl, refl, nodes, n_r, n_s)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    assert torch.isfinite(img).all() and img.max().item() > 0
    n_evals = B.splat(model, hkl, refl, nodes, n_r, n_s, count=True)
    samples = int(hkl.shape[0]) * n_r * n_s * n_s
    return {"workload": f"medium, {n_r} x {n_s}^2 samples per reflection", "n_hkl": int(hkl.shape[0]),
            "samples": samples, "useful_evals": int(n_evals), "splat_ms": ms, "samples_per_s": samples / (ms * 1e-3),
            "evals_per_s": n_evals / (ms * 1e-3), "evals_per_sample": n_evals / samples,
            "pass": "forward splat (binary64 sample geometry and projection, float32 direct sum)"}


def bench_cyl(args, n_sub=300):
    """Exact cylindrical average (periodic trapezoid rule over each pixel's ring, ring step
    equal to the pixel pitch in reciprocal space) over the medium detector for a seeded
    subset of the medium workload's reflections: every ring point within reach of a
    reflection's support is evaluated, several hundred times the gather's evaluations per
    reflection, so the full reflection list would take minutes per pattern."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2608_23245_amd import atoms_to_device
    from paper_2608_23245_amd import binding as B

    wl = fold(W.config1())
    g = wl.geom
    arc = g.pixel / g.distance / g.wavelength
    model = B.make_model(wl)
    ext = (wl.dis.g[0], wl.dis.g[1], wl.dis.g[2], wl.quad.extinction)
    hkl_all = B.enumerate_hkl(model.cell, wl.quad.d_min, wl.quad.d_max, extinction=ext)
    pick = np.sort(np.random.default_rng(12).choice(int(hkl_all.shape[0]), n_sub, replace=False))
    hkl = hkl_all[torch.from_numpy(pick).cuda()].contiguous()
    _, F2 = B.structure_factors(model.cell, atoms_to_device(wl.atoms), hkl, want_F=False)
    refl, _ = B.reflection_prep(model, hkl, F2)
    cull = B.cyl_records(model, hkl)
    nodes = B.node_table(model)
    pix, tile = B.pixel_map(model.geom)
    off, idx = B.cull(model.geom, tile, cull)
    order = B.tile_order(model.geom, off)
    B.profile_cyl(model, refl, nodes, pix, off, idx, arc, order=order)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(2)]
    for e0, e1 in evs:
        e0.record(stream)
        img = B.profile_cyl(model, refl, nodes, pix, off, idx, arc, order=order)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    assert torch.isfinite(img).all() and img.max().item() > 0
    n_evals = B.profile_cyl(model, refl, nodes, pix, off, idx, arc, count=True, order=order)
    achieved = n_evals * SLOTS_PER_EVAL / (ms * 1e-3) / 1e12
    return {"workload": f"medium detector, {n_sub} of its reflections (seeded pick), ring step {arc:.4g} 1/A",
            "n_hkl": n_sub, "pairs": int(idx.shape[0]), "useful_evals": int(n_evals), "cyl_ms": ms,
            "evals_per_s": n_evals / (ms * 1e-3), "kernel": "k_cyl<false, 0>",
            "slots": {"achieved": achieved, "peak": PEAK_SLOTS / 1e12, "unit": "Tslot/s",
                      "frac": achieved / (PEAK_SLOTS / 1e12)},
            "pass": "exact cylindrical average (float32 evaluation, binary64 ring geometry)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path shards by reflections "
              "across GPUs with one image all-reduce, which this build does not implement.", file=sys.stderr)
        sys.exit(2)
    import torch

    import workloads as W

    torch.cuda.set_device(0)
    if args.only_batch:
        print(json.dumps({"batched_forward": bench_batched_forward(args)}), flush=True)
        return
    wl = W.config2()
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    MIRROR["on"] = not args.no_mirror
    MIRROR["updown"] = not args.no_updown
    # the first pattern of the process (code objects loaded, first allocations), timed alone;
    # not in the runs with a fixed tile width (the profiler runs, whose kernel averages must be
    # those of the timed steps)
    cold_ms = None
    if not args.tile_w:
        from paper_2608_23245_amd import Pipeline
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Pipeline(fold(wl)).pattern()
        torch.cuda.synchronize()
        cold_ms = (time.perf_counter() - t0) * 1e3
        log(f"cold first pattern: {cold_ms:.0f} ms")
        torch.cuda.empty_cache()
    if args.tile_w:
        wl = dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, tile_w=args.tile_w))
        tiles = {"tile": f"{args.tile_w}x{64 // args.tile_w}", "tuned": False}
    else:
        wl, tiles = tune_tiles(fold(wl))
    wl = fold(wl)
    ms_step, prof_ms, n_evals, state = forward_leg(wl, args.steps, args.warmup)
    from paper_2608_23245_amd import binding as B
    waves_main = B.launch_waves(B.make_model(wl).geom)
    log(f"forward: {ms_step:.1f} ms/step, profile kernel {prof_ms:.1f} ms, {n_evals:.4e} useful evaluations")
    slots = n_evals * SLOTS_PER_EVAL
    achieved = slots / (prof_ms * 1e-3) / 1e12
    peak = PEAK_SLOTS / 1e12
    out = {
        "metric": "profile-quadrature evals/s & ms/pattern (fwd, fwd+bwd, batched) at stated tol",
        "value": n_evals / (ms_step * 1e-3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_hkl": int(state["hkl"].shape[0]), "pixels": wl.geom.width * wl.geom.height,
                   "tile": tiles["tile"], "mirror_fold": fold_name(wl), "waves_per_tile": waves_main,
                   "nodes": wl.quad.n_nodes ** 2, "culled_pairs": int(state["idx"].shape[0]),
                   "useful_evals_per_step": int(n_evals), "pass": "forward"},
        "ms_per_pattern": ms_step,
        "cold_first_pattern_ms": cold_ms,
        "profile_kernel_ms": prof_ms,
        "profile_kernel_evals_per_s": n_evals / (prof_ms * 1e-3),
        "tile_tuning": tiles,
        "rates": other_rates(n_evals / (prof_ms * 1e-3), prof_ms),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tslot/s", "frac": achieved / peak,
                     "traffic": measured_traffic(), "kernel": "k_profile_units<0>",
                     "sources_sha": profile_source_sha(), "slots_per_eval": SLOTS_PER_EVAL},
    }
    if wl.geom.mirror and not args.no_unfolded and not args.only_headline:
        # the same forward step without the folds, for reference (with the folded launch's pairs
        # per work unit, so that the computed pixels can be compared bit for bit)
        u = B.unit_pairs(int(state["idx"].shape[0]))
        wl0 = dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, mirror=0, tile_waves=waves_main, unit_pairs=u))
        ms0, prof0, n0, st0 = forward_leg(wl0, 1, 1)
        out["unfolded"] = {"ms_per_pattern": ms0, "profile_kernel_ms": prof0, "useful_evals_per_step": int(n0),
                           "waves_per_tile": waves_main, "profile_kernel_evals_per_s": n0 / (prof0 * 1e-3),
                           **compare_unfolded(wl, state["img"], st0["img"])}
        del st0
        torch.cuda.empty_cache()
    if not args.no_cpu and not args.only_headline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(wl, state, args.cpu_block, args.cpu_one_core_pixels)
    del state
    torch.cuda.empty_cache()
    if args.only_headline:
        print(json.dumps(out), flush=True)
        return
    if not args.no_medium:
        log("forward, medium workload")
        out["medium"] = bench_medium(args)
        torch.cuda.empty_cache()
    if not args.no_tilt:
        log("forward, tilted fibre")
        out["tilted"] = bench_tilted(args)
        torch.cuda.empty_cache()
    if not args.no_lineshapes:
        log("forward, Gaussian and Hosemann lineshapes")
        out["lineshapes"] = bench_lineshapes(args)
        torch.cuda.empty_cache()
    if not args.no_cyl:
        log("cylindrical average leg")
        out["cyl"] = bench_cyl(args)
    if not args.no_splat:
        log("forward splat")
        out["splat"] = bench_splat(args)
        torch.cuda.empty_cache()
    if not args.no_bwd:
        log("forward + adjoint")
        out["fwd_bwd"] = bench_fwd_bwd(args)
        torch.cuda.empty_cache()
    if not args.no_batch:
        log(f"batched: {args.batch_models} models")
        out["batched"] = bench_batched(args)
    print(json.dumps(out), flush=True)


def bench_fwd_bwd(args):
    """Refinement step on the medium model: structure factors, pattern, pixel weights of the
    weighted residual against a target image, and the hand-written adjoint down to the atom
    and global gradients.  The target is the image of the perturbed target model."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2608_23245_amd import autograd as AG
    from paper_2608_23245_amd import binding as B

    gw = W.config3()
    gw = dataclasses.replace(gw, model=fold(gw.model), target=fold(gw.target))
    eng_t = AG.PatternEngine(gw.target)
    ta = gw.target.atoms
    at_t = eng_t.atoms(*(torch.as_tensor(v) for v in (ta.x, ta.y, ta.z, ta.B, ta.occ)))
    _, F2t = B.structure_factors(eng_t.cell, at_t, eng_t.hkl)
    target = eng_t.plan.run(eng_t.hkl, F2t).clone()
    del eng_t, at_t, F2t
    torch.cuda.empty_cache()
    eng = AG.PatternEngine(gw.model)
    a = gw.model.atoms
    atoms = eng.atoms(*(torch.as_tensor(v) for v in (a.x, a.y, a.z, a.B, a.occ)))
    w = 1.0 / (target + 1e-3 * target.max())
    stream = torch.cuda.current_stream()
    res = {}

    def step(ev=None):
        F, F2 = B.structure_factors(eng.cell, atoms, eng.hkl)
        img = eng.plan.run(eng.hkl, F2)
        G = (2.0 * w * (img - target)).contiguous()
        if ev is not None:
            ev[0].record(stream)
        out, glob, _ = B.pattern_backward(eng.plan, eng.hkl, F, G, atoms)
        if ev is not None:
            ev[1].record(stream)
        res.update(img=img, G=G, glob=glob)

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    bwd_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    loss = float((w * (res["img"] - target) ** 2).sum().item())
    assert np.isfinite(loss) and torch.isfinite(res["glob"]).all()
    # the profile adjoint kernel alone, on the same pattern and pixel weights, against its
    # evaluations (the forward's support-passing triples: tiles it skips carry no weight)
    model = eng.plan.model
    _, F2 = B.structure_factors(eng.cell, atoms, eng.hkl)
    refl, cull = B.reflection_prep(model, eng.hkl, F2)
    nodes = B.node_table(model)
    pix, tile = B.pixel_map(model.geom)
    off, idx = B.cull(model.geom, tile, cull)
    order = B.tile_order(model.geom, off)
    G = res["G"]
    bws = B.balanced_workspace(model, int(idx.shape[0]))
    B.profile_balanced(model, refl, nodes, pix, tile, off, idx, order=order, ws=bws)  # the work units
    B.profile_adjoint_balanced(model, refl, nodes, pix, tile, off, idx, G, bws, order=order)
    torch.cuda.synchronize()
    aev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(2)]
    for e0, e1 in aev:
        e0.record(stream)
        B.profile_adjoint_balanced(model, refl, nodes, pix, tile, off, idx, G, bws, order=order)
        e1.record(stream)
    torch.cuda.synchronize()
    adj_ms = float(np.mean([a.elapsed_time(b) for a, b in aev]))
    n_evals = B.profile(model, refl, nodes, pix, tile, off, idx, count=True)
    achieved = n_evals * ADJ_SLOTS_PER_EVAL / (adj_ms * 1e-3) / 1e12
    return {"workload": "refinement: medium model vs perturbed target (xyz N(0,0.1 A), B x1.2, sigma 3.5 deg, g .035), "
                        "loss sum w (I - T)^2, w = 1/(T + 1e-3 max T)",
            "ms_per_step": ms, "backward_ms": bwd_ms, "forward_ms": ms - bwd_ms, "loss": loss,
            "profile_adjoint_ms": adj_ms, "useful_evals": int(n_evals), "kernel": "k_profile_adj_units<0>",
            "slots": {"achieved": achieved, "peak": PEAK_SLOTS / 1e12, "unit": "Tslot/s",
                      "frac": achieved / (PEAK_SLOTS / 1e12), "slots_per_eval": ADJ_SLOTS_PER_EVAL},
            "steps": args.steps, "pass": "forward + adjoint (atoms xyz/B/occ, sigma, gamma, N_base, g)"}


def bench_batched_forward(args):
    """The batched forward alone, every model in tile width --batch-tile-w (folded where its
    geometry allows): one warm-up forward, then --steps forwards timed with HIP events."""
    import torch

    import workloads as W
    from paper_2608_23245_amd.batch import BatchEngine

    tw = args.batch_tile_w
    wls = [fold(dataclasses.replace(w, geom=dataclasses.replace(w.geom, tile_w=tw)))
           for w in W.config4(n_models=args.batch_models)]
    t0 = time.perf_counter()
    be = BatchEngine(wls, "cuda", stacked=not args.batch_per_tile)
    be.forward()
    torch.cuda.synchronize()
    log(f"batched forward: set-up and warm-up {time.perf_counter() - t0:.1f} s, {be.totals['pair']} pairs")
    ms = []
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        be.forward()
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    log(f"batched forward: {', '.join(f'{m:.1f}' for m in ms)} ms")
    return {"n_models": len(wls), "tile": f"{tw}x{64 // tw}", "culled_pairs": int(be.totals["pair"]),
            "stacked_pairs": int(be.totals.get("stacked_pair", 0)) if be.stacked else None, "forward_ms": ms}


def bench_batched(args):
    """Batched refinement step (forward + adjoint of every model) captured in one HIP graph,
    against the plain single-model forward of each model run one after the other.  Set-up
    (not timed) picks the batch's pixel-tile shape by timing its forward in each candidate
    shape (autotune.tune_batch)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2608_23245_amd import binding as B
    from paper_2608_23245_amd.autotune import tune_batch
    from paper_2608_23245_amd.batch import GraphStep

    wls = [fold(w) for w in W.config4(n_models=args.batch_models)]
    t0 = time.perf_counter()
    be, tile_ms = tune_batch(wls, candidates=(8, 16, 4))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    shapes = {f"{c}x{64 // c}": be.tile_w.count(c) for c in sorted(set(be.tile_w))}
    tile_ms = {f"{c}x{64 // c}": round(v, 1) for c, v in tile_ms.items()}
    log(f"batched: set-up {setup_s:.1f} s (batched forward per tile shape {tile_ms} ms -> {shapes}), "
        f"{be.totals['pair']} culled pairs")
    glob = be.globals()
    tglob = glob.clone()
    tglob[:, 0] *= 1.1
    be.set_globals(tglob)
    target = be.forward().clone()
    be.set_globals(glob)
    # useful evaluations: counting pass of the single-model kernel on each model's part of the batch
    be.forward()
    torch.cuda.synchronize()
    n_evals = 0
    for m, mod in enumerate(be.models):
        e = be._host_entries[m]
        refl = be.refl[e.hkl_off:e.hkl_off + e.n_hkl]
        nodes = be.nodes[e.node_off:e.node_off + B.node_rows(wls[m].quad.n_nodes)]
        pix = be.pix[e.pix_off:e.pix_off + wls[m].geom.width * wls[m].geom.height]
        tile = be.tile[e.tile_off:e.tile_off + e.n_tiles]
        rowptr = be.rowptr[e.rowptr_off:e.rowptr_off + e.n_tiles + 1]
        idx = be.idx[e.pair_off:e.pair_off + max(be.list_len[m], 1)]
        n_evals += B.profile(mod, refl, nodes, pix, tile, rowptr, idx, count=True)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    be.forward()
    e1.record(stream)
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1)
    log(f"batched: forward {fwd_ms:.1f} ms; capturing the refinement step")
    step = GraphStep(be, target)
    step.capture()
    torch.cuda.synchronize()
    log(f"batched: {args.batch_steps} graph replays")
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        step.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.batch_steps
    assert torch.isfinite(be.d_globals).all()
    del step
    # plain single-model forwards, one after the other (each with its own culling)
    from paper_2608_23245_amd import Pipeline
    torch.cuda.synchronize()
    single_ms = 0.0
    log(f"batched: graph step {ms:.1f} ms; single-model forwards")
    for m, wl in enumerate(wls):
        if m % 64 == 63:
            log(f"batched: single-model forwards {m + 1}/{len(wls)}")
        pipe = Pipeline(wl)
        _, F2 = pipe.structure_factors()
        pipe.pattern(F2)              # sizes the plan's culling capacity
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, F2 = pipe.structure_factors()
        pipe.pattern(F2)
        torch.cuda.synchronize()
        single_ms += (time.perf_counter() - t0) * 1e3
        del pipe
    return {"workload": f"{len(wls)} ragged models (edges U(10,80) A, 500-20000 atoms, 256^2-1024^2 px, "
                        "Voigt sigma U(1,8) deg, eta U(0,1), g U(0,.06), d_min U(2,3) A, 32x32 nodes)",
            "n_models": len(wls), "n_hkl": int(be.totals["hkl"]), "pixels": int(be.totals["pix"]),
            "culled_pairs": int(be.totals["pair"]), "useful_evals_per_forward": int(n_evals),
            "setup_s": setup_s, "tile_shapes": shapes, "tile_tuning_forward_ms": tile_ms, "graph_ms_per_step": ms, "graph_steps": args.batch_steps,
            "batched_forward_ms": fwd_ms, "batched_forward_evals_per_s": n_evals / (fwd_ms * 1e-3),
            "sum_single_forward_ms": single_ms,
            "forward_speedup_vs_single": single_ms / fwd_ms,
            "pass": "one HIP graph: batched forward + pixel weights + batched adjoint of all models"}


def cpu_baseline(wl, state, block, n_one):
    """The FP64 oracle as it stands on a bounded sample of the same workload: the block x block
    pixels whose lower-left pixel is (width/2 + 128, height/2 + 256), over the whole reflection
    list with the oracle's own exact skip.  The structure factors of the reflections that can
    reach the block come first from the oracle's C loop (not timed); then oracle_pattern is
    timed on all the host threads over the block and on one thread over its first n_one pixels.
    The GPU image on the block is compared with the oracle's as a check of the sample."""
    import numpy as np
    import torch

    from oracle import oracle as O
    g = wl.geom
    i0, j0 = g.width // 2 + 128, g.height // 2 + 256
    q = np.array([(j0 + dj) * g.width + (i0 + di) for dj in range(block) for di in range(block)], dtype=np.int64)
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    hkl = np.ascontiguousarray(hkl[~O.extinct_mask(hkl, wl.dis, wl.quad.extinction)])
    R, Z = O.pixel_rz(g)
    Rq, Zq = R.ravel()[q], Z.ravel()[q]
    del R, Z
    t0 = time.perf_counter()
    sub = O.reachable(wl, hkl, Rq, Zq)
    hs = np.ascontiguousarray(hkl[sub])
    P = O.prepare(wl, hkl=hs, F=O.structure_factors_c(hs, wl.cell, wl.atoms), cull_extinct=False)
    setup_s = time.perf_counter() - t0
    threads = O.threads()
    t0 = time.perf_counter()
    vals, n = O.pattern_at(P, Rq, Zq, count=True)
    dt = time.perf_counter() - t0
    O.set_threads(1)
    try:
        t0 = time.perf_counter()
        _, n1 = O.pattern_at(P, Rq[:n_one], Zq[:n_one], count=True)
        dt1 = time.perf_counter() - t0
    finally:
        O.set_threads(threads)
    got = state["img"].reshape(-1)[torch.as_tensor(q, device="cuda")].cpu().numpy().astype(np.float64)
    rel = float(np.linalg.norm(got - vals) / np.linalg.norm(vals))
    log(f"cpu baseline: {n / dt:.3e} evals/s on {threads} threads, {n1 / dt1:.3e} on one")
    return {"value": n / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{block}x{block} pixels of the {g.width}x{g.height} image from ({i0}, {j0}) ({n} useful "
                      f"evaluations, {dt:.1f} s on {threads} threads), over all {hkl.shape[0]} reflections with the "
                      f"oracle's exact skip ({sub.size} can reach the block; their structure factors took "
                      f"{setup_s:.1f} s, not timed); GPU vs oracle rel-L2 on the block {rel:.1e}",
            "one_core": {"value": n1 / dt1, "unit": "evals/s", "cores": 1,
                         "sample": f"the first {n_one} pixels of the block ({n1} useful evaluations, {dt1:.1f} s)"}}


if __name__ == "__main__":
    main()
