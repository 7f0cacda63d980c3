"""The single-model pattern path without a host round trip (fdtbx_profile_pattern_async):
device-written statistics (reflections, culling pairs, useful evaluations, per-step device
times), the pair capacity checked on the device (an overflow leaves the lists empty, the image
zero and the flag set), and a HIP-graph capture whose every replay reproduces the eager image
bit for bit, with the program's own work and synchronisations between the replays."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2608_23245_amd import Pipeline  # noqa: E402
from paper_2608_23245_amd import binding as B  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_async_pattern_stats_and_overflow():
    wl = W.config0()
    pipe = Pipeline(wl)
    _, F2 = pipe.structure_factors()
    ref = pipe.pattern(F2)
    plan = B.PatternPlan(pipe.model, pipe.n_hkl, pair_cap=16)   # far too small
    out = torch.full_like(ref, -1.0)
    st = B.new_stats()
    plan.run_async(pipe.hkl, F2, out, st)
    s = B.read_stats(st)
    say(f"  capacity 16: {s}")
    assert s["overflow"] and s["n_pairs"] > 16 and s["pair_cap"] == 16 and s["n_hkl"] == pipe.n_hkl
    assert torch.count_nonzero(out).item() == 0                # empty lists: a zero image
    plan.grow(s["n_pairs"])
    plan.run_async(pipe.hkl, F2, out, st, count=True)
    s = B.read_stats(st)
    say(f"  capacity {plan.pair_cap}: {s}")
    assert not s["overflow"] and torch.equal(out, ref)
    # the counting pass agrees with the oracle's count of support-passing triples
    _, n_ref = O.pattern(wl, O.prepare(wl, hkl=pipe.hkl.cpu().numpy()), count=True)
    assert abs(s["useful_evals"] - n_ref) <= 1e-4 * n_ref
    assert s["clock_khz"] > 0 and all(v >= 0 for v in s["ms"].values()) and s["total_ms"] > 0


def test_async_pattern_graph_replays():
    """The medium workload (both folds, 16x4 tiles) captured once; between replays the program
    clears the image and changes |F|^2 in place; every replay equals the eager image for the
    |F|^2 it saw."""
    import dataclasses
    wl = W.config1()
    wl = dataclasses.replace(wl, geom=dataclasses.replace(wl.geom, tile_w=16, mirror=3))
    pipe = Pipeline(wl)
    _, F2 = pipe.structure_factors()
    F2 = F2.clone()
    plan = B.PatternPlan(pipe.model, pipe.n_hkl)
    out = torch.empty((wl.geom.height, wl.geom.width), dtype=torch.float32, device="cuda")
    st = B.new_stats()
    plan.run_async(pipe.hkl, F2, out, st)              # sizes the capacity
    first = B.read_stats(st)
    if first["overflow"]:
        plan.grow(first["n_pairs"])
    scales = [1.0, 0.5, 2.0]
    eager = []
    base = F2.clone()
    for c in scales:
        F2.copy_(base * c)
        plan.run_async(pipe.hkl, F2, out, st)
        torch.cuda.synchronize()
        eager.append(out.clone())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.run_async(pipe.hkl, F2, out, st)          # warm-up on the side stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run_async(pipe.hkl, F2, out, st)
    torch.cuda.synchronize()
    for rep in range(2):
        for k, c in enumerate(scales):
            out.fill_(-1.0)
            F2.copy_(base * c)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, eager[k]), (rep, c)
            info = B.read_stats(st)
            assert not info["overflow"] and info["n_pairs"] == first["n_pairs"]
        say(f"  replay round {rep}: images identical to the eager ones; {info['ms']}")
