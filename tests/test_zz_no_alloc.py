"""fdtbx_pattern_backward_noalloc, the backward pass whose workspace is the library's own device
scratch array, against fdtbx_pattern_backward with a caller-given workspace: the same
gradients on two calls in a row, the second on a smaller problem (so the array still holds the
first call's contents), and sizes beyond the array refused on the host before any launch."""
import ctypes
import dataclasses
import math
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2608_23245_amd import autograd as AG  # noqa: E402
from paper_2608_23245_amd import binding as B  # noqa: E402

DEG = math.pi / 180


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def backward(eng, F, Gt, atoms, noalloc):
    if noalloc:
        out, glob, dF2 = B.pattern_backward_noalloc(eng.plan, eng.hkl, F, Gt, atoms)
    else:
        out, glob, dF2 = B.pattern_backward(eng.plan, eng.hkl, F, Gt, atoms)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}, glob.cpu().numpy(), dF2.cpu().numpy()


def medium_crop():
    wl = W.config1()
    g = dataclasses.replace(wl.geom, width=128, height=128, center_x=64.0, center_y=64.0, tile_w=16, mirror=3)
    return dataclasses.replace(wl, geom=g)


def close(got, ref, what):
    # both calls run the same kernels on the same inputs; only the order of the binary64 atomic
    # adds of the per-reflection sums differs, which float32 outputs see as a few ulps
    err = float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))
    say(f"    {what}: {err:.1e} of the largest")
    assert err <= 1e-5, (what, err)


def test_noalloc_backward_matches_the_workspace_call_twice():
    cases = [("medium model, 128x128 crop, 5000 atoms", medium_crop()),
             ("small model, 24 atoms", W.small(31, width=20, height=18, sigma_theta=3 * DEG, gamma_theta=1 * DEG))]
    for name, wl in cases:
        eng = AG.PatternEngine(wl)
        a = wl.atoms
        atoms = eng.atoms(*(torch.as_tensor(v) for v in (a.x, a.y, a.z, a.B, a.occ)))
        F, F2 = B.structure_factors(eng.cell, atoms, eng.hkl)
        eng.plan.run(eng.hkl, F2)
        G = np.random.default_rng(5).normal(size=(wl.geom.height, wl.geom.width))
        Gt = torch.as_tensor(G, dtype=torch.float32).cuda().contiguous()
        need = B.lib().fdtbx_backward_workspace(eng.plan.n_hkl, int(a.x.shape[0]))
        say(f"no-alloc backward, {name}: {eng.plan.n_hkl} reflections, workspace {need} bytes")
        assert need <= B.NOALLOC_SCRATCH_BYTES
        ref = backward(eng, F, Gt, atoms, False)
        got = backward(eng, F, Gt, atoms, True)
        for k in ref[0]:
            close(got[0][k], ref[0][k], k)
        close(got[1], ref[1], "globals")
        close(got[2], ref[2], "dF2")


def test_noalloc_backward_refuses_sizes_beyond_the_scratch():
    wl = W.small(32, width=12, height=10)
    eng = AG.PatternEngine(wl)
    a = wl.atoms
    atoms = eng.atoms(*(torch.as_tensor(v) for v in (a.x, a.y, a.z, a.B, a.occ)))
    F, F2 = B.structure_factors(eng.cell, atoms, eng.hkl)
    eng.plan.run(eng.hkl, F2)
    G = torch.zeros(wl.geom.height, wl.geom.width, dtype=torch.float32, device="cuda")
    # a reflection count whose workspace exceeds the array: refused before anything is read
    n_big = B.NOALLOC_SCRATCH_BYTES // 40
    assert B.lib().fdtbx_backward_workspace(n_big, 0) > B.NOALLOC_SCRATCH_BYTES
    L = B.lib()
    glob = torch.empty(B.N_GLOBALS, dtype=torch.float64, device="cuda")
    rc = L.fdtbx_pattern_backward_noalloc(ctypes.byref(eng.plan.model), B._ptr(eng.hkl), n_big, B._ptr(F),
                                          B._ptr(G), B._ptr(eng.plan.ws), eng.plan.ws_bytes, eng.plan.pair_cap, 0,
                                          *([None] * 7), 1, *([None] * 5), B._ptr(glob), None, B._stream())
    assert rc == -3, rc  # FDTBX_ERR_BUFFER_TOO_SMALL
    assert b"scratch" in L.fdtbx_error_string(rc)
