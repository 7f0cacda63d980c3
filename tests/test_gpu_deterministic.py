"""The fixed-order adjoint (fdtbx_pattern_backward_deterministic, fdtbx_batch_backward_
deterministic): every output reproducible bit for bit across runs and HIP-graph replays, and
equal to the atomic-add adjoint to binary64 rounding of the sums (float32 outputs within a
few units in the last place); the reflection-major pair order is a stable sort of the lists."""
import dataclasses
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2608_23245_amd import autograd as AG  # noqa: E402
from paper_2608_23245_amd import binding as B  # noqa: E402
from paper_2608_23245_amd.batch import BatchEngine, GraphStep  # noqa: E402

DEG = math.pi / 180


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def backward(wl, G, deterministic):
    eng = AG.PatternEngine(wl)
    a = wl.atoms
    atoms = eng.atoms(*(torch.as_tensor(v) for v in (a.x, a.y, a.z, a.B, a.occ)))
    F, F2 = B.structure_factors(eng.cell, atoms, eng.hkl)
    eng.plan.run(eng.hkl, F2)
    Gt = torch.as_tensor(G, dtype=torch.float32).cuda().contiguous()
    out, glob, dF2 = B.pattern_backward(eng.plan, eng.hkl, F, Gt, atoms, deterministic=deterministic)
    torch.cuda.synchronize()
    return eng, {k: v.cpu().numpy() for k, v in out.items()}, glob.cpu().numpy(), dF2.cpu().numpy()


def medium_crop(mirror):
    wl = W.config1()
    g = dataclasses.replace(wl.geom, width=128, height=128, center_x=64.0, center_y=64.0, tile_w=16, mirror=mirror)
    return dataclasses.replace(wl, geom=g)


@pytest.mark.parametrize("mirror", [0, 3])
def test_deterministic_backward_repeats_bit_for_bit(mirror):
    """The medium model on a centred 128x128 crop of its detector (16x4 tiles, folds as given):
    three deterministic backward passes give identical bits, and they agree with the atomic-add
    pass (which the adjoint tests hold to the oracle) to 1e-5 of each group's largest value."""
    wl = medium_crop(mirror)
    G = np.random.default_rng(21).normal(size=(wl.geom.height, wl.geom.width))
    say(f"deterministic backward, medium model on a 128x128 crop, mirror bits {mirror}")
    runs = [backward(wl, G, True) for _ in range(3)]
    _, o0, g0, f0 = runs[0]
    for _, o, g, f in runs[1:]:
        for k in o0:
            assert np.array_equal(o[k], o0[k]), k
        assert np.array_equal(g, g0) and np.array_equal(f, f0)
    _, oa, ga, fa = backward(wl, G, False)
    for k in o0:
        err = np.abs(oa[k] - o0[k]).max() / np.abs(o0[k]).max()
        say(f"  {k}: atomic vs fixed order {err:.1e} of the largest")
        assert err <= 1e-5
    # the fixed-order sums pass through float32 per pair: agreement to float32 rounding
    assert np.abs(ga - g0).max() <= 1e-6 * np.abs(g0).max()
    assert np.abs(fa - f0).max() <= 1e-5 * np.abs(f0).max()


def test_pair_transpose_is_a_stable_sort():
    """fdtbx_pair_transpose on the culling lists of a small workload: every reflection's pairs
    in ascending list position (numpy's stable argsort of the same keys), row pointers as its
    searchsorted; and the pair count read on the device masks the capacity's tail."""
    wl = W.small(7, width=40, height=36, sigma_theta=3 * DEG, gamma_theta=1 * DEG)
    model = B.make_model(wl)
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    h = torch.from_numpy(np.ascontiguousarray(hkl)).cuda()
    _, cull = B.reflection_prep(model, h, torch.ones(h.shape[0], dtype=torch.float32, device="cuda"))
    pix, tile = B.pixel_map(model.geom)
    off, idx = B.cull(model.geom, tile, cull)
    n = int(hkl.shape[0])
    ptr, pairs = B.pair_transpose(n, idx)
    keys = idx.cpu().numpy().astype(np.int64)
    perm = np.argsort(keys, kind="stable")
    assert np.array_equal(pairs.cpu().numpy(), perm)
    assert np.array_equal(ptr.cpu().numpy(), np.searchsorted(keys[perm], np.arange(n + 1)))
    # a longer buffer whose tail is not pairs: the count comes from the device
    pad = torch.cat([idx, torch.zeros(17, dtype=torch.int32, device="cuda")])
    cnt = torch.tensor([keys.size], dtype=torch.int64, device="cuda")
    ptr2, pairs2 = B.pair_transpose(n, pad, cnt)
    assert np.array_equal(ptr2.cpu().numpy(), ptr.cpu().numpy())
    assert np.array_equal(pairs2[:keys.size].cpu().numpy(), perm)


def test_deterministic_batch_graph_replays_bit_for_bit():
    """A small batch with the fixed-order adjoint, captured in a HIP graph: every replay gives
    the eager step's gradients bit for bit, and they agree with the atomic-add batch."""
    wls = [W.small(71, n_atoms=30, width=32, height=16, center=(16.0, 8.0), sigma_theta=3 * DEG, gamma_theta=1 * DEG,
                   g=(0.02, 0.02, 0.0)),
           W.small(72, n_atoms=20, width=24, height=20, sigma_theta=0.0, gamma_theta=2 * DEG)]
    g0 = dataclasses.replace(wls[0].geom, tile_w=16, mirror=3)
    wls[0] = dataclasses.replace(wls[0], geom=g0)
    be = BatchEngine(wls, deterministic=True)
    tgt = BatchEngine(wls)
    glob = tgt.globals()
    glob[:, 0] *= 1.1
    tgt.set_globals(glob)
    target = tgt.forward().clone()
    del tgt
    step = GraphStep(be, target)
    step.eager()
    torch.cuda.synchronize()
    ref_g = {k: v.clone() for k, v in be.grads.items()}
    ref_glob = be.d_globals.clone()
    ref_dF2 = be.dF2.clone()
    step.capture()
    for rep in range(3):
        be.d_globals.fill_(0.0)
        for v in be.grads.values():
            v.fill_(0.0)
        torch.cuda.synchronize()
        step.replay()
        torch.cuda.synchronize()
        for k in ref_g:
            assert torch.equal(be.grads[k], ref_g[k]), (rep, k)
        assert torch.equal(be.d_globals, ref_glob) and torch.equal(be.dF2, ref_dF2), rep
        say(f"  replay {rep}: bit-identical")
    ba = BatchEngine(wls)
    ba.forward()
    G = (2.0 * step.weight * (be.image - target)).contiguous()
    ga, gga = ba.backward(G)
    torch.cuda.synchronize()
    for k in ref_g:
        d = (ga[k] - ref_g[k]).abs().max().item()
        assert d <= 1e-5 * ref_g[k].abs().max().item(), k
    assert (gga - ref_glob).abs().max().item() <= 1e-6 * ref_glob.abs().max().item()
