"""Batched models (fdtbx_batch_forward / fdtbx_batch_backward, persistent launches):
each model's image and gradients equal its unbatched run (and the oracle for one
model), parameters update in place on the device, and a HIP-graph replay of the
refinement step reproduces the eager step on every replay."""
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

from paper_2608_23245_amd import Pipeline  # noqa: E402
from paper_2608_23245_amd import autograd as AG  # noqa: E402
from paper_2608_23245_amd import binding as B  # noqa: E402
from paper_2608_23245_amd.batch import BatchEngine, GraphStep  # noqa: E402

DEG = math.pi / 180


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_batch():
    return [
        W.small(61, n_atoms=40, width=24, height=20, sigma_theta=3 * DEG, gamma_theta=1 * DEG, g=(0.02, 0.02, 0.0)),
        W.small(62, n_atoms=15, width=17, height=29, sigma_theta=0.0, gamma_theta=2 * DEG, n_nodes=20,
                cell=W.Cell(8.0, 12.0, 10.0, 90 * DEG, 104 * DEG, 90 * DEG), center=(5.2, 14.7)),
        W.small(63, n_atoms=60, width=32, height=32, sigma_theta=4 * DEG, gamma_theta=0.0, g=(0.03, 0.0, 0.01),
                n_nodes=16, d_min=4.0, lineshape=1, B_axis=(3.0, 5.0, 1.0)),
        W.small(64, n_atoms=25, width=9, height=40, sigma_theta=2 * DEG, gamma_theta=2 * DEG, center=(-6.0, 20.0)),
        W.small(65, n_atoms=33, width=27, height=11, sigma_theta=5 * DEG, gamma_theta=0.5 * DEG, n_nodes=10,
                cell=W.Cell(11.0, 9.5, 12.5, 95 * DEG, 90 * DEG, 100 * DEG), lineshape=2, g=(0.02, 0.01, 0.0),
                tilt=15 * DEG),
    ]


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def single_backward(wl, G):
    eng = AG.PatternEngine(wl)
    a = wl.atoms
    atoms = eng.atoms(*(torch.as_tensor(v) for v in (a.x, a.y, a.z, a.B, a.occ)))
    F, F2 = B.structure_factors(eng.cell, atoms, eng.hkl)
    img = eng.plan.run(eng.hkl, F2)
    out, glob, _ = B.pattern_backward(eng.plan, eng.hkl, F, G.contiguous(), atoms)
    return img, out, glob


def test_batch_forward_and_backward_match_single_runs():
    wls = small_batch()
    say("batch of", len(wls))
    be = BatchEngine(wls)
    img = be.forward()
    rng = np.random.default_rng(3)
    G = torch.as_tensor(rng.normal(size=img.shape[0]), dtype=torch.float32).cuda()
    grads, glob = be.backward(G)
    torch.cuda.synchronize()
    for m, wl in enumerate(wls):
        Gm = G[be.pix_off[m]:be.pix_off[m + 1]].view(*be.shapes[m])
        ref_img, ref_out, ref_glob = single_backward(wl, Gm)
        r = rel(be.image_of(m).cpu().numpy(), ref_img.cpu().numpy())
        say(f"  model {m}: image rel-L2 vs single {r:.2e}")
        assert r <= 1e-5
        a0, a1 = be.atom_off[m], be.atom_off[m + 1]
        for k in ("x", "y", "z", "B", "occ"):
            got = grads[k][a0:a1].cpu().numpy()
            ref = ref_out[k].cpu().numpy()
            err = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)
            assert err <= 1e-4, (m, k, err)
        gg, rg = glob[m].cpu().numpy(), ref_glob.cpu().numpy()
        assert np.all(np.abs(gg - rg) <= 1e-4 * np.abs(rg) + 1e-12 * np.abs(rg).max()), (m, gg, rg)


def test_batch_model_against_oracle():
    wls = small_batch()
    be = BatchEngine(wls)
    be.forward()
    torch.cuda.synchronize()
    m = 1
    wl = wls[m]
    say("batch model vs oracle")
    hkl = be.hkl[be.hkl_off[m]:be.hkl_off[m + 1]].cpu().numpy()
    ref = O.pattern(wl, O.prepare(wl, hkl=hkl, cull_extinct=False))
    got = be.image_of(m).cpu().numpy().astype(np.float64)
    r = rel(got, ref)
    big = ref > 1e-3 * ref.max()
    px = float(np.max(np.abs(got[big] - ref[big]) / ref[big]))
    say(f"  rel-L2 {r:.2e}, per-pixel {px:.2e}")
    assert r <= 1e-4 and px <= 1e-3


def test_batch_set_globals_in_place():
    wls = small_batch()
    be = BatchEngine(wls)
    glob = be.globals()
    glob[0, 0] *= 1.3          # sigma_theta of model 0
    glob[2, 5] = 0.02          # g_a of model 2
    glob[3, 3] *= 0.8          # N_base_b of model 3
    glob[4, 9] = 4.0           # B_b of model 4
    be.set_globals(glob)
    be.forward()
    torch.cuda.synchronize()
    import copy
    for m in (0, 2, 3, 4):
        wl = copy.deepcopy(wls[m])
        g = glob[m].cpu().tolist()
        wl.dis.sigma_theta, wl.dis.gamma_theta = g[0], g[1]
        wl.dis.N_base, wl.dis.g, wl.dis.B_axis = tuple(g[2:5]), tuple(g[5:8]), tuple(g[8:11])
        # the batch keeps its reflection list (extinction cull of the initial g)
        eng = AG.PatternEngine(wls[m])
        eng.set_globals(g)
        a = wl.atoms
        atoms = eng.atoms(*(torch.as_tensor(v) for v in (a.x, a.y, a.z, a.B, a.occ)))
        _, F2 = B.structure_factors(eng.cell, atoms, eng.hkl)
        ref = eng.plan.run(eng.hkl, F2)
        r = rel(be.image_of(m).cpu().numpy(), ref.cpu().numpy())
        say(f"  model {m} after update: rel-L2 vs single {r:.2e}")
        assert r <= 1e-5


def _folded_16x4(wl):
    """The same model in 16 x 4 tiles with the mirror fold (a centred beam and a width of a
    multiple of 16 are made up for it)."""
    import dataclasses
    w = -(-wl.geom.width // 16) * 16
    g = dataclasses.replace(wl.geom, width=w, center_x=w / 2.0, tile_w=16, mirror=1)
    return dataclasses.replace(wl, geom=g)


@pytest.mark.parametrize("variant", ["default", "folded_16x4"])
def test_graph_replay_matches_eager(variant):
    wls = small_batch()
    if variant == "folded_16x4":
        wls = [_folded_16x4(w) for w in wls]
    be = BatchEngine(wls)
    tgt_eng = BatchEngine(wls)
    glob = tgt_eng.globals()
    glob[:, 0] *= 1.1
    tgt_eng.set_globals(glob)
    target = tgt_eng.forward().clone()
    del tgt_eng
    step = GraphStep(be, target)
    step.eager()
    torch.cuda.synchronize()
    ref_img = be.image.clone()
    ref_g = {k: v.clone() for k, v in be.grads.items()}
    ref_glob = be.d_globals.clone()
    step.capture()
    for rep in range(3):
        # eager work of the program between replays
        be.image.fill_(-1.0)
        be.d_globals.fill_(0.0)
        torch.cuda.synchronize()
        step.replay()
        torch.cuda.synchronize()
        assert torch.equal(be.image, ref_img), rep
        for k in ref_g:
            d = (be.grads[k] - ref_g[k]).abs().max().item()
            assert d <= 1e-6 * ref_g[k].abs().max().item(), (rep, k, d)
        d = (be.d_globals - ref_glob).abs().max().item()
        assert d <= 1e-9 * ref_glob.abs().max().item(), (rep, d)
        say(f"  replay {rep}: image identical, gradients within rounding")


def test_batch_two_benchmark_models_match_single():
    wls = W.config4(n_models=3)[:2]
    say("two models of the 256-model batch:", [(w.atoms.n, w.geom.width) for w in wls])
    be = BatchEngine(wls)
    be.forward()
    torch.cuda.synchronize()
    for m, wl in enumerate(wls):
        ref = Pipeline(wl).pattern()
        r = rel(be.image_of(m).cpu().numpy(), ref.cpu().numpy())
        say(f"  model {m}: rel-L2 vs single {r:.2e}")
        assert r <= 1e-5
