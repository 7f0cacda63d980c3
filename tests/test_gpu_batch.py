"""Batched models (fdtbx_batch_forward / fdtbx_batch_backward, persistent launches):
each model's image and gradients equal its unbatched run and the oracle (two models of a
small batch over their whole detectors; five models of the 256-model benchmark batch, among
them the smallest and largest Lorentzian fraction eta and the largest g, on stratified
pixels), parameters update in place on the device, and a HIP-graph replay of the refinement
step reproduces the eager step on every replay."""
import math
import sys

import numpy as np
import pytest

import gradcheck as GC
import workloads as W
from oracle import oracle as O
from strata import stratified_pixels

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
    glob[2, 5] = 0.02          # g_a of model 2 (lowered: the supports shrink)
    glob[3, 3] *= 1.25         # N_base_b of model 3 (raised: the supports shrink)
    glob[4, 9] = 4.0           # B_b of model 4
    be.set_globals(glob)
    assert be.stale_models() == []
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


def check_group(name, got, ref):
    GC.check(name, got, ref, GC.RANDOM_FLOOR, say=say)  # random cotangents G


def check_globals(wl, gg, ref):
    refg = [ref["sigma_theta"], ref["gamma_theta"], *ref["N_base"], *ref["g"], *ref["B_axis"]]
    for i, n in enumerate(B.GLOBAL_NAMES):
        if n.startswith("g_") and wl.dis.g[i - 5] == 0.0:
            assert gg[i] == 0.0 and refg[i] == 0.0, (n, gg[i], refg[i])  # dA/dg = 0 at g = 0
            continue
        if n == "sigma_theta" and wl.dis.sigma_theta == 0.0:
            # the Lorentzian's one-sided sigma derivative is 0 (the Voigt is smooth in sigma^2);
            # compared on the scale of the gamma gradient, which has the same units
            assert refg[0] == 0.0 and abs(gg[0]) <= 1e-6 * abs(refg[1]), (gg[0], refg[1])
            continue
        check_group(n, [gg[i]], [refg[i]])


def _oracle_problem(wl):
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    hkl = np.ascontiguousarray(hkl[~O.extinct_mask(hkl, wl.dis, wl.quad.extinction)])
    return hkl, O.prepare(wl, hkl=hkl, F=O.structure_factors_c(hkl, wl.cell, wl.atoms), cull_extinct=False)


def test_batch_gradients_small_models_vs_oracle():
    """Two models of the small batch (a Lorentzian one on a monoclinic cell, off-centre, and a
    Voigt one beside a detector only 9 pixels wide): batched image and gradients of
    L = sum G P (G seeded over every pixel) against the oracle."""
    wls = small_batch()
    be = BatchEngine(wls)
    img = be.forward()
    G = torch.as_tensor(np.random.default_rng(5).normal(size=img.shape[0]), dtype=torch.float32).cuda()
    grads, glob = be.backward(G)
    torch.cuda.synchronize()
    for m in (1, 3):
        wl = wls[m]
        say(f"  small batch model {m}")
        hkl, P = _oracle_problem(wl)
        assert np.array_equal(be.hkl[be.hkl_off[m]:be.hkl_off[m + 1]].cpu().numpy(), hkl)
        Gm = G[be.pix_off[m]:be.pix_off[m + 1]].cpu().numpy().astype(np.float64).reshape(be.shapes[m])
        ref_img = O.pattern(wl, P)
        r = rel(be.image_of(m).cpu().numpy(), ref_img)
        say(f"    image rel-L2 vs oracle {r:.2e}")
        assert r <= 1e-4
        ref = O.gradients(wl, P, Gm)
        a0, a1 = be.atom_off[m], be.atom_off[m + 1]
        for k in ("x", "y", "z", "B", "occ"):
            check_group(k, grads[k][a0:a1].cpu().numpy(), ref["atoms"][k])
        check_globals(wl, glob[m].cpu().numpy(), ref)


def _benchmark_picks(wls):
    eta = np.array([w.dis.gamma_theta / (w.dis.sigma_theta + w.dis.gamma_theta) for w in wls])
    g = np.array([w.dis.g[0] for w in wls])
    na = np.array([w.atoms.n for w in wls])
    return {"smallest eta": int(eta.argmin()), "largest eta": int(eta.argmax()), "largest g": int(g.argmax()),
            "fewest atoms": int(na.argmin()), "first": 0}


def test_batch_gradients_benchmark_models_vs_oracle():
    """Five models of the 256-model benchmark batch, batched together in the benchmark's
    launch (16 x 4 tiles, both mirror folds): the smallest and the largest Lorentzian fraction
    (eta 0.0065 and 0.9988, the Voigt next to its Gaussian and Lorentzian limits), the largest g
    (0.060), the fewest atoms and the first model.  With dL/dP = G seeded on 128 stratified
    pixels of each model (zero elsewhere), the batched image there and every atom and global
    gradient against the oracle over each model's whole reflection list."""
    import dataclasses
    all_wls = W.config4(n_models=256)
    picks = _benchmark_picks(all_wls)
    order = sorted(set(picks.values()))
    wls = [dataclasses.replace(all_wls[m], geom=dataclasses.replace(all_wls[m].geom, tile_w=16, mirror=3))
           for m in order]
    say("benchmark-batch models vs oracle:", {k: v for k, v in picks.items()})
    be = BatchEngine(wls)
    img = be.forward()
    torch.cuda.synchronize()
    Gflat = np.zeros(img.shape[0])
    support = {}
    for i, wl in enumerate(wls):
        hkl, P = _oracle_problem(wl)
        assert np.array_equal(be.hkl[be.hkl_off[i]:be.hkl_off[i + 1]].cpu().numpy(), hkl)
        pix = stratified_pixels(wl, P, {"strong": 64, "meridian": 8, "equator": 8, "uniform": 48}, seed=40 + i)
        q = np.array([p for p, _ in pix], dtype=np.int64)
        Gq = np.random.default_rng(50 + i).normal(size=q.size)
        Gflat[be.pix_off[i] + q] = Gq
        support[i] = (hkl, P, q, Gq)
    G = torch.as_tensor(Gflat, dtype=torch.float32).cuda()
    grads, glob = be.backward(G)
    torch.cuda.synchronize()
    for i, wl in enumerate(wls):
        m = order[i]
        name = [k for k, v in picks.items() if v == m]
        hkl, P, q, Gq = support[i]
        say(f"  model {m} ({', '.join(name)}): {wl.atoms.n} atoms, {hkl.shape[0]} reflections, "
            f"{wl.geom.width}^2 px, eta {wl.dis.gamma_theta / (wl.dis.sigma_theta + wl.dis.gamma_theta):.4f}, "
            f"g {wl.dis.g[0]:.4f}")
        R, Z = O.pixel_rz(wl.geom)
        Rq, Zq = R.ravel()[q], Z.ravel()[q]
        ref_img = O.pattern_at(P, Rq, Zq)
        got_img = be.image_of(i).cpu().numpy().ravel()[q].astype(np.float64)
        big = ref_img > 1e-3 * ref_img.max()
        r = rel(got_img, ref_img)
        px = float(np.max(np.abs(got_img[big] - ref_img[big]) / ref_img[big]))
        say(f"    image on the support: rel-L2 {r:.2e}, per-pixel {px:.2e}")
        assert r <= 1e-4 and px <= 1e-3
        # the G of the folded images' mirror pixels is zero; the kernel folds G as it folds P
        ref = O.gradients(wl, P, Gq, Rq, Zq)
        a0, a1 = be.atom_off[i], be.atom_off[i + 1]
        for k in ("x", "y", "z", "B", "occ"):
            check_group(k, grads[k][a0:a1].cpu().numpy(), ref["atoms"][k])
        check_globals(wl, glob[i].cpu().numpy(), ref)


def test_batch_guards_its_culling_lists():
    """Raising g (or lowering N_base) widens the supports beyond the set-up culling lists:
    set_globals refuses such a move, or rebuilds the batch for it, after which the model matches
    the oracle at its new globals.  Moves that shrink the supports pass and leave the images of
    the other models bit for bit as they were."""
    import dataclasses
    wls = small_batch()
    be = BatchEngine(wls)
    img0 = be.forward().clone()
    glob = be.globals()
    up = glob.clone()
    up[0, 5] *= 1.1            # g_a of model 0 up by 10%
    with pytest.raises(Exception, match="culling lists"):
        be.set_globals(up)
    assert be.stale_models() == [0]
    down = glob.clone()
    down[0, 5] *= 0.9          # g down and N_base up: allowed
    down[1, 2] *= 1.1
    be.set_globals(down)
    assert be.stale_models() == []
    img1 = be.forward()
    torch.cuda.synchronize()
    for m in (2, 3, 4):       # untouched models: the same bits
        assert torch.equal(be.image_of(m), img0[be.pix_off[m]:be.pix_off[m + 1]].view(*be.shapes[m]))
    assert not torch.equal(img1, img0)
    be.set_globals(up, on_stale="rebuild")
    assert be.stale_models() == []
    be.forward()
    torch.cuda.synchronize()
    g = up[0].cpu().numpy()
    wl = dataclasses.replace(wls[0], dis=dataclasses.replace(wls[0].dis, g=tuple(float(v) for v in g[5:8])))
    hkl = be.hkl[be.hkl_off[0]:be.hkl_off[1]].cpu().numpy()
    ref = O.pattern(wl, O.prepare(wl, hkl=hkl, cull_extinct=False))
    got = be.image_of(0).cpu().numpy().astype(np.float64)
    r = rel(got, ref)
    big = ref > 1e-3 * ref.max()
    px = float(np.max(np.abs(got[big] - ref[big]) / ref[big]))
    say(f"  rebuilt model 0 at g_a x1.1: rel-L2 vs oracle {r:.2e}, per-pixel {px:.2e}")
    assert r <= 1e-4 and px <= 1e-3
