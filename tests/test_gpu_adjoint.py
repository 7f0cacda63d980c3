"""Parity of the hand-written adjoint (C ABI fdtbx_pattern_backward and the
torch.autograd wrapper) with the FP64 oracle's gradient, which the CPU tests pin
to central finite differences.  Gradients must agree to relative error 1e-3, with
a floor of 1e-3 of the largest gradient of the same group (atom field or global).
At full size, exact identities of the gradient are checked instead."""
import dataclasses
import math
import sys

import numpy as np
import pytest

import gradcheck as GC
import refinement as RF
import workloads as W
from oracle import oracle as O

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


def check_group(name, got, ref, floor=GC.RANDOM_FLOOR):
    GC.check(name, got, ref, floor, say=say)


def gpu_gradients(wl, G):
    eng = AG.PatternEngine(wl)
    atoms = eng.atoms(*(torch.as_tensor(v) for v in (wl.atoms.x, wl.atoms.y, wl.atoms.z, wl.atoms.B, wl.atoms.occ)))
    F, F2 = B.structure_factors(eng.cell, atoms, eng.hkl)
    img = eng.plan.run(eng.hkl, F2)
    Gt = torch.as_tensor(G, dtype=torch.float32).cuda().contiguous()
    out, glob, dF2 = B.pattern_backward(eng.plan, eng.hkl, F, Gt, atoms)
    return eng, img, {k: v.cpu().numpy() for k, v in out.items()}, glob.cpu().numpy(), dF2.cpu().numpy()


CASES = {
    "voigt_g": dict(seed=41, width=20, height=18, sigma_theta=3 * DEG, gamma_theta=2 * DEG, g=(0.03, 0.02, 0.01)),
    "gauss": dict(seed=42, width=17, height=21, sigma_theta=4 * DEG, gamma_theta=0.0, g=(0.02, 0.0, 0.0)),
    "lorentz": dict(seed=43, width=22, height=16, sigma_theta=0.0, gamma_theta=3 * DEG, g=(0.0, 0.0, 0.03)),
    "offcentre": dict(seed=44, width=19, height=19, center=(4.2, 15.3), sigma_theta=2 * DEG, gamma_theta=2 * DEG,
                      g=(0.01, 0.04, 0.0)),
    "no_intensity_model": dict(seed=45, width=16, height=16, sigma_theta=3 * DEG, gamma_theta=1 * DEG,
                               g=(0.03, 0.03, 0.0)),
    "tilted": dict(seed=46, width=18, height=20, sigma_theta=2 * DEG, gamma_theta=1 * DEG, g=(0.02, 0.02, 0.0),
                   tilt=30 * DEG),
    "gaussian_damped": dict(seed=47, width=18, height=16, sigma_theta=2 * DEG, gamma_theta=1 * DEG, g=(0.02, 0.03, 0.01),
                            lineshape=1, B_axis=(4.0, 9.0, 2.5)),
    "hosemann_damped": dict(seed=48, width=17, height=19, sigma_theta=3 * DEG, gamma_theta=0.0, g=(0.03, 0.02, 0.01),
                            lineshape=2, B_axis=(6.0, 1.0, 3.0)),
    "hosemann_small_n": dict(seed=49, width=16, height=16, sigma_theta=2 * DEG, gamma_theta=2 * DEG, g=(0.1, 0.02, 0.0),
                             lineshape=2, size_A=(12.0, 60.0, 50.0)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_adjoint_small_vs_oracle(name):
    wl = W.small(**CASES[name], n_atoms=30)
    if name == "no_intensity_model":
        wl.dis.intensity_model = 0
    say(f"adjoint {name}")
    G = np.random.default_rng(7).normal(size=(wl.geom.height, wl.geom.width))
    eng, img, ga, gg, _ = gpu_gradients(wl, G)
    hkl = eng.hkl.cpu().numpy()
    P = O.prepare(wl, hkl=hkl, cull_extinct=False)
    ref = O.gradients(wl, P, G)
    for k in ("x", "y", "z", "B", "occ"):
        check_group(k, ga[k], ref["atoms"][k])
    names = B.GLOBAL_NAMES
    refg = [ref["sigma_theta"], ref["gamma_theta"], *ref["N_base"], *ref["g"], *ref["B_axis"]]
    for i, n in enumerate(names):
        if ("g_" in n and wl.dis.g[i - 5] == 0.0):
            continue  # dA/dg vanishes at g = 0 on both sides; compared below as zero
        if n == "sigma_theta" and wl.dis.sigma_theta == 0.0:
            # one-sided derivative of the Voigt at sigma = 0+: zero (the oracle's forward
            # difference gives rounding noise); scale by the gamma gradient, same units
            assert abs(gg[0]) <= 1e-6 * abs(refg[1]) and abs(refg[0]) <= 1e-6 * abs(refg[1])
            continue
        check_group(n, [gg[i]], [refg[i]])
    for i in range(3):
        if wl.dis.g[i] == 0.0:
            assert abs(gg[5 + i]) == 0.0 and abs(refg[5 + i]) == 0.0


def _crop(wl, x0, y0, w, h):
    g = wl.geom
    geom = dataclasses.replace(g, width=w, height=h, center_x=g.center_x - x0, center_y=g.center_y - y0)
    return dataclasses.replace(wl, geom=geom)


def test_adjoint_medium_model_on_a_detector_crop():
    """Medium model (all its reflections), 16x16 pixels of its detector with signal."""
    wl = _crop(W.config1(), 700, 560, 16, 16)
    say("adjoint medium crop")
    G = np.random.default_rng(8).normal(size=(16, 16))
    eng, img, ga, gg, dF2 = gpu_gradients(wl, G)
    assert img.max().item() > 0
    hkl = eng.hkl.cpu().numpy()
    R, Z = O.pixel_rz(wl.geom)
    sub = O.reachable(wl, hkl, R, Z)
    say(f"  oracle over the {sub.size} of {hkl.shape[0]} reflections its exact skip leaves at the crop's pixels")
    F = O.structure_factors_c(hkl[sub], wl.cell, wl.atoms)
    P = O.prepare(wl, hkl=np.ascontiguousarray(hkl[sub]), F=F, cull_extinct=False)
    ref = O.gradients(wl, P, G)
    for k in ("x", "y", "z", "B", "occ"):
        check_group(k, ga[k], ref["atoms"][k])
    refg = [ref["sigma_theta"], ref["gamma_theta"], *ref["N_base"], *ref["g"], *ref["B_axis"]]
    for i, n in enumerate(B.GLOBAL_NAMES):
        if n == "g_c":
            continue  # g_c = 0 in this model
        check_group(n, [gg[i]], [refg[i]])
    # reflections that cannot reach the crop carry no gradient (up to float32 support-boundary
    # flips, where the Laue profile has a double zero)
    mask = np.ones(hkl.shape[0], bool)
    mask[sub] = False
    assert np.all(np.abs(dF2[mask]) <= 1e-6 * np.abs(dF2).max())


def test_refinement_gradient_full_size_vs_oracle():
    """The refinement workload at full size in the benchmark's launch (the medium model's
    1024 x 1024 detector, 16 x 4 tiles, both mirror folds, the library's waves per tile) with
    dL/dI = G = 2 w (I - T) on the 256-pixel support of refinement.py and 0 elsewhere: the
    model's image on the support, all 11 global gradients and every atom gradient against
    oracle.gradients over the whole reflection list on the same pixels, to 1e-3 (the 56
    seeded (atom, field) pairs of the finite-difference check reported one by one)."""
    rf = RF.build()
    say(f"refinement gradient, full size: {rf.q.size} support pixels, {rf.hkl.shape[0]} reflections")
    wl = dataclasses.replace(rf.wl, geom=dataclasses.replace(rf.wl.geom, tile_w=16, mirror=3))
    G = np.zeros((wl.geom.height, wl.geom.width))
    G.ravel()[rf.q] = rf.G
    eng, img, ga, gg, _ = gpu_gradients(wl, G)
    assert np.array_equal(eng.hkl.cpu().numpy(), rf.hkl)
    got_I = img.reshape(-1)[torch.as_tensor(rf.q, device="cuda")].cpu().numpy().astype(np.float64)
    big = rf.I > 1e-3 * rf.I.max()
    say(f"  image on the support: rel-L2 {np.linalg.norm(got_I - rf.I) / np.linalg.norm(rf.I):.2e}, "
        f"max per-pixel rel {np.max(np.abs(got_I[big] - rf.I[big]) / rf.I[big]):.2e}")
    assert np.linalg.norm(got_I - rf.I) <= 1e-4 * np.linalg.norm(rf.I)
    ref = O.gradients(rf.wl, rf.P, rf.G, rf.R, rf.Z)
    for k in RF.FIELDS:
        check_group(k, ga[k], ref["atoms"][k], floor=GC.LOSS_FLOOR)
    for a, k in RF.fd_parameters(rf.wl.atoms.n):
        r = ref["atoms"][k][a]
        floor = GC.LOSS_FLOOR * np.abs(ref["atoms"][k]).max()
        assert abs(ga[k][a] - r) <= 1e-3 * max(abs(r), floor), (a, k, ga[k][a], r)
    refg = [ref["sigma_theta"], ref["gamma_theta"], *ref["N_base"], *ref["g"], *ref["B_axis"]]
    for i, n in enumerate(B.GLOBAL_NAMES):
        if n == "g_c":
            assert gg[i] == 0.0 and refg[i] == 0.0  # g_c = 0: dA/dg vanishes on both sides
            continue
        check_group(n, [gg[i]], [refg[i]], floor=GC.LOSS_FLOOR)


def test_adjoint_identities_at_full_size():
    """Medium model at full size with the weighted-residual loss against a perturbed target:
    translation invariance sum_j dL/dx_j = 0 and homogeneity sum_j occ_j dL/docc_j = 2 sum G P."""
    gw = W.config3()
    say("adjoint identities, full medium size")
    eng_t = AG.PatternEngine(gw.target)
    ta = gw.target.atoms
    atoms_t = eng_t.atoms(*(torch.as_tensor(v) for v in (ta.x, ta.y, ta.z, ta.B, ta.occ)))
    _, F2t = B.structure_factors(eng_t.cell, atoms_t, eng_t.hkl)
    target = eng_t.plan.run(eng_t.hkl, F2t).clone()
    del eng_t
    wl = gw.model
    img = None
    eng = AG.PatternEngine(wl)
    a = wl.atoms
    atoms = eng.atoms(*(torch.as_tensor(v) for v in (a.x, a.y, a.z, a.B, a.occ)))
    F, F2 = B.structure_factors(eng.cell, atoms, eng.hkl)
    img = eng.plan.run(eng.hkl, F2)
    w = 1.0 / (target + 1e-3 * target.max())
    G = (2.0 * w * (img - target)).contiguous()
    out, glob, _ = B.pattern_backward(eng.plan, eng.hkl, F, G, atoms)
    torch.cuda.synchronize()
    for k in ("x", "y", "z"):
        v = out[k].double()
        say(f"  sum d{k} = {v.sum().item():.3e} vs sum |d{k}| = {v.abs().sum().item():.3e}")
        assert abs(v.sum().item()) <= 2e-4 * v.abs().sum().item()
    lhs = float((out["occ"].double() * atoms["occ"].double()).sum().item())
    rhs = float(2.0 * (G.double() * img.double()).sum().item())
    say(f"  homogeneity: {lhs:.6e} vs {rhs:.6e}")
    assert abs(lhs - rhs) <= 2e-4 * abs(rhs)
    assert np.all(np.isfinite(glob.cpu().numpy()))


def test_autograd_module_chain_rule():
    """FibreModel's gradients (Cartesian coordinates, sigma/eta, sizes in A) equal the oracle's
    fractional and global gradients pushed through the same parameter maps."""
    wl = W.small(46, n_atoms=20, width=18, height=16, sigma_theta=2 * DEG, gamma_theta=1.5 * DEG, g=(0.02, 0.02, 0.0),
                 cell=W.Cell(9.0, 11.0, 13.0, 90 * DEG, 97 * DEG, 90 * DEG))
    say("autograd module")
    model = AG.FibreModel(wl)
    G = torch.as_tensor(np.random.default_rng(9).normal(size=(16, 18)), dtype=torch.float32).cuda()
    img = model()
    loss = (img * G).sum()
    loss.backward()
    # oracle at the float32-rounded model inputs the engine used
    frac = (model.xyz.detach() @ model.basis_inv).numpy()
    w2 = dataclasses.replace(wl, atoms=W.Atoms(frac[:, 0].astype(np.float32), frac[:, 1].astype(np.float32),
                                               frac[:, 2].astype(np.float32), wl.atoms.B, wl.atoms.occ, wl.atoms.type,
                                               wl.atoms.ff))
    hkl = model.engine.hkl.cpu().numpy()
    P = O.prepare(w2, hkl=hkl, cull_extinct=False)
    ref = O.gradients(w2, P, G.cpu().numpy().astype(np.float64))
    dfrac = np.stack([ref["atoms"]["x"], ref["atoms"]["y"], ref["atoms"]["z"]], 1)
    dcart = dfrac @ model.basis_inv.numpy().T
    check_group("xyz", model.xyz.grad.numpy(), dcart)
    check_group("B", model.B.grad.numpy(), ref["atoms"]["B"])
    check_group("occ", model.occ.grad.numpy(), ref["atoms"]["occ"])
    s, e = model.sigma.item(), model.eta.item()
    check_group("sigma", [model.sigma.grad.item()], [(1 - e) * ref["sigma_theta"] + e * ref["gamma_theta"]])
    check_group("eta", [model.eta.grad.item()], [-s * ref["sigma_theta"] + s * ref["gamma_theta"]])
    edges = np.array([wl.cell.a, wl.cell.b, wl.cell.c])
    check_group("size", model.size.grad.numpy(), ref["N_base"] / edges)
    check_group("g_ab", model.g.grad.numpy()[:2], ref["g"][:2])
    check_group("B_axis", model.B_axis.grad.numpy(), ref["B_axis"])


def test_autograd_refuses_a_backward_after_a_later_forward():
    """Two forwards on one engine: the first graph's backward would read the second forward's
    workspace and globals, so it raises; the second graph's backward runs."""
    wl = W.small(47, n_atoms=12, width=14, height=12, sigma_theta=2 * DEG)
    say("autograd: backward after a later forward")
    model = AG.FibreModel(wl)
    first = model().sum()
    with torch.no_grad():
        model.sigma.mul_(1.05)
    second = model().sum()
    with pytest.raises(RuntimeError, match="another forward"):
        first.backward()
    second.backward()
    assert model.sigma.grad is not None and torch.isfinite(model.sigma.grad).all()
