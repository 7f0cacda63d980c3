"""The oracle's gradient of the refinement loss (refinement.py: the medium model against its
perturbed target on a 256-pixel support) against binary64 central finite differences with
absolute step 1e-5 (reading R19), for the 64 parameters of the check: the 8 globals
sigma_theta, gamma_theta, N_base (3), g (3) (the node extent T held fixed) and 56 seeded
(atom, field) pairs (fractional x, y, z, B, occupancy).  The loss keeps its weights w and the
target T fixed, so dL/dtheta = sum_q G_q dI_q/dtheta with G = 2 w (I - T), which is what
oracle.gradients returns for that G.

The atom differences use the linearity of the image in the weights W = |F|^2 I_para: the
per-(pixel, reflection) profiles are tabulated once (oracle.profile_table with the exact
skip), and a moved atom changes F by the difference of its own terms (Eq. structure_factor
is a sum over atoms).  The globals are differenced through the whole oracle image."""
import dataclasses

import numpy as np
import pytest

import refinement as RF
from oracle import oracle as O

pytestmark = pytest.mark.slow

H = 1e-5


def loss(rf, I):
    return float(np.sum(rf.w * (I - rf.T) ** 2))


def _with_global(wl, name, v):
    d = wl.dis
    if name in ("sigma_theta", "gamma_theta"):
        return dataclasses.replace(wl, dis=dataclasses.replace(d, **{name: v}))
    axis = "abc".index(name[-1])
    if name.startswith("N_base"):
        N = list(d.N_base)
        N[axis] = v
        return dataclasses.replace(wl, dis=dataclasses.replace(d, N_base=tuple(N)))
    g = list(d.g)
    g[axis] = v
    return dataclasses.replace(wl, dis=dataclasses.replace(d, g=tuple(g)))


def _global_value(wl, name):
    d = wl.dis
    if name in ("sigma_theta", "gamma_theta"):
        return getattr(d, name)
    axis = "abc".index(name[-1])
    return (d.N_base if name.startswith("N_base") else d.g)[axis]


def _check(name, fd, g, floor):
    err = abs(fd - g) / max(abs(g), floor)
    print(f"  {name}: oracle {g:+.6e}  fd {fd:+.6e}  rel {err:.1e}", flush=True)
    assert err <= 2e-4, (name, fd, g)


@pytest.fixture(scope="module")
def problem():
    rf = RF.build()
    ref = O.gradients(rf.wl, rf.P, rf.G, rf.R, rf.Z)
    return rf, ref


def test_refinement_globals_match_finite_differences(problem):
    rf, ref = problem
    names = ("sigma_theta", "gamma_theta", "N_base_a", "N_base_b", "N_base_c", "g_a", "g_b", "g_c")
    refg = dict(zip(names, [ref["sigma_theta"], ref["gamma_theta"], *ref["N_base"], *ref["g"]]))
    floor = 1e-3 * max(abs(v) for v in refg.values())
    for name in names:
        v0 = _global_value(rf.wl, name)
        Ls = []
        for v in (v0 + H, v0 - H):
            wl = _with_global(rf.wl, name, v)
            P = O.prepare(wl, hkl=rf.hkl, F=rf.F, cull_extinct=False)
            Ls.append(loss(rf, O.pattern_at(P, rf.R, rf.Z)))
        _check(name, (Ls[0] - Ls[1]) / (2 * H), refg[name], floor)


def test_refinement_atoms_match_finite_differences(problem):
    rf, ref = problem
    P = O.prepare(rf.wl, hkl=rf.hkl, F=rf.F, cull_extinct=False)
    table = O.profile_table(P, rf.R, rf.Z, use_skip=True)               # [pixel][reflection]
    lor = rf.wl.quad.delta / (rf.R + rf.wl.quad.delta)
    factor = P.Ip * P.Dw                                                   # W = |F|^2 factor
    a = rf.wl.atoms

    def image(F):
        return lor * (table @ ((F.real * F.real + F.imag * F.imag) * factor))

    # the tabulated image is the oracle image (same terms, another grouping of the sums)
    np.testing.assert_allclose(image(rf.F), rf.I, rtol=1e-12, atol=0)

    def one_atom(j, field, v):
        vals = {k: np.array([getattr(a, k)[j]], dtype=np.float64) for k in ("x", "y", "z", "B", "occ")}
        vals[field] = np.array([v])
        return dataclasses.replace(a, x=vals["x"], y=vals["y"], z=vals["z"], B=vals["B"], occ=vals["occ"],
                                   type=a.type[j:j + 1])

    for j, field in RF.fd_parameters(a.n):
        v0 = float(getattr(a, field)[j])
        t0 = O.structure_factors(rf.hkl, rf.wl.cell, one_atom(j, field, v0))
        Ls = []
        for v in (v0 + H, v0 - H):
            F = rf.F - t0 + O.structure_factors(rf.hkl, rf.wl.cell, one_atom(j, field, v))
            Ls.append(loss(rf, image(F)))
        g = ref["atoms"][field][j]
        _check(f"atom {j} {field}", (Ls[0] - Ls[1]) / (2 * H), g, 1e-3 * np.abs(ref["atoms"][field]).max())
