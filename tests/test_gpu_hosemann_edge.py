"""The one-period support of the Hosemann lineshape, decided in float32 on the GPU and in
binary64 by the oracle.

The Hosemann factor of Eq. Z is periodic in u and does not vanish at the edge of its support
(|u| = 1/2 per axis: (1 - A)/(1 + A) there).  A node whose u lies within about 1e-7 of the edge
can fall inside the support in binary64 and outside in float32, or the reverse, and then
carries its whole term into one image and not the other.  On a pixel whose value is mostly
such edge terms this one term can exceed the per-pixel tolerance, as it does at one pixel of
one workload of an extended launch sweep (seed 315 of the sweep's generator; relative L2 of
the image 7e-6).  This test takes that workload and checks that the deviation at every pixel
above 1e-3 of the maximum is within the tolerance once the oracle's edge terms (nodes within
1e-6 of an edge, decided either way) are allowed to be counted or not: the image is the
oracle's up to rounding and the float32 decisions at the support edge, and nothing else."""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2608_23245_amd import Pipeline  # noqa: E402
from test_gpu_launch_sweep import random_case  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def edge_terms(wl, P, Rp, Zp, eps=1e-6):
    """Sum of the pattern terms W_h r0^2 omega_k prod_i f(u_i) at ring point (Rp, Zp) whose
    nodes lie within eps of the support edge on some axis, split into those the oracle counts
    (inside) and those it does not, before the Lorentz factor; and the oracle's sum."""
    zhat = np.array([0.0, 0.0, 1.0])
    d1, d2, om = P.nodes.d1, P.nodes.d2, P.nodes.omega
    c = 1.0 / np.sqrt(1.0 + d1 * d1 + d2 * d2)
    total = inside_edge = outside_edge = 0.0
    for h in range(P.hkl.shape[0]):
        p = Rp * P.ep[h] + Zp * zhat
        s = P.r0[h] * c[:, None] * (P.S[h][None, :] + d1[:, None] * P.e1[h][None, :] + d2[:, None] * P.e2[h][None, :])
        u = (p[None, :] - s) @ P.avec.T
        inside = np.all(np.abs(u) <= 0.5, axis=1)
        term = P.W[h] * P.r0[h] ** 2 * om * np.prod(O.axis_profile(2, P.N[h][None, :], u), axis=1)
        near = np.min(np.abs(np.abs(u) - 0.5), axis=1) < eps
        total += term[inside].sum()
        inside_edge += term[inside & near].sum()
        outside_edge += term[~inside & near].sum()
    return total, inside_edge, outside_edge


def test_hosemann_deviation_is_the_support_edge():
    wl, _ = random_case(315)
    assert wl.dis.lineshape == 2
    g = wl.geom
    pipe = Pipeline(wl)
    img = pipe.pattern().cpu().numpy().astype(np.float64)
    P = O.prepare(wl, hkl=pipe.hkl.cpu().numpy())
    ref = O.pattern(wl, P)
    R, Z = O.pixel_rz(g)
    delta = wl.quad.delta
    big = ref > 1e-3 * ref.max()
    rel = np.where(big, np.abs(img - ref) / np.where(big, ref, 1.0), 0.0)
    r = float(np.linalg.norm(img - ref) / np.linalg.norm(ref))
    say(f"Hosemann edge case: {g.width}x{g.height}, rel-L2 {r:.2e}, worst per-pixel {rel.max():.2e}")
    assert r <= 1e-4
    worst = 0.0
    for j, i in zip(*np.nonzero(rel > 5e-4)):
        lor = delta / (R[j, i] + delta)  # the Lorentz factor of Eq. lorentz
        total, e_in, e_out = edge_terms(wl, P, R[j, i], Z[j, i])
        assert abs(lor * total - ref[j, i]) <= 1e-9 * ref[j, i]  # the decomposition is the oracle's
        # the GPU may count each edge term or not: its value lies in [ref - e_in, ref + e_out]
        lo, hi = ref[j, i] - lor * e_in, ref[j, i] + lor * e_out
        d = max(lo - img[j, i], img[j, i] - hi, 0.0) / ref[j, i]
        say(f"  pixel ({j}, {i}): {rel[j, i]:.2e} from the oracle; edge terms {lor * e_in / ref[j, i]:.2e} counted, "
            f"{lor * e_out / ref[j, i]:.2e} not; outside that range by {d:.1e}")
        worst = max(worst, d)
    assert worst <= 1e-5
