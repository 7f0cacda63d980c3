"""The gradient tolerance of the GPU tests: the method's bound of 1e-3 relative error on the
gradients (reading R19), applied per gradient group (an atom field, or a global).

A group passes when its relative L2 error is at most 1e-3 and every element is within 1e-3
of max(|reference|, floor * the group's largest |reference|).  The floor reflects what float32
evaluation can give an element that is small against its group: the per-reflection adjoint
sums carry a relative error of about 1e-6 (float32 profile values; measured against the
oracle), and an atom's gradient is a sum over reflections whose terms cancel, so an element
of 1e-3 of the group's largest holds only a few digits.  With the cotangent of a weighted-
residual loss (the refinement workload) the floor is 1e-3; with a random cotangent G, whose
signs make the sums over pixels and reflections cancel far more, it is 1e-2.
"""
import numpy as np

LOSS_FLOOR = 1e-3
RANDOM_FLOOR = 1e-2


def errors(got, ref, floor):
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    big = np.abs(ref).max()
    rel_l2 = float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))
    elem = float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), max(floor * big, 1e-300))))
    return rel_l2, elem


def check(name, got, ref, floor, tol=1e-3, say=print):
    rel_l2, elem = errors(got, ref, floor)
    say(f"  {name}: rel-L2 {rel_l2:.2e}, max element error {elem:.2e} (floor {floor:g} of the largest "
        f"{np.abs(np.asarray(ref, dtype=np.float64)).max():.3e})")
    assert rel_l2 <= tol and elem <= tol, (name, rel_l2, elem)
