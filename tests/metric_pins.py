"""Pins of the oracle's comparison helpers (rel-L2 and the element-wise error).

Every parity bound in the suite is a value of these helpers, so they are pinned
to facts that do not depend on their code: small integer vectors whose norms
are exact (3-4-5 and 1-2-2-3 triangles), a relative scaling y = (1 + d) y_ref
whose rel-L2 is |d| by definition, an error orthogonal to the reference, the
asymmetry that fixes which argument is the denominator, rupture independence
along the leading axis, and the stated rule for a reference that is zero.

``failures(mod)`` returns the list of pins that the helpers of ``mod`` break;
the oracle must break none, and planted mistakes must break at least one.
"""
import numpy as np


def failures(mod):
    bad = []

    def check(name, got, want, tol=1e-15):
        if not np.allclose(np.asarray(got, dtype=float), np.asarray(want, dtype=float), rtol=tol, atol=tol):
            bad.append(f"{name}: got {got!r}, want {want!r}")

    ref = np.array([3.0, 4.0, 0.0])                      # ||ref|| = 5
    # a relative scaling by (1 + d) has rel-L2 |d|, not d^2 nor d / (1 + d)
    for d in (0.1, -0.25, 1e-3):
        check(f"scaling d={d}", mod.rel_l2((1.0 + d) * ref, ref), abs(d), tol=1e-14)
    # an error orthogonal to the reference: ||e|| / ||ref|| with e = (0, 0, 1)
    check("orthogonal error", mod.rel_l2(ref + np.array([0.0, 0.0, 1.0]), ref), 0.2)
    # e = (-4, 3, 0) * 2 is orthogonal too: ||e|| = 10
    check("orthogonal error 2", mod.rel_l2(ref + 2.0 * np.array([-4.0, 3.0, 0.0]), ref), 2.0)
    # the denominator is the reference: y = 2 ref gives 1, y = ref / 2 gives 1/2
    check("denominator is the reference", mod.rel_l2(2.0 * ref, ref), 1.0)
    check("denominator is the reference 2", mod.rel_l2(0.5 * ref, ref), 0.5)
    # multi-dimensional inputs are one vector: (1, 2, 2) and (0, 0, 3) have norms 3 and 3
    r2 = np.array([[1.0, 2.0, 2.0], [0.0, 0.0, 0.0]])
    e2 = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 3.0]])
    check("all entries count", mod.rel_l2(r2 + e2, r2), 1.0)
    # a zero reference: the stated rule is the absolute norm of the result
    check("zero reference", mod.rel_l2(np.array([3.0, -4.0]), np.zeros(2)), 5.0)
    check("zero reference, zero result", mod.rel_l2(np.zeros(4), np.zeros(4)), 0.0)
    # identical arrays
    check("identity", mod.rel_l2(ref, ref), 0.0)
    # per rupture: each leading index against its own reference, however different the norms
    yr = np.stack([1e6 * ref, ref, np.array([1.0, 2.0, 2.0])])
    yy = np.stack([1e6 * ref * 1.5, ref, np.array([1.0, 2.0, 2.0]) + np.array([0.0, 0.0, 3.0])])
    got = mod.rel_l2_per_rupture(yy, yr)
    if np.shape(got) != (3,):
        bad.append(f"per rupture shape {np.shape(got)}")
    else:
        check("per rupture", got, [0.5, 0.0, 1.0])
    # element-wise: one spike of 0.5 against a largest reference entry of 4
    spike = ref.copy()
    spike[2] += 0.5
    check("max-abs spike", mod.max_abs_rel(spike, ref), 0.125)
    # the element-wise value is not diluted by the norm: a 0.5 spike among 10^4 unit entries
    big = np.ones(10000)
    bs = big.copy()
    bs[1234] += 0.5
    check("max-abs not diluted", mod.max_abs_rel(bs, big), 0.5)
    check("rel-L2 is diluted", mod.rel_l2(bs, big), 0.005)
    check("max-abs zero reference", mod.max_abs_rel(np.array([0.0, -2.0]), np.zeros(2)), 2.0)
    got = mod.max_abs_rel_per_rupture(np.stack([spike, 2.0 * ref]), np.stack([ref, ref]))
    if np.shape(got) != (2,):
        bad.append(f"max-abs per rupture shape {np.shape(got)}")
    else:
        check("max-abs per rupture", got, [0.125, 1.0])
    return bad
