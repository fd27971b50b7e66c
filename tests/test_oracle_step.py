"""Pins of the oracle's step compositions (Sec. 3.2, Sec. 5.1)."""
import numpy as np
import pytest

import workloads as W
from oracle import step as ost


def _problem(inst):
    return ost.Problem(inst.n, inst.lo, inst.hi, inst.degree, inst.vel, inst.m, inst.feq_kind, inst.feq_param)


def _initial(prob, w0):
    x = prob.mesh.node_coords().reshape(-1, prob.mesh.dim)
    w = w0(x).reshape(prob.m, prob.mesh.nc, prob.mesh.nd)
    return prob.feq(w), prob.inflow_from_w(w0)


@pytest.mark.parametrize("scheme", [ost.LIE, ost.STRANG, ost.STRANG_COLLAPSED])
def test_constant_scalar_state_is_preserved(scheme):
    inst = W.Instance(2, (4, 5), 2, 1.0, 1, "advection", {"a": [0.4, -0.2]}, W.uniform_state([0.7]))
    prob = _problem(inst)
    f0, fb = _initial(prob, inst.w0)
    f = ost.run(prob, f0, fb, 0.05, 0.5, 2.0, scheme, 4)
    assert np.max(np.abs(f - f0)) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_constant_euler_state_is_preserved(dim):
    state = [1.1, 0.2, -0.1, 2.7] if dim == 2 else [0.9, 0.1, 0.0, -0.2, 2.5]
    inst = W.Instance(dim, (3,) * dim, 2, 3.0, dim + 2, "euler", {"gamma": 1.4}, W.uniform_state(state))
    prob = _problem(inst)
    f0, fb = _initial(prob, inst.w0)
    f = ost.run(prob, f0, fb, 0.02, 0.5, 2.0, ost.STRANG_COLLAPSED, 3)
    assert np.max(np.abs(f - f0)) < 1e-12 * np.max(np.abs(f0))


def test_collapsed_strang_equals_strang_composition():
    # the collapsed form fuses T(dt/2) T(dt/2) into T(dt); for CN these differ
    # only at O(dt^3) per fused pair, but with a single step they coincide.
    inst = W.make("adv2d_16", scale=4).instances[0]
    prob = _problem(inst)
    f0, fb = _initial(prob, inst.w0)
    a = ost.run(prob, f0, fb, 0.05, 0.5, 2.0, ost.STRANG, 1)
    b = ost.run(prob, f0, fb, 0.05, 0.5, 2.0, ost.STRANG_COLLAPSED, 1)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)


@pytest.mark.slow
def test_collapsed_strang_is_second_order_in_time():
    inst = W.Instance(2, (6, 6), 3, 1.0, 1, "advection", {"a": [0.5, 0.25]},
                      W.gaussian_bump(1.0, (0.4, 0.45), 20.0))
    prob = _problem(inst)
    f0, fb = _initial(prob, inst.w0)
    t_end = 0.2

    def w_at(nsteps):
        f = ost.run(prob, f0, fb, t_end / nsteps, 0.5, 2.0, ost.STRANG_COLLAPSED, nsteps)
        return np.sum(f, axis=0)

    ref = w_at(64)
    errs = [np.linalg.norm(w_at(n) - ref) for n in (4, 8, 16)]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.7 < r < 2.4 for r in rates), (errs, rates)
