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


def _order_rates(scheme, omega, nsteps_list, ref_steps, t_end=0.2, degree=3, cells=6):
    inst = W.Instance(2, (cells, cells), degree, 1.0, 1, "advection", {"a": [0.5, 0.25]},
                      W.gaussian_bump(1.0, (0.4, 0.45), 20.0))
    prob = _problem(inst)
    f0, fb = _initial(prob, inst.w0)

    def f_at(n):
        dt = t_end / n
        # omega is given for dt; keep tau fixed across the refinements
        return ost.run(prob, f0, fb, dt, 0.5, ost.omega_for(dt, TAU_DT, omega), scheme, n)

    ref = f_at(ref_steps)
    errs = [np.linalg.norm(f_at(n) - ref) for n in nsteps_list]
    return errs, [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


TAU_DT = 0.05   # omega below is the collision factor over this step: tau = 0.05 (2 - w)/(2 w)


def test_omega_for_matches_crank_nicolson_collision():
    # eq. collision_cn: omega(h) = 2h/(2 tau + h); tau from omega over dt
    tau = 0.013
    dt = 0.05
    omega = 2 * dt / (2 * tau + dt)
    for h in (dt, dt / 2, -dt / 3, 0.37 * dt):
        assert abs(ost.omega_for(h, dt, omega) - 2 * h / (2 * tau + h)) < 1e-14
    assert ost.omega_for(0.123, dt, 2.0) == 2.0


@pytest.mark.slow
def test_kin_composition_is_second_order_with_relaxation_time():
    errs, rates = _order_rates(ost.KIN, 1.6, [4, 8, 16], 64)
    assert all(1.7 < r < 2.5 for r in rates), (errs, rates)


@pytest.mark.slow
def test_kin_composition_is_second_order_at_tau_zero():
    errs, rates = _order_rates(ost.KIN, 2.0, [4, 8, 16], 64)
    assert all(1.7 < r < 2.5 for r in rates), (errs, rates)


@pytest.mark.slow
def test_triple_jump_of_kin_is_fourth_order():
    # the negative middle stage makes the composition only conditionally
    # stable on the strongly damped upwind modes: test in its asymptotic range
    errs, rates = _order_rates(ost.KIN4, 1.6, [16, 32], 128, t_end=0.1, degree=1, cells=4)
    assert all(3.5 < r < 5.0 for r in rates), (errs, rates)


def test_kin_step_is_time_symmetric_with_relaxation_time():
    # M_2^kin is a palindrome of time-symmetric stages when tau > 0
    inst = W.make("adv2d_16", scale=4).instances[0]
    prob = _problem(inst)
    f0, fb = _initial(prob, inst.w0)
    f0 = f0 * (1 + 0.1 * np.random.default_rng(1).standard_normal(f0.shape))
    dt, tau = 0.03, 0.02
    omega = 2 * dt / (2 * tau + dt)
    g = ost.run(prob, f0, fb, dt, 0.5, omega, ost.KIN, 1)
    back = ost.run(prob, g, fb, -dt, 0.5, 2 * (-dt) / (2 * tau - dt), ost.KIN, 1)
    assert np.max(np.abs(back - f0)) < 1e-12 * np.max(np.abs(f0))
