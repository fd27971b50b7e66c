"""Pins of the oracle's moments, equilibria and collision (Sec. 2, eq. collision_cn)."""
import numpy as np
import pytest

from oracle import relax as rx
from oracle import step as ost

D2Q4 = np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [0.0, -1.0]])
D3Q6 = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [-1.0, 0.0, 0.0],
                 [0.0, -1.0, 0.0], [0.0, 0.0, -1.0], [0.0, 0.0, 1.0]])


def _euler_state(dim, npts, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.8, 1.2, npts)
    u = rng.uniform(-0.3, 0.3, (dim, npts))
    p = rng.uniform(0.8, 1.2, npts)
    energy = p / 0.4 + 0.5 * rho * np.sum(u * u, axis=0)
    return np.vstack([rho[None], rho * u, energy[None]])


@pytest.mark.parametrize("vel,lam", [(D2Q4, 3.0), (D3Q6, 3.0), (D2Q4, 1.0)])
def test_euler_equilibrium_moments(vel, lam):
    dim = vel.shape[1]
    w = _euler_state(dim, 50, 1)
    q = rx.euler_flux(w, 1.4)
    feq = rx.equilibrium(w, vel * lam, q, lam)
    np.testing.assert_allclose(np.sum(feq, axis=0), w, rtol=1e-14, atol=1e-14)
    for k in range(dim):
        np.testing.assert_allclose(np.einsum("i,i...->...", vel[:, k] * lam, feq), q[k], rtol=1e-13, atol=1e-13)


def test_euler_flux_at_rest_is_pressure_only():
    # rho = 2, u = 0, E = p/(gamma-1) with p = 3: q^k = (0, p e_k, 0)
    w = np.array([[2.0], [0.0], [0.0], [0.0], [3.0 / 0.4]])
    q = rx.euler_flux(w, 1.4)
    for k in range(3):
        want = np.zeros(5)
        want[1 + k] = 3.0
        np.testing.assert_allclose(q[k][:, 0], want, atol=1e-14)


def test_euler_flux_of_moving_state():
    # 1D-like check in 2D: rho=1, u=(2,0), p=1 -> q^x = (2, 4+1, 0, (E+p) 2)
    rho, u, p = 1.0, 2.0, 1.0
    energy = p / 0.4 + 0.5 * rho * u * u
    q = rx.euler_flux(np.array([[rho], [rho * u], [0.0], [energy]]), 1.4)
    np.testing.assert_allclose(q[0][:, 0], [2.0, 5.0, 0.0, (energy + p) * 2.0], atol=1e-14)
    np.testing.assert_allclose(q[1][:, 0], [0.0, 0.0, 1.0, 0.0], atol=1e-14)


def test_scalar_advection_equilibrium_reduces_to_printed_form():
    # lambda = 1, D2Q4: f_i^eq = w/4 + (v_i . a) w / 2
    a = np.array([0.5, 0.25])
    w = np.random.default_rng(2).uniform(0.5, 1.5, (1, 30))
    feq = rx.equilibrium(w, D2Q4, rx.advection_flux(w, a), 1.0)
    for i in range(4):
        np.testing.assert_allclose(feq[i], w / 4 + (D2Q4[i] @ a) * w / 2, rtol=1e-15)


@pytest.mark.parametrize("omega", [2.0, 1.3, 0.4])
def test_collision_conserves_moments(omega):
    rng = np.random.default_rng(4)
    f = rng.uniform(0.1, 1.0, (6, 5, 40))
    prob_feq = lambda w: rx.equilibrium(w, D3Q6 * 3.0, rx.euler_flux(w, 1.4), 3.0)
    f = prob_feq(_euler_state(3, 40, 3)) + 0.01 * f
    g = rx.relax(f, omega, prob_feq)
    np.testing.assert_allclose(rx.moments(g), rx.moments(f), rtol=1e-14, atol=1e-14)


def test_equilibrium_is_fixed_point_and_omega2_involution():
    feq_fn = lambda w: rx.equilibrium(w, D2Q4 * 3.0, rx.euler_flux(w, 1.4), 3.0)
    w = _euler_state(2, 25, 5)
    feq = feq_fn(w)
    np.testing.assert_allclose(rx.relax(feq, 1.7, feq_fn), feq, rtol=1e-14, atol=1e-14)
    f = feq + 0.05 * np.random.default_rng(6).standard_normal(feq.shape)
    back = rx.relax(rx.relax(f, 2.0, feq_fn), 2.0, feq_fn)
    np.testing.assert_allclose(back, f, rtol=1e-12, atol=1e-12)


def test_collision_matches_explicit_crank_nicolson_form():
    # eq. collision_cn: C_2 F = (2 tau - dt) F/(2 tau + dt) + 2 dt F^eq/(2 tau + dt)
    tau, dt = 0.03, 0.02
    omega = 2 * dt / (2 * tau + dt)
    feq_fn = lambda w: rx.equilibrium(w, D2Q4, rx.advection_flux(w, [0.3, -0.2]), 1.0)
    f = np.random.default_rng(8).uniform(0.2, 1.0, (4, 1, 17))
    want = (2 * tau - dt) * f / (2 * tau + dt) + 2 * dt * feq_fn(rx.moments(f)) / (2 * tau + dt)
    np.testing.assert_allclose(rx.relax(f, omega, feq_fn), want, rtol=1e-14)


def test_plain_moments_close_to_exactly_rounded():
    f = np.random.default_rng(9).standard_normal((6, 3, 200)) * 1e3
    np.testing.assert_allclose(rx.moments(f), rx.moments_fsum(f), rtol=0, atol=1e-12 * np.max(np.abs(f)))
