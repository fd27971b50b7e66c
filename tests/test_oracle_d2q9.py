"""Pins of the oracle's D2Q9 isothermal model and its gravity source step
(Sec. 5.1, Euler with gravity; source integrator S_2 of Sec. 3.2).

What fixes them: the lattice isotropy sums of the D2Q9 weights, the moment
conditions P f^eq = w and sum_i f_i^eq v_i v_i = Pi (the isothermal Euler
flux rho c^2 I + rho u u of Sec. 5.1), the time symmetry S(-h) S(h) = Id of
Sec. 3.2, and the hydrostatic steady state rho_0 exp(-g y / c^2) of Sec. 5.1,
which the splitting schemes must approach at their orders (1 for Lie, 2 for
Strang and collapsed Strang), as the paper reports for this test.
"""
import numpy as np
import pytest

from oracle import relax as rx
from oracle import step as ost

D2Q9 = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]], float)


def _state(npts, seed, umax=0.3):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, npts)
    u = rng.uniform(-umax, umax, (2, npts))
    return np.vstack([rho, rho * u[0], rho * u[1]])


@pytest.mark.parametrize("lam", [1.0, 2.5])
def test_weights_reproduce_lattice_isotropy(lam):
    vel = D2Q9 * lam
    wt = rx.d2q9_weights(vel, lam)
    c2 = lam * lam / 3.0
    assert abs(np.sum(wt) - 1.0) < 1e-15
    np.testing.assert_allclose(wt @ vel, 0.0, atol=1e-15)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", wt, vel, vel), c2 * np.eye(2), rtol=1e-14)
    # fourth-order sums of the standard lattice: <v_x^4> = 3 c^4, <v_x^2 v_y^2> = c^4
    assert abs(np.sum(wt * vel[:, 0] ** 4) - 3 * c2 * c2) < 1e-13 * lam ** 4
    assert abs(np.sum(wt * vel[:, 0] ** 2 * vel[:, 1] ** 2) - c2 * c2) < 1e-13 * lam ** 4


@pytest.mark.parametrize("lam", [1.0, 2.5])
def test_equilibrium_moments_and_isothermal_flux(lam):
    vel = D2Q9 * lam
    w = _state(40, 1)
    feq = rx.d2q9_equilibrium(w, vel, lam)
    assert feq.shape == (9, 1, 40)
    np.testing.assert_allclose(rx.d2q9_moments(feq, vel), w, rtol=1e-14, atol=1e-14)
    c2 = lam * lam / 3.0
    rho = w[0]
    u = w[1:] / rho
    second = np.einsum("ia,ib,in->abn", vel, vel, feq[:, 0])
    for a in range(2):
        for b in range(2):
            want = rho * u[a] * u[b] + (rho * c2 if a == b else 0.0)
            np.testing.assert_allclose(second[a, b], want, rtol=1e-13, atol=1e-14)


def test_equilibrium_at_rest_is_weighted_density():
    w = np.array([[1.7], [0.0], [0.0]])
    feq = rx.d2q9_equilibrium(w, D2Q9, 1.0)
    np.testing.assert_allclose(feq[:, 0, 0], 1.7 * rx.d2q9_weights(D2Q9, 1.0), rtol=1e-15)
    assert abs(feq[0, 0, 0] - 1.7 * 4 / 9) < 1e-15 and abs(feq[5, 0, 0] - 1.7 / 36) < 1e-15


def test_equilibrium_follows_velocity_order():
    perm = np.random.default_rng(3).permutation(9)
    w = _state(7, 2)
    a = rx.d2q9_equilibrium(w, D2Q9, 1.0)
    b = rx.d2q9_equilibrium(w, D2Q9[perm], 1.0)
    np.testing.assert_allclose(b, a[perm], rtol=1e-15)


def test_not_a_d2q9_set_is_rejected():
    with pytest.raises(ValueError):
        rx.d2q9_weights(D2Q9[:8], 1.0)
    bad = D2Q9.copy()
    bad[5] = [2.0, 0.0]
    with pytest.raises(ValueError):
        rx.d2q9_weights(bad, 1.0)


def _problem(g=1.0, n=(3, 2), degree=1):
    return ost.Problem(n, (0.0, 0.0), (1.0, 1.0), degree, D2Q9, 1, "d2q9", {"g": g})


def _random_f(prob, seed):
    rng = np.random.default_rng(seed)
    w = _state(prob.mesh.nc * prob.mesh.nd, seed).reshape(3, prob.mesh.nc, prob.mesh.nd)
    return prob.feq(w) + 0.01 * rng.standard_normal((9, 1, prob.mesh.nc, prob.mesh.nd))


def test_source_moves_momentum_exactly_and_keeps_the_rest():
    prob = _problem(g=2.0)
    f = _random_f(prob, 5)
    h = 0.3
    w = prob.moments(f)
    f2 = prob.source(f, h)
    w2 = prob.moments(f2)
    np.testing.assert_allclose(w2[0], w[0], rtol=1e-14)
    np.testing.assert_allclose(w2[1], w[1], atol=1e-14)
    np.testing.assert_allclose(w2[2], w[2] - h * 2.0 * w[0], atol=1e-13)
    # the non-equilibrium part is untouched
    np.testing.assert_allclose(f2 - prob.feq(w2), f - prob.feq(w), atol=1e-14)


def test_source_is_time_symmetric():
    prob = _problem(g=1.3)
    f = _random_f(prob, 6)
    np.testing.assert_array_equal(prob.source(f, 0.0), f)
    back = prob.source(prob.source(f, 0.2), -0.2)
    np.testing.assert_allclose(back, f, atol=1e-14)
    # two half steps make one full step (the moment update is exact)
    np.testing.assert_allclose(prob.source(prob.source(f, 0.1), 0.1), prob.source(f, 0.2), atol=1e-14)


def test_collision_keeps_moments_and_fixes_equilibrium():
    prob = _problem()
    f = _random_f(prob, 7)
    for omega in (1.0, 1.7, 2.0):
        np.testing.assert_allclose(prob.moments(prob.collide(f, omega)), prob.moments(f), atol=1e-14)
    feq = prob.feq(prob.moments(f))
    np.testing.assert_allclose(prob.collide(feq, 2.0), feq, atol=1e-15)
    np.testing.assert_allclose(prob.collide(prob.collide(f, 2.0), 2.0), f, atol=1e-14)


# ---- hydrostatic steady state (Sec. 5.1) --------------------------------------
LAM, G, RHO0 = 1.0, 1.0, 1.0
C2 = LAM * LAM / 3.0
T_END = 0.12


def _w_hydro(x):
    rho = RHO0 * np.exp(-G * x[:, 1] / C2)
    return np.vstack([rho, 0.0 * rho, 0.0 * rho])


def _hydro_error(n, degree, scheme, theta, omega, nsteps, g_source=G):
    prob = ost.Problem((n, n), (0.0, 0.0), (1.0, 1.0), degree, D2Q9 * LAM, 1, "d2q9", {"g": g_source})
    x = prob.mesh.node_coords().reshape(-1, 2)
    w0 = _w_hydro(x).reshape(3, prob.mesh.nc, prob.mesh.nd)
    fb = prob.inflow_from_w(_w_hydro)
    f = ost.run(prob, prob.feq(w0), fb, T_END / nsteps, theta, omega, scheme, nsteps)
    w = prob.moments(f)
    return np.linalg.norm(w - w0) / np.linalg.norm(w0)


@pytest.mark.slow
@pytest.mark.parametrize("name,scheme,theta,omega,n,degree,lo,hi", [
    ("M1s, first-order blocks", ost.LIE, 1.0, 1.0, 4, 3, 0.75, 1.2),
    ("M1,2s, second-order blocks", ost.LIE, 0.5, 2.0, 4, 3, 0.8, 1.2),
    ("M2s Strang", ost.STRANG, 0.5, 2.0, 4, 4, 1.8, 2.3),
    ("M2s collapsed", ost.STRANG_COLLAPSED, 0.5, 2.0, 4, 4, 1.7, 2.3),
])
def test_hydrostatic_state_convergence_orders(name, scheme, theta, omega, n, degree, lo, hi):
    errs = [_hydro_error(n, degree, scheme, theta, omega, N) for N in (5, 10)]
    rate = np.log2(errs[0] / errs[1])
    print(f"{name}: errors {errs}, rate {rate:.2f}")
    assert lo <= rate <= hi, (name, errs, rate)
    assert errs[1] < 0.02


@pytest.mark.slow
def test_wrong_source_sign_breaks_hydrostatic_balance():
    # a planted mistake: gravity with the opposite sign in the source step
    right = _hydro_error(4, 3, ost.STRANG, 0.5, 2.0, 10)
    wrong = _hydro_error(4, 3, ost.STRANG, 0.5, 2.0, 10, g_source=-G)
    assert wrong > 20 * right, (right, wrong)


# ---- M_2^kin and its triple jump with the gravity source (Sec. 3.2 + Sec. 5.1) ----
# The paper gives M_2^kin without a source.  The oracle's reading: each
# collision C(h/2) of M_2^kin(h) carries the source over h/2, as
# S(h/4) C(h/2) S(h/4).  The pins below fix what that reading determines:
# the source commutes with the collision (so its split around one collision
# is immaterial), the composition stays time symmetric, it approaches the
# hydrostatic state at order 2, and the triple jump raises the time order to
# 4.  Planted mistakes (all the source at the first collision; half the
# total source) must fail them.


def _kin_variant(prob, f0, fb, dt, theta, omega, nsteps, pre=(0.25, 0.25), post=(0.25, 0.25)):
    """M_2^kin(dt) steps with source fractions (pre, post) x dt around the
    two collisions; (1/4, 1/4) each is the oracle's reading."""
    f = np.array(f0, dtype=float, copy=True)
    for _ in range(nsteps):
        wh = ost.omega_for(dt / 2, dt, omega)
        f = prob.transport(f, fb, fb, dt / 4, theta)
        f = prob.local(f, pre[0] * dt, wh, post[0] * dt)
        f = prob.transport(f, fb, fb, dt / 2, theta)
        f = prob.local(f, pre[1] * dt, wh, post[1] * dt)
        f = prob.transport(f, fb, fb, dt / 4, theta)
    return f


ALL_AT_FIRST = dict(pre=(0.5, 0.0), post=(0.5, 0.0))     # planted: total right, placement asymmetric
HALF_SOURCE = dict(pre=(0.125, 0.125), post=(0.125, 0.125))  # planted: half the total source


def _kin_setup():
    prob = _problem(g=1.3, n=(3, 2), degree=2)
    f = _random_f(prob, 4)
    fb = [prob.feq(_state(prob.entries(v)["coords"].shape[0], 10 + v))[v] for v in range(9)]
    return prob, f, fb


def _omega_backwards(dt, omega):
    """Collision factor over -dt for the relaxation time that omega fixes over dt."""
    tau = dt * (2.0 - omega) / (2.0 * omega)
    return -2.0 * dt / (2.0 * tau - dt)


@pytest.mark.parametrize("h", [0.3, -0.2])
@pytest.mark.parametrize("omega", [1.6, 2.0])
def test_source_commutes_with_collision(h, omega):
    # S moves only the equilibrium part, C relaxes only the non-equilibrium part
    prob, f, _ = _kin_setup()
    a = prob.source(prob.collide(f, omega), h)
    b = prob.collide(prob.source(f, h), omega)
    assert np.linalg.norm(a - b) <= 1e-14 * np.linalg.norm(a)


@pytest.mark.parametrize("scheme", [ost.KIN, ost.KIN4], ids=["kin", "kin4"])
def test_kin_compositions_with_source_are_time_symmetric(scheme):
    # tau > 0 (omega = 1.6) and g != 0: M(-dt) M(dt) = Id (Sec. 3.2)
    prob, f, fb = _kin_setup()
    dt, omega = 0.05, 1.6
    g = ost.run(prob, f, fb, dt, 0.5, omega, scheme, 1)
    back = ost.run(prob, g, fb, -dt, 0.5, _omega_backwards(dt, omega), scheme, 1)
    assert np.linalg.norm(g - f) > 1e-3 * np.linalg.norm(f)
    assert np.linalg.norm(back - f) <= 1e-13 * np.linalg.norm(f)


def test_planted_asymmetric_source_breaks_time_symmetry():
    prob, f, fb = _kin_setup()
    dt, omega = 0.05, 1.6
    ob = _omega_backwards(dt, omega)
    ok = _kin_variant(prob, _kin_variant(prob, f, fb, dt, 0.5, omega, 1), fb, -dt, 0.5, ob, 1)
    bad = _kin_variant(prob, _kin_variant(prob, f, fb, dt, 0.5, omega, 1, **ALL_AT_FIRST), fb, -dt, 0.5, ob, 1,
                       **ALL_AT_FIRST)
    assert np.linalg.norm(ok - f) <= 1e-13 * np.linalg.norm(f)
    assert np.linalg.norm(bad - f) > 1e-3 * np.linalg.norm(f)
    # and the oracle's KIN is the symmetric variant
    np.testing.assert_allclose(ost.run(prob, f, fb, dt, 0.5, omega, ost.KIN, 2),
                               _kin_variant(prob, f, fb, dt, 0.5, omega, 2), rtol=0, atol=1e-14)


def _hydro_variant_error(n, degree, omega, nsteps, **kw):
    prob = ost.Problem((n, n), (0.0, 0.0), (1.0, 1.0), degree, D2Q9 * LAM, 1, "d2q9", {"g": G})
    x = prob.mesh.node_coords().reshape(-1, 2)
    w0 = _w_hydro(x).reshape(3, prob.mesh.nc, prob.mesh.nd)
    fb = prob.inflow_from_w(_w_hydro)
    f = _kin_variant(prob, prob.feq(w0), fb, T_END / nsteps, 0.5, omega, nsteps, **kw)
    return np.linalg.norm(prob.moments(f) - w0) / np.linalg.norm(w0)


@pytest.mark.slow
@pytest.mark.parametrize("omega", [2.0, 1.6])
def test_kin_hydrostatic_state_second_order(omega):
    errs = [_hydro_error(4, 4, ost.KIN, 0.5, omega, N) for N in (5, 10)]
    rate = np.log2(errs[0] / errs[1])
    print(f"M2kin omega={omega}: errors {errs}, rate {rate:.2f}")
    assert 1.8 <= rate <= 2.3 and errs[1] < 2e-4, (errs, rate)


@pytest.mark.slow
def test_planted_source_mistakes_fail_the_hydrostatic_test():
    # all the source at the first collision: first order
    errs = [_hydro_variant_error(4, 4, 2.0, N, **ALL_AT_FIRST) for N in (5, 10)]
    assert np.log2(errs[0] / errs[1]) < 1.3, errs
    # half the source: the hydrostatic balance is lost, no convergence
    errs = [_hydro_variant_error(4, 4, 2.0, N, **HALF_SOURCE) for N in (5, 10)]
    assert min(errs) > 0.04, errs


@pytest.mark.slow
@pytest.mark.parametrize("scheme,lo,hi", [(ost.KIN, 1.8, 2.2), (ost.KIN4, 3.6, 4.4)], ids=["kin", "kin4"])
def test_kin_time_order_with_source(scheme, lo, hi):
    # time self-convergence on one spatial discretisation (the hydrostatic
    # error of the triple jump is dominated by the spatial error): differences
    # of successive halvings of dt shrink at the time order
    prob = ost.Problem((4, 4), (0.0, 0.0), (1.0, 1.0), 2, D2Q9 * LAM, 1, "d2q9", {"g": G})
    x = prob.mesh.node_coords().reshape(-1, 2)
    w0 = _w_hydro(x).reshape(3, prob.mesh.nc, prob.mesh.nd)
    fb = prob.inflow_from_w(_w_hydro)
    ws = {N: prob.moments(ost.run(prob, prob.feq(w0), fb, T_END / N, 0.5, 2.0, scheme, N)) for N in (6, 12, 24)}
    rate = np.log2(np.linalg.norm(ws[6] - ws[12]) / np.linalg.norm(ws[12] - ws[24]))
    print(f"scheme {scheme}: time order {rate:.2f}")
    assert lo <= rate <= hi, rate
