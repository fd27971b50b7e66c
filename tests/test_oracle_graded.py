"""Pins of the oracle on tensor-product graded meshes (box cells of varying
size along each axis; the affine cell maps of Sec. 3.1 with per-cell
Jacobians): equal edges reproduce the uniform mesh, Q_d polynomials are
differentiated exactly (nodal DG collocation), constants are preserved, the
weighted upwind operator is dissipative, the sweep equals the global direct
solve, and polynomial profiles are translated exactly by the theta-scheme.
A planted mistake (every cell given the average size) must break them."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import mesh as omesh
from oracle import transport as tr

CASES = [
    # dim, n, degree, velocity, stretch, jitter
    (1, (6,), 2, (0.8,), 1.5, 0.3),
    (2, (4, 5), 1, (1.0, 0.0), 1.2, 0.2),
    (2, (5, 4), 3, (0.0, -1.0), 2.0, 0.0),
    (2, (4, 4), 2, (-0.6, 0.9), 1.0, 0.3),
    (3, (3, 2, 4), 2, (0.0, 0.0, -1.0), 1.5, 0.2),
    (3, (3, 3, 2), 1, (0.7, -0.4, 0.5), 0.8, 0.25),
]


def _mesh(case):
    dim, n, d, v, stretch, jitter = case
    hi = np.array([1.0, 1.3, 0.7][:dim])
    edges = [W.graded_edges(n[k], 0.0, hi[k], stretch, jitter, seed=k) for k in range(dim)]
    return omesh.Mesh(n, None, None, d, edges), np.array(v, float)


def _weights(m):
    # omega_{L,i} = omegahat_i det(tau_L'), det = prod_k (cell size along k) / 2
    sizes = [np.diff(e) / 2.0 for e in m.edges]
    multi = m.cell_multi(np.arange(m.nc))
    det = np.prod([sizes[k][multi[:, k]] for k in range(m.dim)], axis=0)
    return (det[:, None] * m.what[None, :]).ravel()


def _qd_poly(dim, d, seed):
    rng = np.random.default_rng(seed)
    coef = rng.standard_normal((d + 1,) * dim)

    def p(x):
        out = np.zeros(len(x))
        for idx in np.ndindex(coef.shape):
            out += coef[idx] * np.prod([x[:, k] ** idx[k] for k in range(dim)], axis=0)
        return out

    def grad(x):
        g = np.zeros((len(x), dim))
        for idx in np.ndindex(coef.shape):
            for k in range(dim):
                if idx[k] == 0:
                    continue
                term = coef[idx] * idx[k] * x[:, k] ** (idx[k] - 1)
                for l in range(dim):
                    if l != k:
                        term = term * x[:, l] ** idx[l]
                g[:, k] += term
        return g
    return p, grad


def test_graded_edges_are_increasing_and_span_the_box():
    for stretch, jitter in [(0.0, 0.0), (1.5, 0.0), (2.0, 0.4)]:
        e = W.graded_edges(9, 0.25, 2.0, stretch, jitter, seed=3)
        assert e[0] == 0.25 and e[-1] == 2.0 and np.all(np.diff(e) > 0)
    np.testing.assert_allclose(W.graded_edges(4, 0.0, 1.0, 0.0), [0, 0.25, 0.5, 0.75, 1.0], atol=1e-15)


def test_equal_edges_reproduce_the_uniform_mesh():
    n, lo, hi = (4, 3), np.zeros(2), np.array([1.0, 1.3])
    uni = omesh.Mesh(n, lo, hi, 2)
    edges = [np.linspace(lo[k], hi[k], n[k] + 1) for k in range(2)]
    grd = omesh.Mesh(n, None, None, 2, edges)
    v = np.array([0.6, -0.8])
    a, _, ea = tr.assemble(uni, v)
    b, _, eb = tr.assemble(grd, v)
    assert abs(a - b).max() <= 1e-12 * abs(a).max()
    np.testing.assert_allclose(ea["coords"], eb["coords"], atol=1e-14)


@pytest.mark.parametrize("case", CASES)
def test_polynomials_in_qd_are_differentiated_exactly(case):
    m, v = _mesh(case)
    lh, bb, ent = tr.assemble(m, v)
    p, grad = _qd_poly(m.dim, m.degree, 7)
    x = m.node_coords().reshape(-1, m.dim)
    lhs = lh @ p(x) + bb @ p(ent["coords"])
    rhs = -grad(x) @ v
    scale = np.max(np.abs(lh).sum(axis=1)) * np.max(np.abs(p(x)))
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * scale


@pytest.mark.parametrize("case", CASES)
def test_constant_states_are_preserved(case):
    m, v = _mesh(case)
    lh, bb, ent = tr.assemble(m, v)
    r = lh @ np.ones(m.nc * m.nd) + bb @ np.ones(ent["cell"].size)
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(lh).sum(axis=1))


@pytest.mark.parametrize("case", CASES)
def test_upwind_dissipation_weighted(case):
    m, v = _mesh(case)
    lh, _, _ = tr.assemble(m, v)
    wdiag = sp.diags(_weights(m))
    rng = np.random.default_rng(3)
    for _ in range(5):
        f = rng.standard_normal(m.nc * m.nd)
        assert f @ (wdiag @ (lh @ f)) <= 1e-12 * (f @ f)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_sweep_equals_global_direct_solve(case, theta):
    m, v = _mesh(case)
    ent = tr.inflow_entries(m, v)
    rng = np.random.default_rng(11)
    f = rng.standard_normal((2, m.nc, m.nd))
    fbo = rng.standard_normal((2, ent["cell"].size))
    fbn = rng.standard_normal((2, ent["cell"].size))
    dt = 0.37 * np.min(m.h) / np.max(np.abs(v))
    a = tr.theta_step_direct(m, v, f, fbo, fbn, dt, theta)
    b = tr.theta_step_sweep(m, v, f, fbo, fbn, dt, theta)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("theta,tdeg", [(0.5, 2), (1.0, 1)])
def test_polynomial_profile_is_translated_exactly(case, theta, tdeg):
    m, v = _mesh(case)
    k = min(m.degree, tdeg)
    rng = np.random.default_rng(13)
    terms = [idx for idx in np.ndindex((k + 1,) * m.dim) if sum(idx) <= k]
    coef = rng.standard_normal(len(terms))

    def p(x):
        return sum(c * np.prod([x[:, j] ** t[j] for j in range(m.dim)], axis=0) for c, t in zip(coef, terms))

    ent = tr.inflow_entries(m, v)
    x = m.node_coords().reshape(-1, m.dim)
    dt = 0.53 * np.min(m.h) / np.max(np.abs(v))
    f = p(x).reshape(1, m.nc, m.nd)
    g = tr.theta_step_sweep(m, v, f, p(ent["coords"])[None], p(ent["coords"] - dt * v)[None], dt, theta)
    want = p(x - dt * v).reshape(1, m.nc, m.nd)
    assert np.max(np.abs(g - want)) <= 1e-12 * np.max(np.abs(want))


def test_planted_average_cell_size_is_caught():
    # the cell maps take the average cell size (volume and face terms), the
    # node coordinates stay right, so the faces still match
    m, v = _mesh(CASES[3])
    avg = [(e[-1] - e[0]) / (len(e) - 1) for e in m.edges]
    orig = m.jacobian
    coords = m.node_coords()
    m.node_coords = lambda cells=None: coords if cells is None else coords[np.asarray(cells, dtype=np.int64)]

    def wrong_jacobian(cells):
        jac = orig(cells)
        for k in range(m.dim):
            jac[:, k, k] = avg[k] / 2.0
        return jac
    m.jacobian = wrong_jacobian
    lh, bb, ent = tr.assemble(m, v)
    p, grad = _qd_poly(m.dim, m.degree, 7)
    x = m.node_coords().reshape(-1, m.dim)
    lhs = lh @ p(x) + bb @ p(ent["coords"])
    rhs = -grad(x) @ v
    scale = np.max(np.abs(lh).sum(axis=1)) * np.max(np.abs(p(x)))
    assert np.max(np.abs(lhs - rhs)) > 1e-6 * scale
