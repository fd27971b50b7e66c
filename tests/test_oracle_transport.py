"""Pins of the oracle's DG transport operator and theta-scheme step.

Every check below is fixed by the paper or by mathematics, not by the oracle
itself: constant preservation and dissipation (Sec. 3.1, properties of the
transport matrix), exactness on Q_d polynomials (nodal DG collocation), a
hand-derived 1D example, the dependency-graph figure of Sec. 4.1, block
triangularity in topological order (Sec. 4.1), the sweep against a global
sparse direct solve, the discrete mass balance, time symmetry of T_2
(eq. prop_sym) and exact translation of polynomial profiles.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from conftest import read_golden
from oracle import mesh as omesh
from oracle import transport as tr

CASES = [
    # dim, n, degree, velocity, box size
    (1, (5,), 1, (0.7,), (1.0,)),
    (1, (4,), 3, (-1.3,), (2.0,)),
    (2, (3, 4), 1, (1.0, 0.0), (1.0, 1.3)),
    (2, (3, 4), 2, (0.0, -1.0), (1.0, 1.3)),
    (2, (4, 3), 3, (-2.0, 0.0), (1.0, 0.7)),
    (2, (3, 3), 4, (0.5, -0.3), (1.0, 1.0)),
    (3, (2, 3, 2), 1, (0.0, 0.0, 1.0), (1.0, 1.3, 0.7)),
    (3, (2, 2, 3), 2, (-0.4, 0.9, 0.2), (1.0, 1.0, 1.0)),
    (3, (2, 3, 2), 2, (0.0, -1.0, 0.0), (1.0, 0.5, 2.0)),
]


def _mesh(case):
    dim, n, d, v, size = case
    return omesh.Mesh(n, np.zeros(dim), np.array(size), d), np.array(v, float)


def _weights(m):
    # omega_{L,i} = omegahat_i det(tau_L') with tau_L' = diag(h/2)  (eq. map_GL)
    return np.tile(m.what * np.prod(m.h / 2.0), m.nc)


def _qd_poly(dim, d, seed):
    """Random p in Q_d (degree <= d in each variable) and its gradient."""
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


@pytest.mark.parametrize("case", CASES)
def test_constant_states_are_preserved(case):
    m, v = _mesh(case)
    lh, bb, ent = tr.assemble(m, v)
    r = lh @ np.ones(m.nc * m.nd) + bb @ np.ones(ent["cell"].size)
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(lh).sum(axis=1))


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
def test_upwind_dissipation_weighted(case):
    m, v = _mesh(case)
    lh, _, _ = tr.assemble(m, v)
    wdiag = sp.diags(_weights(m))
    rng = np.random.default_rng(3)
    for _ in range(5):
        f = rng.standard_normal(m.nc * m.nd)
        assert f @ (wdiag @ (lh @ f)) <= 1e-12 * (f @ f)


def test_one_cell_1d_degree1_worked_example():
    vals = {}
    for row in read_golden("dg1d_degree1_one_cell.txt"):
        key, _, val = row[0].partition("=")
        vals[key.strip()] = [float(t) for t in val.split(",")]
    h, v = vals["h"][0], vals["v"][0]
    m = omesh.Mesh((1,), (0.0,), (h,), 1)
    lh, bb, ent = tr.assemble(m, (v,))
    np.testing.assert_allclose(lh.toarray().ravel(), vals["L"], atol=1e-14)
    np.testing.assert_allclose(bb.toarray().ravel(), vals["b"], atol=1e-14)
    # f = x on [0, h]: derivative -v at both nodes
    np.testing.assert_allclose(lh @ np.array([0.0, h]) + bb @ np.array([0.0]), [-v, -v], atol=1e-14)


def test_dependency_graph_levels_of_the_paper_figure():
    rows = read_golden("dependency_levels_3x3.txt")
    m = omesh.Mesh((3, 3), (0.0, 0.0), (1.0, 1.0), 1)
    levels = tr.topological_levels(m, (1.0, 1.0))
    for lev, cells in rows:
        want = sorted(int(c) for c in cells.split(","))
        assert sorted(np.nonzero(levels == int(lev))[0].tolist()) == want


@pytest.mark.parametrize("v,axis", [((1.0, 0.0, 0.0), 0), ((0.0, -2.0, 0.0), 1), ((0.0, 0.0, 0.5), 2)])
def test_axis_aligned_levels_are_planes(v, axis):
    m = omesh.Mesh((3, 4, 5), np.zeros(3), np.ones(3), 1)
    levels = tr.topological_levels(m, v)
    pos = m.cell_multi(np.arange(m.nc))[:, axis]
    want = pos if v[axis] > 0 else m.n[axis] - 1 - pos
    np.testing.assert_array_equal(levels, want)


def test_cycle_is_rejected():
    # a velocity field is constant, so a cycle needs a forged edge list
    m = omesh.Mesh((2, 2), (0.0, 0.0), (1.0, 1.0), 1)
    orig = tr.dependency_edges
    try:
        tr.dependency_edges = lambda mesh, v: (np.array([0, 1, 3, 2]), np.array([1, 3, 2, 0]))
        with pytest.raises(ValueError):
            tr.topological_levels(m, (1.0, 1.0))
    finally:
        tr.dependency_edges = orig


@pytest.mark.parametrize("case", CASES)
def test_block_lower_triangular_in_topological_order(case):
    m, v = _mesh(case)
    lh, _, _ = tr.assemble(m, v)
    levels = tr.topological_levels(m, v)
    order = np.argsort(levels, kind="stable")
    rank = np.empty(m.nc, dtype=np.int64)
    rank[order] = np.arange(m.nc)
    coo = lh.tocoo()
    rb = rank[coo.row // m.nd]
    cb = rank[coo.col // m.nd]
    nz = coo.data != 0.0
    assert np.all(cb[nz] <= rb[nz])


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


def _boundary_flux(m, v, f, fb, ent):
    """Phi = -sum over boundary GL points of mu (v.n)^+ f_L + mu (v.n)^- f^b.

    Written from the divergence theorem on the whole box: face measure
    mu_i |c n| with c n = prod(h/2) (2/h_k) n on an axis-aligned face.
    """
    rfaces = tr.reference_faces(m)
    total = 0.0
    cells = np.arange(m.nc)
    jh = np.prod(m.h / 2.0)
    for e, (axis, side, nhat, on, mu) in enumerate(rfaces):
        nbr = m.neighbour(cells, axis, side)
        bnd = cells[nbr < 0]
        vn = v[axis] * side * jh * 2.0 / m.h[axis]
        if vn > 0:
            total -= vn * np.sum(mu[None, :] * f[bnd, :])
    if ent["cell"].size:
        total -= np.sum(ent["coef"] * np.prod(m.h / 2.0) * m.what[ent["node"]] * fb)
    return total


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_discrete_mass_balance(case, theta):
    m, v = _mesh(case)
    ent = tr.inflow_entries(m, v)
    rng = np.random.default_rng(5)
    f = rng.standard_normal((1, m.nc, m.nd))
    fbo = rng.standard_normal((1, ent["cell"].size))
    fbn = rng.standard_normal((1, ent["cell"].size))
    dt = 0.41 * np.min(m.h) / np.max(np.abs(v))
    g = tr.theta_step_sweep(m, v, f, fbo, fbn, dt, theta)
    wts = m.what * np.prod(m.h / 2.0)
    lhs = np.sum(wts[None, :] * (g[0] - f[0]))
    rhs = dt * (theta * _boundary_flux(m, v, g[0], fbn[0], ent)
                + (1 - theta) * _boundary_flux(m, v, f[0], fbo[0], ent))
    assert abs(lhs - rhs) < 1e-12 * (np.sum(np.abs(wts[None, :] * f[0])) + 1.0)


@pytest.mark.parametrize("case", CASES)
def test_crank_nicolson_is_time_symmetric(case):
    m, v = _mesh(case)
    ent = tr.inflow_entries(m, v)
    rng = np.random.default_rng(9)
    f = rng.standard_normal((1, m.nc, m.nd))
    fb = rng.standard_normal((1, ent["cell"].size))
    dt = 0.29 * np.min(m.h) / np.max(np.abs(v))
    g = tr.theta_step_sweep(m, v, f, fb, fb, dt, 0.5)
    back = tr.theta_step_sweep(m, v, g, fb, fb, -dt, 0.5)
    # rounding is amplified by the conditioning of T_2(dt) (the backward step
    # undoes strong upwind damping); bound it with the dense operator
    lh, _, _ = tr.assemble(m, v)
    eye = np.eye(m.nc * m.nd)
    cond = np.linalg.cond(np.linalg.solve(eye - 0.5 * dt * lh.toarray(), eye + 0.5 * dt * lh.toarray()))
    assert np.linalg.norm(back - f) <= max(1e-12, 1e-14 * cond) * np.linalg.norm(f)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("theta,tdeg", [(0.5, 2), (1.0, 1)])
def test_polynomial_profile_is_translated_exactly(case, theta, tdeg):
    m, v = _mesh(case)
    k = min(m.degree, tdeg)
    rng = np.random.default_rng(13)
    # total degree <= k: its translate is a polynomial of degree <= k in t
    terms = [idx for idx in np.ndindex((k + 1,) * m.dim) if sum(idx) <= k]
    coef = rng.standard_normal(len(terms))

    def p(x):
        return sum(c * np.prod([x[:, j] ** t[j] for j in range(m.dim)], axis=0) for c, t in zip(coef, terms))

    ent = tr.inflow_entries(m, v)
    x = m.node_coords().reshape(-1, m.dim)
    dt = 0.53 * np.min(m.h) / np.max(np.abs(v))
    f = p(x).reshape(1, m.nc, m.nd)
    fbo = p(ent["coords"])[None]
    fbn = p(ent["coords"] - dt * v)[None]
    g = tr.theta_step_sweep(m, v, f, fbo, fbn, dt, theta)
    want = p(x - dt * v).reshape(1, m.nc, m.nd)
    assert np.max(np.abs(g - want)) <= 1e-12 * np.max(np.abs(want))


# --- planted mistakes: each must be caught by one of the pins above --------
def test_planted_transposed_derivative_is_caught():
    m, v = _mesh(CASES[5])
    m.dmat = m.dmat.T.copy()
    lh, bb, ent = tr.assemble(m, v)
    p, grad = _qd_poly(m.dim, m.degree, 7)
    x = m.node_coords().reshape(-1, m.dim)
    err = np.max(np.abs(lh @ p(x) + bb @ p(ent["coords"]) + grad(x) @ v))
    assert err > 1e-3


def test_planted_wrong_face_sign_is_caught():
    m, v = _mesh(CASES[3])
    orig = tr.reference_faces

    def flipped(mesh):
        return [(a, s, -nh, on, mu) for (a, s, nh, on, mu) in orig(mesh)]
    try:
        tr.reference_faces = flipped
        lh, bb, ent = tr.assemble(m, v)
        r = lh @ np.ones(m.nc * m.nd) + bb @ np.ones(ent["cell"].size)
    finally:
        tr.reference_faces = orig
    assert np.max(np.abs(r)) > 1e-3


def test_planted_wrong_face_weight_is_caught():
    m, v = _mesh(CASES[4])
    orig = tr.reference_faces

    def doubled(mesh):
        return [(a, s, nh, on, 2.0 * mu) for (a, s, nh, on, mu) in orig(mesh)]
    try:
        tr.reference_faces = doubled
        lh, bb, ent = tr.assemble(m, v)
        r = lh @ np.ones(m.nc * m.nd) + bb @ np.ones(ent["cell"].size)
    finally:
        tr.reference_faces = orig
    assert np.max(np.abs(r)) > 1e-3
