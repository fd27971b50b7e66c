"""Pins of the oracle on uniform affine meshes: every cell the same
parallelogram / parallelepiped spanned by the lattice vectors a_k (the
columns of A), tau_L(xh) = corner_L + A (xh + 1) / 2 (Sec. 3.1: affine maps,
cofactor of eq. co_mat, weights of eq. map_GL).

* Total-degree-d polynomials map to Q_d on the reference cell, so they are
  differentiated exactly: L_h p + b(p) = -v . grad p.
* Constants are preserved; the weighted upwind operator is dissipative.
* The sweep equals the global direct solve; the theta-scheme translates
  polynomial profiles exactly.
* The affine reduction: with the same cell numbering, the mesh of lattice A
  and velocity v has the same discrete operator and the same inflow
  couplings as the unit box mesh (cells [0,1]^D) with velocity A^{-1} v: the
  cofactor turns v into A^{-1} v in every volume and face term.
* Planted mistakes must fail: the transposed lattice matrix in the cell
  maps, and the velocity transformed with A instead of A^{-1}.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import mesh as omesh
from oracle import transport as tr

CASES = [
    # dim, n, degree, lattice A (columns = cell edge vectors), velocity
    (2, (4, 3), 1, [[0.25, 0.10], [0.0, 0.30]], (1.0, 0.0)),
    (2, (3, 4), 2, [[0.30, 0.0], [-0.08, 0.25]], (0.0, 1.0)),
    (2, (4, 4), 3, [[0.25, 0.12], [0.05, 0.20]], (-0.6, 0.9)),
    (2, (3, 3), 2, [[0.3, -0.1], [0.1, 0.3]], (1.0, 1.0)),
    (3, (3, 2, 3), 1, [[0.3, 0.1, 0.0], [0.0, 0.4, 0.05], [0.0, 0.0, 0.3]], (0.0, 0.0, -1.0)),
    (3, (2, 3, 2), 2, [[0.4, 0.0, 0.1], [0.05, 0.3, 0.0], [0.0, -0.06, 0.35]], (0.7, -0.4, 0.5)),
]


def _mesh(case, axes=None):
    dim, n, d, a, v = case
    a = np.array(a, float)
    return omesh.Mesh(n, np.array([0.1, -0.2, 0.3][:dim]), None, d, axes=a if axes is None else axes), \
        np.array(v, float), a


def _weights(m):
    det = np.linalg.det(m.axes / 2.0)
    return np.tile(det * m.what, m.nc)


def _pd_poly(dim, d, seed):
    """A random polynomial of total degree d and its gradient."""
    rng = np.random.default_rng(seed)
    terms = [idx for idx in np.ndindex((d + 1,) * dim) if sum(idx) <= d]
    coef = rng.standard_normal(len(terms))

    def p(x):
        return sum(c * np.prod([x[:, j] ** t[j] for j in range(dim)], axis=0) for c, t in zip(coef, terms))

    def grad(x):
        g = np.zeros((len(x), dim))
        for c, t in zip(coef, terms):
            for k in range(dim):
                if t[k] == 0:
                    continue
                term = c * t[k] * x[:, k] ** (t[k] - 1)
                for j in range(dim):
                    if j != k:
                        term = term * x[:, j] ** t[j]
                g[:, k] += term
        return g
    return p, grad


def test_lattice_geometry():
    m, _, a = _mesh(CASES[2])
    x = m.node_coords()
    # cell (1, 2): its corner node is lo + a_0 + 2 a_1, its far node adds a_0 + a_1
    c = m.cell_flat(np.array([[1, 2]]))[0]
    np.testing.assert_allclose(x[c, 0], m.lo + a[:, 0] + 2 * a[:, 1], atol=1e-15)
    np.testing.assert_allclose(x[c, -1], m.lo + 2 * a[:, 0] + 3 * a[:, 1], atol=1e-15)
    with pytest.raises(ValueError):
        omesh.Mesh((2, 2), np.zeros(2), None, 1, axes=[[0.0, 1.0], [1.0, 0.0]])   # det < 0


@pytest.mark.parametrize("case", CASES)
def test_polynomials_of_degree_d_are_differentiated_exactly(case):
    m, v, _ = _mesh(case)
    lh, bb, ent = tr.assemble(m, v)
    p, grad = _pd_poly(m.dim, m.degree, 7)
    x = m.node_coords().reshape(-1, m.dim)
    lhs = lh @ p(x) + bb @ p(ent["coords"])
    rhs = -grad(x) @ v
    scale = np.max(np.abs(lh).sum(axis=1)) * np.max(np.abs(p(x)))
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * scale


@pytest.mark.parametrize("case", CASES)
def test_constant_states_are_preserved(case):
    m, v, _ = _mesh(case)
    lh, bb, ent = tr.assemble(m, v)
    r = lh @ np.ones(m.nc * m.nd) + bb @ np.ones(ent["cell"].size)
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(lh).sum(axis=1))


@pytest.mark.parametrize("case", CASES)
def test_upwind_dissipation_weighted(case):
    m, v, _ = _mesh(case)
    lh, _, _ = tr.assemble(m, v)
    wdiag = sp.diags(_weights(m))
    rng = np.random.default_rng(3)
    for _ in range(5):
        f = rng.standard_normal(m.nc * m.nd)
        assert f @ (wdiag @ (lh @ f)) <= 1e-12 * (f @ f)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_sweep_equals_global_direct_solve(case, theta):
    m, v, _ = _mesh(case)
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
    m, v, _ = _mesh(case)
    p, _ = _pd_poly(m.dim, min(m.degree, tdeg), 13)
    ent = tr.inflow_entries(m, v)
    x = m.node_coords().reshape(-1, m.dim)
    dt = 0.53 * np.min(m.h) / np.max(np.abs(v))
    f = p(x).reshape(1, m.nc, m.nd)
    g = tr.theta_step_sweep(m, v, f, p(ent["coords"])[None], p(ent["coords"] - dt * v)[None], dt, theta)
    want = p(x - dt * v).reshape(1, m.nc, m.nd)
    assert np.max(np.abs(g - want)) <= 1e-12 * np.max(np.abs(want))


def _reduction_gap(m, v, a):
    """Largest differences between the lattice mesh with velocity v and the
    unit box mesh with velocity A^{-1} v: operator, inflow couplings, inflow
    cells/nodes, dependency levels."""
    box = omesh.Mesh(m.n, np.zeros(m.dim), np.array(m.n, float), m.degree)
    vb = np.linalg.solve(a, v)
    la, _, ea = tr.assemble(m, v)
    lb, _, eb = tr.assemble(box, vb)
    op = abs(la - lb).max() / abs(lb).max()
    same_entries = (np.array_equal(ea["cell"], eb["cell"]) and np.array_equal(ea["node"], eb["node"])
                    and np.array_equal(ea["face"], eb["face"]))
    coef = np.max(np.abs(ea["coef"] - eb["coef"])) / np.max(np.abs(eb["coef"])) if same_entries else np.inf
    levels = np.array_equal(tr.topological_levels(m, v), tr.topological_levels(box, vb))
    return op, coef, levels


@pytest.mark.parametrize("case", CASES)
def test_lattice_mesh_equals_unit_box_mesh_with_transformed_velocity(case):
    m, v, a = _mesh(case)
    op, coef, levels = _reduction_gap(m, v, a)
    assert op <= 1e-13 and coef <= 1e-13 and levels


def test_planted_transposed_lattice_is_caught():
    # cell maps built from A^T (the node coordinates stay those of A, so the
    # faces still match): the exactness pin must fail
    m, v, a = _mesh(CASES[2])
    coords = m.node_coords()
    m.node_coords = lambda cells=None: coords if cells is None else coords[np.asarray(cells, dtype=np.int64)]
    m.jacobian = lambda cells: np.broadcast_to(a.T / 2.0, (len(np.atleast_1d(cells)), 2, 2)).copy()
    lh, bb, ent = tr.assemble(m, v)
    p, grad = _pd_poly(m.dim, m.degree, 7)
    x = m.node_coords().reshape(-1, m.dim)
    lhs = lh @ p(x) + bb @ p(ent["coords"])
    rhs = -grad(x) @ v
    scale = np.max(np.abs(lh).sum(axis=1)) * np.max(np.abs(p(x)))
    assert np.max(np.abs(lhs - rhs)) > 1e-6 * scale


def test_planted_forward_transformed_velocity_is_caught():
    # the reduction with A v instead of A^{-1} v must not match
    m, v, a = _mesh(CASES[3])
    box = omesh.Mesh(m.n, np.zeros(2), np.array(m.n, float), m.degree)
    la, _, _ = tr.assemble(m, v)
    lb, _, _ = tr.assemble(box, a @ v)
    assert abs(la - lb).max() > 1e-3 * abs(la).max()
