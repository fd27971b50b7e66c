"""CPU checks of the C ABI: the library loads, exports every declared
symbol, validates its arguments, and its host logic (dependency-graph
levels, layouts, coordinates, cell operator) agrees with the oracle.
No device compute is called here."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT, read_golden
from oracle import mesh as omesh
from oracle import transport as otr


def _load_build_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "pdg_build", os.path.join(ROOT, "paper_1702_00169_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def lib():
    b = _load_build_module()
    if not os.path.exists(b.LIB):
        b.build()
    import paper_1702_00169_amd as P
    return P


def _declared():
    text = open(os.path.join(ROOT, "include", "pdg.h")).read()
    return sorted(set(re.findall(r"\b(pdg_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "pdg_transport_sweep" in names and len(names) >= 14
    so = ctypes.CDLL(lib.LIB_PATH)
    for name in names:
        assert hasattr(so, name), name
    assert set(names) == set(lib.EXPORTED)


def _desc(**kw):
    d = dict(dim=2, n=[4, 3], degree=2, v=[[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [0.0, -1.0]], m=1,
             feq="advection", feq_param=[0.5, 0.25])
    d.update(kw)
    return d


@pytest.mark.parametrize("kw,status", [
    (dict(dim=1, n=[4]), 1), (dict(dim=4), 1), (dict(degree=0), 1), (dict(degree=5), 2),
    (dict(n=[0, 3]), 1), (dict(hi=[1.0, -1.0]), 1), (dict(v=[[float("nan"), 0.0]]), 1),
    (dict(m=0), 1), (dict(m=9), 1),
])
def test_setup_rejects_bad_descriptors(lib, kw, status):
    with pytest.raises(lib.PdgError) as ei:
        lib.pdg_setup_mesh([_desc(**kw)])
    assert ei.value.status == status


def test_null_arguments_are_rejected(lib):
    so = lib._lib
    out = ctypes.c_void_p()
    assert so.pdg_setup_mesh(None, 1, ctypes.byref(out)) == lib.PDG_EINVAL
    assert so.pdg_layout(None, None, None, None, None, None, None) == lib.PDG_EINVAL
    assert so.pdg_transport_sweep(None, None, None, None, 0.1, None) == lib.PDG_EINVAL
    assert so.pdg_relax(None, None, None, None) == lib.PDG_EINVAL
    assert so.pdg_step(None, None, None, 1, None) == lib.PDG_EINVAL
    assert so.pdg_state_to_f64(None, None, None, None) == lib.PDG_EINVAL
    assert so.pdg_state_from_f64(None, None, None, None) == lib.PDG_EINVAL


def test_calls_before_prepare_report_state_error(lib):
    ctx = lib.pdg_setup_mesh([_desc()])
    dummy = ctypes.c_void_p(16)
    assert lib._lib.pdg_transport_sweep(ctx, dummy, dummy, dummy, 0.1, None) == lib.PDG_ESTATE
    assert lib._lib.pdg_relax(ctx, dummy, None, None) == lib.PDG_ESTATE
    assert lib._lib.pdg_step(ctx, dummy, dummy, 2, None) == lib.PDG_ESTATE
    assert lib._lib.pdg_state_to_f64(ctx, dummy, dummy, None) == lib.PDG_ESTATE
    assert lib._lib.pdg_state_from_f64(ctx, dummy, dummy, None) == lib.PDG_ESTATE
    # precisions beyond the 48-bit state are rejected before any device work
    assert lib._lib.pdg_prepare(ctx, 0.01, 0.5, 2.0, 2, 4, None) == lib.PDG_EINVAL
    assert lib._lib.pdg_prepare(ctx, 0.01, 0.5, 2.0, 2, -1, None) == lib.PDG_EINVAL
    lib.pdg_destroy(ctx)


def test_status_strings(lib):
    for s in range(8):
        assert lib.pdg_status_string(s).startswith("PDG_")


def test_levels_of_the_paper_figure(lib):
    ctx = lib.pdg_setup_mesh([_desc(n=[3, 3], degree=1, v=[[1.0, 1.0]])])
    lev = np.zeros(9, np.int32)
    lib.pdg_levels(ctx, 0, 0, lev)
    for level, cells in read_golden("dependency_levels_3x3.txt"):
        assert sorted(np.nonzero(lev == int(level))[0].tolist()) == sorted(int(c) for c in cells.split(","))
    lib.pdg_destroy(ctx)


def test_axis_aligned_levels_are_planes_and_match_oracle(lib):
    vel = [[0.0, 0.0, -2.0], [1.0, 0.0, 0.0], [0.0, 0.5, 0.0], [0.3, -0.2, 0.1]]
    ctx = lib.pdg_setup_mesh([_desc(dim=3, n=[3, 4, 5], degree=1, v=vel)])
    m = omesh.Mesh((3, 4, 5), np.zeros(3), np.ones(3), 1)
    for v in range(4):
        lev = np.zeros(60, np.int32)
        lib.pdg_levels(ctx, 0, v, lev)
        np.testing.assert_array_equal(lev, otr.topological_levels(m, vel[v]))
    lib.pdg_destroy(ctx)


def test_topo_levels_detects_cycles(lib):
    lev = np.zeros(4, np.int32)
    src = np.array([0, 1, 3, 2], np.int32)
    dst = np.array([1, 3, 2, 0], np.int32)
    assert lib.pdg_topo_levels(4, src, dst, lev) == lib.PDG_ENOTDAG
    src = np.array([0, 0, 1, 2], np.int32)
    dst = np.array([1, 2, 3, 3], np.int32)
    assert lib.pdg_topo_levels(4, src, dst, lev) == lib.PDG_OK
    np.testing.assert_array_equal(lev, [0, 1, 1, 2])
    bad = np.array([0, 7], np.int32)
    assert lib.pdg_topo_levels(4, bad, bad, lev) == lib.PDG_EINVAL


def test_layout_sizes(lib):
    descs = [_desc(), _desc(dim=3, n=[2, 3, 4], degree=3, m=5,
                            v=[[1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0], [0, 0, -1], [0, 0, 1]],
                            feq="euler", feq_param=[1.4])]
    prob = lib.Problem(descs)
    lay = prob.layout
    f0 = 4 * 1 * 9 * 12
    f1 = 6 * 5 * 64 * 24
    assert lay["f_elems"] == f0 + f1 and list(lay["f_off"]) == [0, f0, f0 + f1]
    assert lay["w_elems"] == 9 * 12 + 5 * 64 * 24
    fb0 = 3 * (3 + 4 + 3 + 4)                 # per velocity: (d+1) nodes x transverse cells
    fb1 = 5 * 16 * (12 + 8 + 12 + 8 + 6 + 6)
    assert lay["fb_elems"] == fb0 + fb1
    prob.close()


@pytest.mark.parametrize("dim,n,degree", [(2, (3, 5), 3), (3, (2, 3, 4), 2), (2, (4, 2), 4)])
def test_coordinates_match_oracle(lib, dim, n, degree):
    vel = np.vstack([np.eye(dim), -np.eye(dim)])
    hi = [1.0, 2.0, 0.5][:dim]
    prob = lib.Problem([_desc(dim=dim, n=list(n), degree=degree, v=vel, hi=hi, lo=[0.0] * dim)])
    vol, inflow = prob.node_coords(0)
    m = omesh.Mesh(n, np.zeros(dim), np.array(hi), degree)
    want = m.node_coords()                                   # (nc, nd, D)
    np.testing.assert_allclose(np.transpose(vol, (2, 1, 0)), want, atol=1e-14)
    off = 0
    for v in range(vel.shape[0]):
        ent = otr.inflow_entries(m, vel[v])
        npts = ent["coords"].shape[0]
        pts = inflow[off:off + dim * npts].reshape(dim, npts).T
        a = pts[np.lexsort(np.round(pts, 12).T[::-1])]
        b = ent["coords"][np.lexsort(np.round(ent["coords"], 12).T[::-1])]
        np.testing.assert_allclose(a, b, atol=1e-14)
        off += dim * npts
    prob.close()


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
@pytest.mark.parametrize("vel", [(1.3, 0.0, 0.0), (0.0, -0.7, 0.0), (0.0, 0.0, 2.0), (-3.0, 0.0, 0.0)])
def test_host_cell_operator_is_the_oracle_block(lib, degree, vel):
    """Kronecker(I, line block) in downwind-local order == oracle Gamma_{L<-L}."""
    hi = [1.0, 1.7, 0.6]
    prob = lib.Problem([_desc(dim=3, n=[3, 2, 2], degree=degree, v=[list(vel)], hi=hi, lo=[0.0] * 3)])
    npn = degree + 1
    gam = np.zeros(npn * npn)
    kappa = lib.pdg_line_operator(prob.ctx, 0, 0, gam)
    gam = gam.reshape(npn, npn)
    m = omesh.Mesh((3, 2, 2), np.zeros(3), np.array(hi), degree)
    blk = otr.cell_blocks(m, np.array(vel), np.array([5]))
    ax = int(np.nonzero(vel)[0][0])
    s = 1 if vel[ax] > 0 else -1
    idx = m.node_idx
    want = blk.gll[0]
    got = np.zeros_like(want)
    for i in range(m.nd):
        for j in range(m.nd):
            if all(idx[i, k] == idx[j, k] for k in range(3) if k != ax):
                qi = idx[i, ax] if s > 0 else degree - idx[i, ax]
                qj = idx[j, ax] if s > 0 else degree - idx[j, ax]
                got[i, j] = gam[qi, qj]
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13 * np.abs(want).max())
    # inflow coupling: -kappa at the inflow node of the face opposite to v
    fc = [f for f in blk.faces if f["axis"] == ax and f["side"] == -s][0]
    np.testing.assert_allclose(fc["coef"][0], -kappa, rtol=1e-13)
    prob.close()


D2Q9 = [[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]]


@pytest.mark.parametrize("dim,degree,vel", [
    (2, 2, (1.0, 1.0)), (2, 3, (-0.7, 0.4)), (2, 1, (0.3, -1.1)), (2, 4, (-1.0, -1.0)), (2, 2, (0.0, 0.0)),
    (3, 2, (1.0, -1.0, 0.5)), (3, 1, (0.0, 0.8, -0.3)), (3, 2, (0.0, 0.0, -1.0)),
])
def test_host_dense_cell_operator_is_the_oracle_block(lib, dim, degree, vel):
    """Gamma_{L<-L} of any velocity, downwind-local order, == oracle block."""
    hi = [1.0, 1.7, 0.6][:dim]
    n = [3, 2, 2][:dim]
    prob = lib.Problem([_desc(dim=dim, n=n, degree=degree, v=[list(vel)], hi=hi, lo=[0.0] * dim)])
    npn = degree + 1
    nd = npn ** dim
    gam = np.zeros(nd * nd)
    kap = np.zeros(3)
    lib.pdg_cell_operator(prob.ctx, 0, 0, gam, kap)
    gam = gam.reshape(nd, nd)
    m = omesh.Mesh(tuple(n), np.zeros(dim), np.array(hi), degree)
    blk = otr.cell_blocks(m, np.array(vel), np.array([1]))
    idx = m.node_idx
    # oracle node i (physical tensor index) -> downwind-local index q
    q = np.zeros(nd, dtype=np.int64)
    for i in range(nd):
        for a in range(dim):
            qa = idx[i, a] if vel[a] >= 0 else degree - idx[i, a]
            q[i] += qa * npn ** a
    np.testing.assert_allclose(gam[np.ix_(q, q)], blk.gll[0], rtol=1e-13,
                               atol=1e-13 * max(1.0, np.abs(blk.gll[0]).max()))
    for fc in blk.faces:
        a = fc["axis"]
        if vel[a] == 0 or fc["side"] != (-1 if vel[a] > 0 else 1):
            continue
        np.testing.assert_allclose(fc["coef"][0], -kap[a], rtol=1e-13)
    for a in range(dim):
        if vel[a] == 0:
            assert kap[a] == 0.0
    prob.close()


def test_d2q9_setup_layout_and_levels(lib):
    prob = lib.Problem([_desc(n=[5, 4], degree=2, v=D2Q9)])
    lay = prob.layout
    # fb: one face block per non-zero component: axis-aligned 3*n_other, diagonal both faces
    per = [0, 3 * 4, 3 * 5, 3 * 4, 3 * 5] + [3 * 4 + 3 * 5] * 4
    assert lay["fb_elems"] == sum(per)
    m = omesh.Mesh((5, 4), np.zeros(2), np.ones(2), 2)
    for v in range(9):
        lev = np.zeros(20, np.int32)
        lib.pdg_levels(prob.ctx, 0, v, lev)
        np.testing.assert_array_equal(lev, otr.topological_levels(m, D2Q9[v]))
    # inflow coordinates, velocity by velocity, == oracle inflow entries
    _, inflow = prob.node_coords(0)
    off = 0
    for v in range(9):
        ent = otr.inflow_entries(m, np.array(D2Q9[v], float))
        npts = ent["coords"].shape[0]
        if npts == 0:
            assert vel_is_zero(D2Q9[v])
            continue
        pts = np.concatenate([b.T for b in _split_faces(inflow[off:off + 2 * npts], D2Q9[v], (5, 4), 3)])
        a = pts[np.lexsort(np.round(pts, 12).T[::-1])]
        b = ent["coords"][np.lexsort(np.round(ent["coords"], 12).T[::-1])]
        np.testing.assert_allclose(a, b, atol=1e-14)
        off += 2 * npts
    prob.close()


def vel_is_zero(v):
    return all(c == 0 for c in v)


def _split_faces(flat, vel, n, npn):
    """Split one velocity's inflow coordinate block into its face blocks (D, t*tau)."""
    dim = len(n)
    out = []
    off = 0
    for a in range(dim):
        if vel[a] == 0:
            continue
        npts = npn ** (dim - 1) * int(np.prod(n)) // n[a]
        out.append(flat[off:off + dim * npts].reshape(dim, npts))
        off += dim * npts
    return out


def _d2q9_desc(**kw):
    d = dict(dim=2, n=[5, 4], degree=2, v=np.array(D2Q9, float) * 1.5, m=1, feq="d2q9", feq_param=[0.7])
    d.update(kw)
    return d


def test_d2q9_model_layout_has_three_moments(lib):
    prob = lib.Problem([_d2q9_desc(), _desc()])
    lay = prob.layout
    nodes = 20 * 9
    assert lay["w_off"][1] == 3 * nodes                 # rho, rho u_x, rho u_y
    assert lay["w_elems"] == 3 * nodes + 12 * 9       # then the scalar instance (m = 1)
    assert lay["f_elems"] == 9 * nodes + 4 * 12 * 9
    prob.close()


@pytest.mark.parametrize("kw", [
    dict(m=2), dict(v=np.array(D2Q9[:8] + [[2, 0]], float)), dict(v=np.array(D2Q9, float) * [1.0, 2.0]),
    dict(v=np.array(D2Q9[:8] + [[1, 1]], float)), dict(feq_param=[float("inf")]),
    dict(v=np.zeros((9, 2))),
])
def test_d2q9_model_rejects_a_malformed_lattice(lib, kw):
    with pytest.raises(lib.PdgError) as e:
        lib.Problem([_d2q9_desc(**kw)])
    assert e.value.status == lib.PDG_EINVAL


def test_d2q9_model_accepts_any_velocity_order(lib):
    perm = np.random.default_rng(0).permutation(9)
    prob = lib.Problem([_d2q9_desc(v=np.array(D2Q9, float)[perm] * 0.5)])
    assert prob.layout["w_elems"] == 3 * 20 * 9
    prob.close()


def test_source_before_prepare_is_a_state_error(lib):
    prob = lib.Problem([_d2q9_desc()])
    assert lib._lib.pdg_source(prob.ctx, ctypes.c_void_p(8), 0.1, None) == lib.PDG_ESTATE
    assert lib._lib.pdg_source(None, ctypes.c_void_p(8), 0.1, None) == lib.PDG_EINVAL
    assert lib._lib.pdg_source(prob.ctx, None, 0.1, None) == lib.PDG_EINVAL
    prob.close()


# ---- graded meshes (per-axis cell edges) ------------------------------------
import workloads as W  # noqa: E402


def _graded_edges(n, hi, graded_axes):
    return [W.graded_edges(n[k], 0.0, hi[k], 1.4, 0.25, seed=k) if k in graded_axes else None
            for k in range(len(n))]


@pytest.mark.parametrize("dim,n,degree,graded_axes", [
    (2, (5, 4), 2, (0,)), (2, (4, 6), 3, (0, 1)), (3, (3, 4, 2), 1, (1, 2)), (3, (2, 3, 4), 2, (0, 1, 2)),
])
def test_graded_coordinates_match_oracle(lib, dim, n, degree, graded_axes):
    vel = np.vstack([np.eye(dim), -np.eye(dim)])
    hi = [1.0, 2.0, 0.5][:dim]
    edges = _graded_edges(n, hi, graded_axes)
    prob = lib.Problem([_desc(dim=dim, n=list(n), degree=degree, v=vel, hi=hi, lo=[0.0] * dim, edges=edges)])
    vol, inflow = prob.node_coords(0)
    full = [e if e is not None else np.linspace(0.0, hi[k], n[k] + 1) for k, e in enumerate(edges)]
    m = omesh.Mesh(n, None, None, degree, full)
    np.testing.assert_allclose(np.transpose(vol, (2, 1, 0)), m.node_coords(), atol=1e-14)
    off = 0
    for v in range(vel.shape[0]):
        ent = otr.inflow_entries(m, vel[v])
        npts = ent["coords"].shape[0]
        pts = inflow[off:off + dim * npts].reshape(dim, npts).T
        a = pts[np.lexsort(np.round(pts, 12).T[::-1])]
        b = ent["coords"][np.lexsort(np.round(ent["coords"], 12).T[::-1])]
        np.testing.assert_allclose(a, b, atol=1e-14)
        off += dim * npts
    prob.close()


@pytest.mark.parametrize("degree", [1, 3])
@pytest.mark.parametrize("vel", [(1.3, 0.0), (-0.7, 0.0), (0.0, 2.0), (0.0, -1.1)])
def test_graded_line_operator_is_the_oracle_block_of_the_first_cell(lib, degree, vel):
    n, hi = (4, 3), [1.0, 1.7]
    edges = _graded_edges(n, hi, (0, 1))
    prob = lib.Problem([_desc(dim=2, n=list(n), degree=degree, v=[list(vel)], hi=hi, lo=[0.0, 0.0], edges=edges)])
    npn = degree + 1
    gam = np.zeros(npn * npn)
    kappa = lib.pdg_line_operator(prob.ctx, 0, 0, gam)
    gam = gam.reshape(npn, npn)
    m = omesh.Mesh(n, None, None, degree, edges)
    ax = int(np.nonzero(vel)[0][0])
    s = 1 if vel[ax] > 0 else -1
    multi = [1, 1]
    multi[ax] = 0 if s > 0 else n[ax] - 1                  # the chain's upwind-most cell
    cell = multi[0] + n[0] * multi[1]
    blk = otr.cell_blocks(m, np.array(vel), np.array([cell]))
    idx = m.node_idx
    want = blk.gll[0]
    got = np.zeros_like(want)
    for i in range(m.nd):
        for j in range(m.nd):
            if all(idx[i, k] == idx[j, k] for k in range(2) if k != ax):
                qi = idx[i, ax] if s > 0 else degree - idx[i, ax]
                qj = idx[j, ax] if s > 0 else degree - idx[j, ax]
                got[i, j] = gam[qi, qj]
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13 * np.abs(want).max())
    fc = [f for f in blk.faces if f["axis"] == ax and f["side"] == -s][0]
    np.testing.assert_allclose(fc["coef"][0], -kappa, rtol=1e-13)
    prob.close()


@pytest.mark.parametrize("edges", [
    [np.array([0.0, 0.5, 0.4, 1.0, 1.2, 1.5]), None], [np.array([0.0, 0.1, 0.2, 0.3, np.nan, 1.0]), None],
    [np.array([0.0, 0.1, 0.2, 0.3, 0.4, 0.4]), None],
])
def test_graded_edges_are_validated(lib, edges):
    with pytest.raises(lib.PdgError) as e:
        lib.Problem([_desc(n=[5, 3], edges=edges)])
    assert e.value.status == lib.PDG_EINVAL


@pytest.mark.parametrize("dim,degree,vel", [
    (2, 2, (1.0, 1.0)), (2, 3, (-0.7, 0.4)), (2, 1, (0.3, -1.1)), (3, 2, (1.0, -1.0, 0.5)), (3, 1, (0.0, 0.8, -0.3)),
])
def test_graded_dense_cell_operator_is_the_oracle_block_of_the_first_cell(lib, dim, degree, vel):
    """Dense velocities on graded meshes: the block of the upwind-most cell
    (cell sizes of that cell along every graded axis)."""
    n = [4, 3, 3][:dim]
    hi = [1.0, 1.7, 0.6][:dim]
    edges = _graded_edges(n, hi, tuple(range(dim)))
    prob = lib.Problem([_desc(dim=dim, n=n, degree=degree, v=[list(vel)], hi=hi, lo=[0.0] * dim, edges=edges)])
    npn = degree + 1
    nd = npn ** dim
    gam = np.zeros(nd * nd)
    kap = np.zeros(3)
    lib.pdg_cell_operator(prob.ctx, 0, 0, gam, kap)
    gam = gam.reshape(nd, nd)
    m = omesh.Mesh(tuple(n), None, None, degree, edges)
    multi = [0 if vel[a] >= 0 else n[a] - 1 for a in range(dim)]
    cell = int(m.cell_flat(np.array([multi]))[0])
    blk = otr.cell_blocks(m, np.array(vel), np.array([cell]))
    idx = m.node_idx
    q = np.zeros(nd, dtype=np.int64)
    for i in range(nd):
        for a in range(dim):
            qa = idx[i, a] if vel[a] >= 0 else degree - idx[i, a]
            q[i] += qa * npn ** a
    np.testing.assert_allclose(gam[np.ix_(q, q)], blk.gll[0], rtol=1e-13,
                               atol=1e-13 * max(1.0, np.abs(blk.gll[0]).max()))
    prob.close()


# ---- uniform affine lattices (every cell the same parallelogram / parallelepiped)
AFFINE = [
    (2, (4, 3), 2, [[0.25, 0.10], [0.0, 0.30]]),
    (2, (3, 4), 3, [[0.30, 0.0], [-0.08, 0.25]]),
    (3, (3, 2, 3), 1, [[0.3, 0.1, 0.0], [0.0, 0.4, 0.05], [0.0, 0.0, 0.3]]),
]


@pytest.mark.parametrize("dim,n,degree,axes", AFFINE)
def test_affine_coordinates_and_levels_match_oracle(lib, dim, n, degree, axes):
    axes = np.array(axes)
    lo = np.array([0.1, -0.2, 0.3][:dim])
    vel = np.vstack([np.eye(dim), -np.eye(dim), [[0.6, -0.8, 0.3][:dim]]])
    prob = lib.Problem([_desc(dim=dim, n=list(n), degree=degree, v=vel, lo=list(lo), hi=[0.0] * dim, axes=axes)])
    m = omesh.Mesh(n, lo, None, degree, axes=axes)
    vol, inflow = prob.node_coords(0)
    np.testing.assert_allclose(np.transpose(vol, (2, 1, 0)), m.node_coords(), atol=1e-14)
    off = 0
    for v in range(vel.shape[0]):
        ent = otr.inflow_entries(m, vel[v])
        # one block [D][t][tau] per index axis along which A^{-1} v is non-zero
        vt = np.linalg.solve(axes, vel[v])
        blocks = []
        for a in range(dim):
            if vt[a] == 0:
                continue
            npts = (degree + 1) ** (dim - 1) * (m.nc // n[a])
            blocks.append(inflow[off:off + dim * npts].reshape(dim, npts).T)
            off += dim * npts
        pts = np.concatenate(blocks)
        a = pts[np.lexsort(np.round(pts, 12).T[::-1])]
        b = ent["coords"][np.lexsort(np.round(ent["coords"], 12).T[::-1])]
        np.testing.assert_allclose(a, b, atol=1e-14)
        lev = np.zeros(m.nc, np.int32)
        lib.pdg_levels(prob.ctx, 0, v, lev)
        assert np.array_equal(lev, otr.topological_levels(m, vel[v]))
    prob.close()


@pytest.mark.parametrize("dim,n,degree,axes", AFFINE)
@pytest.mark.parametrize("vel", [(1.0, 0.0, 0.0), (0.0, -1.0, 0.0), (0.7, 0.7, -0.2)])
def test_affine_cell_operator_is_the_oracle_block(lib, dim, n, degree, axes, vel):
    """The block of the index frame (velocity A^{-1} v on unit cells), in
    downwind-local order, equals the oracle's block of the affine cell."""
    axes = np.array(axes)
    v = np.array(vel[:dim])
    prob = lib.Problem([_desc(dim=dim, n=list(n), degree=degree, v=[list(v)], lo=[0.0] * dim, hi=[0.0] * dim,
                              axes=axes)])
    npn = degree + 1
    nd = npn ** dim
    gam = np.zeros(nd * nd)
    kap = np.zeros(3)
    lib.pdg_cell_operator(prob.ctx, 0, 0, gam, kap)
    m = omesh.Mesh(n, np.zeros(dim), None, degree, axes=axes)
    blk = otr.cell_blocks(m, v, np.array([1]))
    vt = np.linalg.solve(axes, v)
    idx = m.node_idx
    q = np.zeros(nd, dtype=np.int64)
    for i in range(nd):
        for a in range(dim):
            qa = idx[i, a] if vt[a] >= 0 else degree - idx[i, a]
            q[i] += qa * npn ** a
    np.testing.assert_allclose(gam.reshape(nd, nd)[np.ix_(q, q)], blk.gll[0], rtol=1e-12,
                               atol=1e-12 * np.abs(blk.gll[0]).max())
    for fc in blk.faces:
        a = fc["axis"]
        if vt[a] == 0 or fc["side"] != (-1 if vt[a] > 0 else 1):
            continue
        np.testing.assert_allclose(fc["coef"][0], -kap[a], rtol=1e-12)
    prob.close()


@pytest.mark.parametrize("kw", [
    dict(axes=[[0.0, 1.0], [1.0, 0.0]]),                         # negative determinant
    dict(axes=[[1.0, 2.0], [0.5, 1.0]]),                         # singular
    dict(axes=[[float("nan"), 0.0], [0.0, 1.0]]),
    dict(axes=[[1.0, 0.0], [0.0, 1.0]], edges=[[0.0, 0.5, 1.0, 2.0, 3.0], None]),   # with graded edges
])
def test_affine_lattice_is_validated(lib, kw):
    with pytest.raises(lib.PdgError) as ei:
        lib.pdg_setup_mesh([_desc(**kw)])
    assert ei.value.status == lib.PDG_EINVAL
