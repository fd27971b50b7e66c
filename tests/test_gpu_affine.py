"""GPU parity on uniform affine meshes (every cell the same parallelogram /
parallelepiped spanned by the lattice vectors a_k, Sec. 3.1 affine cell
maps): the transport sweep on the paper's velocity sets (a physical velocity
along a box axis can cross the lattice obliquely and take the dense path),
and whole time steps with the relaxation in physical velocity components,
against the oracle assembled on the physical cells."""
import itertools

import numpy as np
import pytest

import workloads as W
from helpers import (gpu_fb_from_function, gpu_initial_state, gpu_state, gpu_to_oracle, inst_dict,
                     oracle_fb_from_function, oracle_initial_state, oracle_problem, oracle_to_gpu, rel_errors,
                     sizes)
from oracle import step as ost
from oracle import transport as otr

pytestmark = pytest.mark.gpu

D2Q4 = np.array([[1, 0], [0, 1], [-1, 0], [0, -1]], float)
D2Q9 = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]], float)
D3Q6 = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 0, 0], [0, -1, 0], [0, 0, -1]], float)
D3Q27 = np.array(list(itertools.product([0, 1, -1], repeat=3)), float)


def _lattice(n, shear):
    """Columns a_k: cell edge vectors of a sheared unit-size domain."""
    n = np.asarray(n, float)
    dim = len(n)
    a = np.diag(1.0 / n)
    s = np.asarray(shear, float).reshape(dim, dim)
    return a + s / n[None, :]


CASES = [
    # name, n, degree, velocities, m, shear (added to the identity, columns scaled by 1/n)
    ("d2q4_12x9_d2", (12, 9), 2, D2Q4, 1, [[0.0, 0.35], [0.0, 0.2]]),
    ("d2q9_16x16_d2", (16, 16), 2, D2Q9, 1, [[0.0, 0.3], [-0.1, 0.1]]),
    ("d2q9_24x16_d3_m2", (24, 16), 3, D2Q9 * 0.8, 2, [[0.2, -0.25], [0.05, 0.0]]),
    ("d2q9_9x30_d1", (9, 30), 1, D2Q9, 1, [[0.0, 0.5], [0.0, 0.0]]),
    ("d2q9_32x24_d4", (32, 24), 4, D2Q9 * 1.2, 1, [[-0.1, 0.2], [0.1, 0.0]]),
    ("d3q6_7x6x5_d2", (7, 6, 5), 2, D3Q6, 1, [[0.0, 0.2, 0.1], [0.0, 0.0, -0.15], [0.0, 0.0, 0.1]]),
    ("d3q27_6x5x7_d1_m2", (6, 5, 7), 1, D3Q27 * 0.9, 2, [[0.1, 0.0, 0.2], [0.05, 0.0, 0.0], [0.0, -0.1, 0.0]]),
]
BARS = {0: 1e-12, 2: 1e-10, 3: 1e-10, 1: 2e-5}


@pytest.fixture(scope="module")
def lib():
    import paper_1702_00169_amd as P
    return P


def _instance(case):
    name, n, degree, vel, m, shear = case
    dim = len(n)
    inst = W.Instance(dim, n, degree, 1.0, m, "advection", {"a": [0.1] * dim}, W.uniform_state([1.0] * m))
    inst.vel = np.asarray(vel, float)
    inst.lo = np.array([0.2, -0.4, 0.1][:dim])
    inst.axes = _lattice(n, shear)
    return inst


def _cell_size(inst):
    return np.min(np.linalg.norm(inst.axes, axis=0))


@pytest.fixture(params=["level", "claim", "transfer"])
def schedule(request, monkeypatch):
    """Dense-tile schedule, read by the library at prepare (the transfer
    schedule applies to 2D meshes of full 8 x 8 tiles)."""
    monkeypatch.setenv("PDG_DENSE_SCHEDULE", request.param)
    return request.param


def _sweep(lib, torch, case, prec, theta=0.5, seed=0):
    inst = _instance(case)
    print(f"affine sweep case={case[0]} prec={prec} theta={theta}", flush=True)
    prob = lib.Problem([inst_dict(inst)])
    nc, nd = sizes(inst)
    dt = 0.77 * _cell_size(inst) / np.max(np.abs(inst.vel))
    prob.prepare(dt, theta=theta, omega=2.0, precision=prec)
    nv, m = inst.vel.shape[0], inst.m
    f_or = W.random_state(seed, (nv, m, nc, nd))
    if prec == 1:
        f_or = f_or.astype(np.float32).astype(np.float64)
    fo = W.smooth_field(seed + 1, inst.dim, m)
    fn = W.smooth_field(seed + 2, inst.dim, m)
    fbo = torch.tensor(gpu_fb_from_function(prob, [inst], lambda i, v, p: fo(p)), device="cuda")
    fbn = torch.tensor(gpu_fb_from_function(prob, [inst], lambda i, v, p: fn(p)), device="cuda")
    f = gpu_state(prob, torch, oracle_to_gpu(f_or))
    prob.transport_sweep(f, fbo, fbn, dt)
    prob.sync_status()
    got = gpu_to_oracle(prob.state_to_f64(f).cpu().numpy(), inst)
    oprob = oracle_problem(inst)
    ofo = oracle_fb_from_function(oprob, 0, lambda i, v, p: fo(p))
    ofn = oracle_fb_from_function(oprob, 0, lambda i, v, p: fn(p))
    want = np.empty_like(f_or)
    for v in range(nv):
        want[v] = otr.theta_step_sweep(oprob.mesh, inst.vel[v], f_or[v], ofo[v], ofn[v], dt, theta,
                                       levels=oprob.levels(v))
    per_v = [rel_errors(got[v], want[v])[0] for v in range(nv)]
    prob.close()
    return rel_errors(got, want), per_v


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", [0, 2, 3, 1], ids=["fp64", "fp32refine", "fp32refine48", "fp32"])
def test_affine_sweep_matches_oracle(lib, case, prec, schedule):
    torch = pytest.importorskip("torch")
    print(f"schedule={schedule}", flush=True)
    (l2, mx), per_v = _sweep(lib, torch, case, prec)
    print(f"  rel L2 {l2:.3e} max {mx:.3e}; worst velocity {max(per_v):.3e}")
    assert l2 <= BARS[prec] and mx <= 10 * BARS[prec] and max(per_v) <= 10 * BARS[prec]


@pytest.mark.parametrize("theta", [1.0, 0.6])
def test_affine_sweep_theta(lib, theta):
    torch = pytest.importorskip("torch")
    (l2, mx), _ = _sweep(lib, torch, CASES[2], 0, theta, seed=3)
    assert l2 <= 1e-12 and mx <= 1e-11


def _euler_lattice(dim, n, shear, degree, seed):
    rng = np.random.default_rng(seed)
    lo = np.array([-0.3, 0.1, 0.0][:dim])
    axes = _lattice(n, shear)
    centre = lo + axes @ (0.5 * np.array(n, float))
    if dim == 2:
        w0 = W.isentropic_vortex(centre + rng.uniform(-0.05, 0.05, 2), 0.15, 0.8)
        inst = W.Instance(2, n, degree, 3.0, 4, "euler", {"gamma": W.GAMMA}, w0)
    else:
        bump = W.gaussian_bump(0.1, centre + rng.uniform(-0.05, 0.05, 3), 30.0)
        w0 = W.euler_at_rest(lambda x: 1.0 + bump(x)[0], lambda x: 1.0 + 0.5 * bump(x)[0], 3)
        inst = W.Instance(3, n, degree, 3.0, 5, "euler", {"gamma": W.GAMMA}, w0)
    inst.lo = lo
    inst.axes = axes
    return inst


STEP_CASES = [
    ("euler2d_sheared", lambda s: _euler_lattice(2, (14, 11), [[0.0, 0.3], [0.0, 0.1]], 2, s)),
    ("euler2d_rotated", lambda s: _euler_lattice(2, (10, 12), [[0.1, -0.2], [0.25, 0.05]], 3, s)),
    ("euler3d_sheared", lambda s: _euler_lattice(3, (6, 5, 7), [[0.0, 0.2, 0.0], [0.0, 0.0, 0.15],
                                                               [0.0, 0.0, 0.0]], 1, s)),
]


@pytest.mark.parametrize("case", STEP_CASES, ids=[c[0] for c in STEP_CASES])
@pytest.mark.parametrize("prec", [0, 3], ids=["fp64", "fp32refine48"])
def test_affine_steps_match_oracle(lib, case, prec):
    """Collapsed Strang steps (Sec. 5.1) of the Euler kinetic model: the
    relaxation acts on the physical velocity components, transport on the
    lattice."""
    torch = pytest.importorskip("torch")
    name, make = case
    print(f"affine steps case={name} prec={prec}", flush=True)
    inst = make(0)
    dt = 0.6 * _cell_size(inst) / inst.lam
    prob = lib.Problem([inst_dict(inst)])
    prob.prepare(dt, theta=0.5, omega=1.8, scheme=2, precision=prec)
    f, fb = gpu_initial_state(prob, [inst], torch, None)
    prob.step(f, fb, 3)
    torch.cuda.synchronize()
    got = gpu_to_oracle(prob.state_to_f64(f).cpu().numpy(), inst)
    oprob = oracle_problem(inst)
    f0, fb0 = oracle_initial_state(oprob, inst)
    want = ost.run(oprob, f0, fb0, dt, 0.5, 1.8, 2, 3)
    l2, mx = rel_errors(got, want)
    print(f"  rel L2 {l2:.3e} max {mx:.3e}")
    prob.close()
    bar = BARS[prec]
    assert l2 <= bar and mx <= 10 * bar


def test_affine_mesh_with_identity_axes_equals_box_mesh(lib):
    """Axes a_k = h_k e_k give the box mesh [lo, lo + n h] cell for cell."""
    torch = pytest.importorskip("torch")
    inst = _instance(CASES[1])
    box = _instance(CASES[1])
    box.axes = None
    box.hi = box.lo + np.array(box.n, float) * 0.0625
    inst.axes = np.diag([0.0625, 0.0625])
    outs = []
    for i in (inst, box):
        prob = lib.Problem([inst_dict(i)])
        prob.prepare(0.01)
        nc, nd = sizes(i)
        f = torch.tensor(oracle_to_gpu(W.random_state(1, (i.vel.shape[0], i.m, nc, nd))), device="cuda")
        fb = torch.tensor(gpu_fb_from_function(prob, [i], lambda k, v, p: np.sin(p.sum(axis=1))[None]),
                          device="cuda")
        prob.transport_sweep(f, fb, fb, 0.01)
        prob.sync_status()
        outs.append(f.cpu().numpy())
        prob.close()
    np.testing.assert_allclose(outs[0], outs[1], rtol=1e-13, atol=1e-13)
