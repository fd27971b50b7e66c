"""GPU parity on tensor-product graded meshes (box cells whose size varies
along each axis; the affine cell maps of Sec. 3.1 with per-cell Jacobians):
the transport sweep of axis-aligned velocities, whose cell operator then
changes from cell to cell along a chain, whole time steps, and a batch that
mixes graded and uniform instances, against the oracle."""
import numpy as np
import pytest

import workloads as W
from helpers import (gpu_fb_from_function, gpu_initial_state, gpu_to_oracle, inst_dict, oracle_fb_from_function,
                     oracle_initial_state, oracle_problem, oracle_to_gpu, rel_errors, sizes)
from oracle import step as ost
from oracle import transport as otr

pytestmark = pytest.mark.gpu

BARS = {0: 1e-12, 2: 1e-10, 1: 1e-5}


@pytest.fixture(scope="module")
def lib():
    import paper_1702_00169_amd as P
    return P


def _graded(inst, axes, stretch=1.4, jitter=0.25):
    inst.edges = [W.graded_edges(inst.n[k], inst.lo[k], inst.hi[k], stretch, jitter, seed=11 + k) if k in axes
                  else None for k in range(inst.dim)]
    return inst


CASES = [
    # name, dim, n, degree, lambda, m, graded axes
    ("2d_24x17_d2_x", 2, (24, 17), 2, 1.0, 1, (0,)),
    ("2d_19x30_d3_y_m3", 2, (19, 30), 3, 3.0, 3, (1,)),
    ("2d_40x9_d1_xy", 2, (40, 9), 1, 1.0, 2, (0, 1)),
    ("2d_7x11_d4_xy", 2, (7, 11), 4, 1.0, 1, (0, 1)),
    ("3d_9x7x6_d2_xyz", 3, (9, 7, 6), 2, 1.0, 1, (0, 1, 2)),
    ("3d_5x6x8_d3_z_m2", 3, (5, 6, 8), 3, 3.0, 2, (2,)),
]


def _instance(case):
    name, dim, n, degree, lam, m, axes = case
    inst = W.Instance(dim, n, degree, lam, m, "advection", {"a": [0.1] * dim}, W.uniform_state([1.0] * m))
    inst.hi = np.array([1.0, 1.7, 0.6][:dim])
    return _graded(inst, axes)


def _sweep(lib, torch, inst, prec, theta, half, seed=0):
    prob = lib.Problem([inst_dict(inst)])
    nc, nd = sizes(inst)
    h = min(np.min(np.diff(e)) if e is not None else (inst.hi[k] - inst.lo[k]) / inst.n[k]
            for k, e in enumerate(inst.edges))
    dt = 0.83 * h / inst.lam
    prob.prepare(dt, theta=theta, omega=2.0, precision=prec)
    nv, m = inst.vel.shape[0], inst.m
    f_or = W.random_state(seed, (nv, m, nc, nd))
    if prec == 1:
        f_or = f_or.astype(np.float32).astype(np.float64)
    fo, fn = W.smooth_field(seed + 1, inst.dim, m), W.smooth_field(seed + 2, inst.dim, m)
    fbo = torch.tensor(gpu_fb_from_function(prob, [inst], lambda i, v, p: fo(p)), device="cuda")
    fbn = torch.tensor(gpu_fb_from_function(prob, [inst], lambda i, v, p: fn(p)), device="cuda")
    f = torch.tensor(oracle_to_gpu(f_or), dtype=torch.float32 if prec == 1 else torch.float64, device="cuda")
    dsub = 0.5 * dt if half else dt
    prob.transport_sweep(f, fbo, fbn, dsub)
    prob.sync_status()
    got = gpu_to_oracle(f.double().cpu().numpy(), inst)
    oprob = oracle_problem(inst)
    ofo = oracle_fb_from_function(oprob, 0, lambda i, v, p: fo(p))
    ofn = oracle_fb_from_function(oprob, 0, lambda i, v, p: fn(p))
    want = np.empty_like(f_or)
    for v in range(nv):
        want[v] = otr.theta_step_sweep(oprob.mesh, inst.vel[v], f_or[v], ofo[v], ofn[v], dsub, theta,
                                       levels=oprob.levels(v))
    prob.close()
    return rel_errors(got, want)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", [0, 2, 1], ids=["fp64", "fp32refine", "fp32"])
def test_graded_sweep_matches_oracle(lib, case, prec):
    torch = pytest.importorskip("torch")
    print(f"graded sweep case={case[0]} prec={prec}", flush=True)
    l2, mx = _sweep(lib, torch, _instance(case), prec, 0.5, False)
    print(f"  rel L2 {l2:.3e} max {mx:.3e}")
    assert l2 <= BARS[prec] and mx <= 10 * BARS[prec]


@pytest.mark.parametrize("theta,half", [(1.0, False), (0.5, True), (0.7, True)])
def test_graded_sweep_theta_and_half_step(lib, theta, half):
    torch = pytest.importorskip("torch")
    print(f"graded sweep theta={theta} half={half}", flush=True)
    l2, mx = _sweep(lib, torch, _instance(CASES[1]), 0, theta, half, seed=3)
    assert l2 <= 1e-12 and mx <= 1e-11


def _euler_graded(n, degree, axes):
    wl = W.make("euler2d_256", scale=n)
    inst = wl.instances[0]
    inst.degree = degree
    return _graded(inst, axes, stretch=1.0, jitter=0.2), wl


@pytest.mark.parametrize("scheme", [2, 3], ids=["collapsed", "kin"])
@pytest.mark.parametrize("prec", [0, 2], ids=["fp64", "fp32refine"])
def test_graded_euler_steps_match_oracle(lib, scheme, prec):
    torch = pytest.importorskip("torch")
    print(f"graded euler steps scheme={scheme} prec={prec}", flush=True)
    inst, wl = _euler_graded(14, 2, (0, 1))
    steps = 3
    prob = lib.Problem([inst_dict(inst)])
    prob.prepare(wl.dt, theta=wl.theta, omega=wl.omega, scheme=scheme, precision=prec)
    f, fb = gpu_initial_state(prob, [inst], torch, torch.float64)
    prob.step(f, fb, steps)
    prob.sync_status()
    got = gpu_to_oracle(f.cpu().numpy(), inst)
    oprob = oracle_problem(inst)
    f0, fb0 = oracle_initial_state(oprob, inst)
    want = ost.run(oprob, f0, fb0, wl.dt, wl.theta, wl.omega, scheme, steps)
    l2, mx = rel_errors(got, want)
    print(f"  rel L2 {l2:.3e} max {mx:.3e}")
    bar = 1e-12 if prec == 0 else 1e-10
    assert l2 <= bar and mx <= 10 * bar
    prob.close()


def test_batch_mixing_graded_and_uniform_instances(lib):
    torch = pytest.importorskip("torch")
    print("graded + uniform batch", flush=True)
    rng = np.random.default_rng(4)
    insts = []
    for n, d, axes in [(21, 2, (0,)), (13, 3, ()), (30, 1, (0, 1)), (9, 4, (1,))]:
        inst = W.adv2d_instance(rng, n, d, rng.uniform(-0.4, 0.4, 2))
        insts.append(_graded(inst, axes) if axes else inst)
    dt, steps = 0.01, 3
    prob = lib.Problem([inst_dict(i) for i in insts])
    prob.prepare(dt, theta=0.5, omega=2.0, scheme=2)
    f, fb = gpu_initial_state(prob, insts, torch, torch.float64)
    prob.step(f, fb, steps)
    prob.sync_status()
    out = f.cpu().numpy()
    for i, inst in enumerate(insts):
        got = gpu_to_oracle(out, inst, prob.layout["f_off"][i])
        oprob = oracle_problem(inst)
        f0, fb0 = oracle_initial_state(oprob, inst)
        want = ost.run(oprob, f0, fb0, dt, 0.5, 2.0, 2, steps)
        l2, mx = rel_errors(got, want)
        print(f"  instance {i}: rel L2 {l2:.3e}")
        assert l2 <= 1e-12 and mx <= 1e-11
    prob.close()


def test_graded_autotune_and_tiles(lib):
    """Graded chains are tuned like strided chains (class kind 2); any valid
    tile solves the same system, up to the rounding of the segment combine."""
    torch = pytest.importorskip("torch")
    print("graded autotune", flush=True)
    inst = _instance(CASES[4])
    prob = lib.Problem([inst_dict(inst)])
    prob.prepare(0.02)
    scratch = torch.zeros(prob.layout["f_elems"], dtype=torch.float64, device="cuda")
    fb = torch.ones(prob.layout["fb_elems"], dtype=torch.float64, device="cuda")
    tiles = prob.autotune(scratch, fb, reps=1)
    assert {(t["np"], t["x_kind"]) for t in tiles} == {(3, 2)}
    results = []
    f0 = torch.tensor(W.random_state(5, (prob.layout["f_elems"],)), device="cuda")
    for C, S in [(64, 4), (16, 1), (8, 2)]:
        prob.set_tiles([dict(np=3, x_kind=2, C=C, S=S)])
        f = f0.clone()
        prob.transport_sweep(f, fb, fb, 0.02)
        prob.sync_status()
        results.append(f.cpu().numpy())
    with pytest.raises(lib.PdgError):
        prob.set_tiles([dict(np=3, x_kind=2, C=64, S=8)])     # longer than a graded segment
    for r in results[1:]:
        assert rel_errors(r, results[0])[0] <= 1e-14
    prob.close()


def test_graded_graph_replay_equals_eager(lib, monkeypatch):
    torch = pytest.importorskip("torch")
    print("graded graph replay", flush=True)
    inst, wl = _euler_graded(12, 2, (0, 1))
    outs = []
    for no_graph in (False, True):
        if no_graph:
            monkeypatch.setenv("PDG_NO_GRAPH", "1")
        prob = lib.Problem([inst_dict(inst)])
        prob.prepare(wl.dt)
        f, fb = gpu_initial_state(prob, [inst], torch, torch.float64)
        prob.step(f, fb, 2)
        torch.cuda.synchronize()
        prob.step(f, fb, 4)
        torch.cuda.synchronize()
        outs.append(f.clone())
        prob.close()
    assert torch.equal(outs[0], outs[1])
