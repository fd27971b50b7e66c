"""GPU parity of the D2Q9 isothermal gravity model (Sec. 5.1): the lattice
equilibrium, the collision with moments through P, the source step S_2 of
Sec. 3.2, whole steps of the compositions with the source (dense transport
of the diagonal velocities included), and the hydrostatic run of the paper's
convergence test, against the oracle."""
import numpy as np
import pytest

import workloads as W
from helpers import (gpu_fb_from_function, gpu_initial_state, gpu_to_oracle, gpu_w_inflow_from_function,
                     inst_dict, oracle_initial_state, oracle_problem, oracle_to_gpu, rel_errors, sizes)
from oracle import step as ost

pytestmark = pytest.mark.gpu

PRECS = [0, 2, 1]
PREC_IDS = ["fp64", "fp32refine", "fp32"]


@pytest.fixture(scope="module")
def lib():
    import paper_1702_00169_amd as P
    return P


def _inst(n=(6, 5), degree=2, lam=1.3, g=0.8, bump=0.1):
    inst = W.gravity2d_instance(n[0], degree, lam=lam, g=g, bump=bump)
    inst.n = tuple(n)
    return inst


def _random_w(seed, inst):
    nc, nd = sizes(inst)
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, (nc, nd))
    u = rng.uniform(-0.2, 0.2, (2, nc, nd)) * inst.lam
    return np.stack([rho, rho * u[0], rho * u[1]])


def _random_f(seed, inst, oprob):
    nc, nd = sizes(inst)
    noise = 0.02 * np.random.default_rng(seed + 100).standard_normal((9, 1, nc, nd))
    return oprob.feq(_random_w(seed, inst)) + noise


def _dtype(torch, prec):
    return torch.float32 if prec == 1 else torch.float64


def _bar(prec, fp64=1e-13):
    return {0: fp64, 2: fp64, 1: 2e-6}[prec]


@pytest.mark.parametrize("prec", PRECS, ids=PREC_IDS)
def test_equilibrium_matches_oracle(lib, prec):
    torch = pytest.importorskip("torch")
    print(f"d2q9 equilibrium prec={prec}", flush=True)
    inst = _inst()
    prob = lib.Problem([inst_dict(inst)])
    prob.prepare(0.01, precision=prec)
    w = _random_w(1, inst)
    f = torch.empty(prob.layout["f_elems"], dtype=_dtype(torch, prec), device="cuda")
    prob.equilibrium(torch.tensor(np.transpose(w, (0, 2, 1)).ravel(), device="cuda"), f)
    torch.cuda.synchronize()
    got = gpu_to_oracle(f.double().cpu().numpy(), inst)
    want = oracle_problem(inst).feq(w)
    l2, mx = rel_errors(got, want)
    print(f"  rel L2 {l2:.3e} max {mx:.3e}")
    assert l2 <= _bar(prec, 1e-14) and mx <= 10 * _bar(prec, 1e-14)
    prob.close()


def test_inflow_equilibrium_matches_oracle(lib):
    torch = pytest.importorskip("torch")
    print("d2q9 inflow equilibrium", flush=True)
    inst = _inst()
    prob = lib.Problem([inst_dict(inst)])
    prob.prepare(0.01)
    oprob = oracle_problem(inst)
    w_in = gpu_w_inflow_from_function(prob, [inst], lambda i, v, pts: inst.w0(pts), 3)
    assert w_in.size == 3 * prob.layout["fb_elems"]
    fb = torch.empty(prob.layout["fb_elems"], dtype=torch.float64, device="cuda")
    prob.inflow_equilibrium(torch.tensor(w_in, device="cuda"), fb)
    torch.cuda.synchronize()
    want = gpu_fb_from_function(prob, [inst], lambda i, v, pts: oprob.feq(inst.w0(pts))[v])
    l2, mx = rel_errors(fb.cpu().numpy(), want)
    assert l2 <= 1e-14 and mx <= 1e-13
    prob.close()


@pytest.mark.parametrize("prec", PRECS, ids=PREC_IDS)
@pytest.mark.parametrize("omega", [1.6, 2.0])
def test_relax_matches_oracle(lib, prec, omega):
    torch = pytest.importorskip("torch")
    print(f"d2q9 relax prec={prec} omega={omega}", flush=True)
    inst = _inst()
    prob = lib.Problem([inst_dict(inst)])
    prob.prepare(0.01, omega=omega, precision=prec)
    oprob = oracle_problem(inst)
    f_or = _random_f(2, inst, oprob)
    if prec == 1:
        f_or = f_or.astype(np.float32).astype(np.float64)
    f = torch.tensor(oracle_to_gpu(f_or), dtype=_dtype(torch, prec), device="cuda")
    w_out = torch.zeros(prob.layout["w_elems"], dtype=torch.float64, device="cuda")
    prob.relax(f, w_out)
    torch.cuda.synchronize()
    got = gpu_to_oracle(f.double().cpu().numpy(), inst)
    l2, mx = rel_errors(got, oprob.collide(f_or, omega))
    wl2, wmx = rel_errors(np.transpose(w_out.cpu().numpy().reshape(3, -1, sizes(inst)[0]), (0, 2, 1)),
                          oprob.moments(f_or))
    print(f"  f rel L2 {l2:.3e} max {mx:.3e}; w rel L2 {wl2:.3e}")
    assert l2 <= _bar(prec) and mx <= 10 * _bar(prec)
    assert wl2 <= 1e-14 and wmx <= 1e-13


@pytest.mark.parametrize("prec", PRECS, ids=PREC_IDS)
def test_source_matches_oracle_and_inverts(lib, prec):
    torch = pytest.importorskip("torch")
    print(f"d2q9 source prec={prec}", flush=True)
    inst = _inst()
    prob = lib.Problem([inst_dict(inst)])
    prob.prepare(0.01, precision=prec)
    oprob = oracle_problem(inst)
    f_or = _random_f(3, inst, oprob)
    if prec == 1:
        f_or = f_or.astype(np.float32).astype(np.float64)
    f = torch.tensor(oracle_to_gpu(f_or), dtype=_dtype(torch, prec), device="cuda")
    h = 0.037
    prob.source(f, h)
    torch.cuda.synchronize()
    got = gpu_to_oracle(f.double().cpu().numpy(), inst)
    l2, mx = rel_errors(got, oprob.source(f_or, h))
    print(f"  rel L2 {l2:.3e} max {mx:.3e}")
    assert l2 <= _bar(prec) and mx <= 10 * _bar(prec)
    prob.source(f, -h)   # S(-h) S(h) = Id (Sec. 3.2)
    torch.cuda.synchronize()
    back = gpu_to_oracle(f.double().cpu().numpy(), inst)
    l2b, _ = rel_errors(back, f_or)
    assert l2b <= (1e-14 if prec != 1 else 1e-6)
    prob.source(f, 0.0)
    prob.close()


def test_source_leaves_instances_without_source_alone(lib):
    torch = pytest.importorskip("torch")
    inst = _inst()
    adv = W.make("adv2d_16", scale=5).instances[0]
    prob = lib.Problem([inst_dict(adv), inst_dict(inst)])
    prob.prepare(0.01)
    f = torch.rand(prob.layout["f_elems"], dtype=torch.float64, device="cuda") + 0.5
    g = f.clone()
    prob.source(f, 0.05)
    torch.cuda.synchronize()
    a = prob.layout["f_off"][1]
    assert torch.equal(f[:a], g[:a])
    assert not torch.equal(f[a:], g[a:])
    prob.close()


SCHEMES = [(0, 1.0, 1.0), (0, 0.5, 2.0), (1, 0.5, 2.0), (2, 0.5, 2.0), (3, 0.5, 1.6)]
SCHEME_IDS = ["lie_theta1", "lie", "strang", "collapsed", "kin"]


@pytest.mark.parametrize("scheme,theta,omega", SCHEMES, ids=SCHEME_IDS)
@pytest.mark.parametrize("prec", PRECS, ids=PREC_IDS)
def test_gravity_steps_match_oracle(lib, scheme, theta, omega, prec):
    torch = pytest.importorskip("torch")
    print(f"d2q9 steps scheme={scheme} theta={theta} omega={omega} prec={prec}", flush=True)
    inst = _inst()
    dt, steps = 0.02, 4
    prob = lib.Problem([inst_dict(inst)])
    prob.prepare(dt, theta=theta, omega=omega, scheme=scheme, precision=prec)
    f, fb = gpu_initial_state(prob, [inst], torch, _dtype(torch, prec))
    prob.step(f, fb, steps)
    prob.sync_status()
    got = gpu_to_oracle(f.double().cpu().numpy(), inst)
    oprob = oracle_problem(inst)
    f0, fb0 = oracle_initial_state(oprob, inst)
    want = ost.run(oprob, f0, fb0, dt, theta, omega, scheme, steps)
    l2, mx = rel_errors(got, want)
    print(f"  rel L2 {l2:.3e} max {mx:.3e}")
    bar = {0: 1e-12, 2: 1e-10, 1: 1e-5}[prec]
    assert l2 <= bar and mx <= 10 * bar
    prob.close()


def _hydro_gpu_and_oracle(lib, torch, nsteps, n=8, degree=4, scheme=1):
    lam, g, t_end = 1.0, 1.0, 0.12
    inst = W.gravity2d_instance(n, degree, lam=lam, g=g)
    dt = t_end / nsteps
    prob = lib.Problem([inst_dict(inst)])
    prob.prepare(dt, theta=0.5, omega=2.0, scheme=scheme)
    f, fb = gpu_initial_state(prob, [inst], torch, torch.float64)
    prob.step(f, fb, nsteps)
    prob.sync_status()
    oprob = oracle_problem(inst)
    got = oprob.moments(gpu_to_oracle(f.cpu().numpy(), inst))
    f0, fb0 = oracle_initial_state(oprob, inst)
    want = oprob.moments(ost.run(oprob, f0, fb0, dt, 0.5, 2.0, scheme, nsteps))
    x = oprob.mesh.node_coords().reshape(-1, 2)
    exact = inst.w0(x).reshape(3, oprob.mesh.nc, oprob.mesh.nd)
    prob.close()
    return got, want, exact


def test_hydrostatic_run_matches_oracle_and_converges_at_second_order(lib):
    """The paper's Euler-gravity convergence test (Sec. 5.1) with Strang M_2^s."""
    torch = pytest.importorskip("torch")
    errs = []
    for nsteps in (5, 10):
        print(f"d2q9 hydrostatic nsteps={nsteps}", flush=True)
        got, want, exact = _hydro_gpu_and_oracle(lib, torch, nsteps)
        l2, mx = rel_errors(got, want)
        assert l2 <= 1e-12 and mx <= 1e-11, (l2, mx)
        errs.append(np.linalg.norm(got - exact) / np.linalg.norm(exact))
    rate = np.log2(errs[0] / errs[1])
    print(f"  errors vs the steady state {errs}, rate {rate:.2f}")
    assert 1.8 <= rate <= 2.3


@pytest.mark.parametrize("schedule", ["level", "claim", "transfer"])
def test_gravity_graph_replay_equals_eager(lib, monkeypatch, schedule):
    """The captured step (dense tiles with their fill kernels, or the three
    launches of the transfer schedule; chains; the S C S node kernel) replays
    to the same bits as the eager launches."""
    torch = pytest.importorskip("torch")
    print(f"d2q9 graph replay schedule={schedule}", flush=True)
    monkeypatch.setenv("PDG_DENSE_SCHEDULE", schedule)
    inst = _inst(n=(24, 16) if schedule == "transfer" else (20, 13), degree=2)
    outs = []
    for no_graph in (False, True):
        if no_graph:
            monkeypatch.setenv("PDG_NO_GRAPH", "1")
        prob = lib.Problem([inst_dict(inst)])
        prob.prepare(0.02, scheme=2)
        f, fb = gpu_initial_state(prob, [inst], torch, torch.float64)
        prob.step(f, fb, 2)
        torch.cuda.synchronize()
        prob.step(f, fb, 4)
        prob.sync_status()
        outs.append(f.clone())
        prob.close()
    assert torch.equal(outs[0], outs[1])
