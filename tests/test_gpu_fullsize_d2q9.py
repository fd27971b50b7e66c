"""Parity of the D2Q9 Euler-gravity workload (Sec. 5.1) at its full size
(256^2 cells, degree 3), in the launch configuration bench.py times.

Transport: one sweep of every velocity on the whole domain is compared with
the oracle's level sweep of the whole domain, cell by cell: the dense tiled
sweep of the four diagonal velocities (1024 tiles each, under the transfer
schedule that the library picks for this mesh, the claimed schedule that
hands traces between running tiles, and the levelled one), the chain kernel of the four axis velocities and the identity of the
rest velocity.

Node-local step: S(dt/2) C S(dt/2) is compared on every node.
"""
import numpy as np
import pytest

import workloads as W
from helpers import (gpu_initial_state, gpu_state_values, gpu_to_oracle, inst_dict, oracle_initial_state,
                     oracle_problem, oracle_to_gpu, rel_errors, sizes)
from oracle import step as ost
from oracle import transport as otr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_1702_00169_amd as P
    return P


@pytest.fixture(scope="module")
def oracle_sweep():
    """The oracle's sweep T(dt/2) of every velocity from f = f^eq(w0) on the
    whole 256^2 mesh (oracle layout (9, 1, nc, nd))."""
    wl = W.make("gravity2d_256")
    inst = wl.instances[0]
    oprob = oracle_problem(inst)
    f0, fb = oracle_initial_state(oprob, inst)
    out = np.empty_like(f0)
    for v in range(inst.vel.shape[0]):
        out[v] = otr.theta_step_sweep(oprob.mesh, inst.vel[v], f0[v], fb[v], fb[v], wl.dt / 2, wl.theta,
                                      levels=oprob.levels(v))
    return out


@pytest.mark.parametrize("prec,schedule", [(0, "transfer"), (2, "transfer"), (3, "transfer"), (1, "transfer"),
                                           (0, "claim"), (3, "claim"), (0, "level")],
                         ids=["fp64-transfer", "fp32refine-transfer", "fp32refine48-transfer", "fp32-transfer",
                              "fp64-claim", "fp32refine48-claim", "fp64-level"])
def test_gravity2d_256_whole_domain_sweep(lib, oracle_sweep, monkeypatch, prec, schedule):
    torch = pytest.importorskip("torch")
    monkeypatch.setenv("PDG_DENSE_SCHEDULE", schedule)
    wl = W.make("gravity2d_256")
    inst = wl.instances[0]
    print(f"gravity2d_256 whole-domain sweep prec={prec} schedule={schedule}", flush=True)
    prob = lib.Problem([inst_dict(inst)])
    prob.prepare(wl.dt, theta=wl.theta, omega=wl.omega, scheme=lib.PDG_STRANG_COLLAPSED, precision=prec)
    f, fb = gpu_initial_state(prob, [inst], torch, None)
    prob.transport_sweep(f, fb, fb, wl.dt / 2)
    prob.sync_status()
    got = gpu_to_oracle(gpu_state_values(prob, f), inst)     # (9, 1, nc, nd)
    bar = {0: 1e-12, 1: 2e-5, 2: 1e-10, 3: 1e-10}[prec]
    for v in range(inst.vel.shape[0]):
        l2, mx = rel_errors(got[v], oracle_sweep[v])
        print(f"  velocity {inst.vel[v]}: rel L2 {l2:.3e} max {mx:.3e}")
        assert l2 <= bar and mx <= 10 * bar, (v, l2, mx)
    prob.close()


@pytest.mark.parametrize("prec", [0, 2, 1], ids=["fp64", "fp32refine", "fp32"])
def test_gravity2d_256_local_step_on_every_node(lib, prec):
    torch = pytest.importorskip("torch")
    wl = W.make("gravity2d_256")
    inst = wl.instances[0]
    print(f"gravity2d_256 full-size S C S prec={prec}", flush=True)
    oprob = ost.Problem(inst.n, inst.lo, inst.hi, inst.degree, inst.vel, inst.m, inst.feq_kind, inst.feq_param)
    nc, nd = sizes(inst)
    rng = np.random.default_rng(9)
    x = oprob.mesh.node_coords().reshape(-1, 2)
    f_or = oprob.feq(inst.w0(x).reshape(3, nc, nd)) * (1.0 + 0.01 * rng.standard_normal((9, 1, nc, nd)))
    if prec == 1:
        f_or = f_or.astype(np.float32).astype(np.float64)
    prob = lib.Problem([inst_dict(inst)])
    prob.prepare(wl.dt, theta=wl.theta, omega=1.7, precision=prec)
    f = torch.tensor(oracle_to_gpu(f_or), dtype=torch.float32 if prec == 1 else torch.float64, device="cuda")
    h = wl.dt / 2
    prob.source(f, h)
    prob.relax(f)
    prob.source(f, h)
    torch.cuda.synchronize()
    got = gpu_to_oracle(f.double().cpu().numpy(), inst)
    want = oprob.local(f_or, h, 1.7, h)
    l2, mx = rel_errors(got, want)
    print(f"  rel L2 {l2:.3e} max {mx:.3e}")
    bar = {0: 1e-13, 2: 1e-13, 1: 2e-6}[prec]
    assert l2 <= bar and mx <= 10 * bar
    prob.close()
