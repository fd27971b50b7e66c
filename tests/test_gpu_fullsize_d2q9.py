"""Parity of the D2Q9 Euler-gravity workload (Sec. 5.1) at its full size
(256^2 cells, degree 3), in the launch configuration bench.py times.

Transport: after one sweep, the values of a cell depend only on the cells of
its upwind cone (Sec. 4.1): for a velocity with non-negative components the
cells at or below-left of it.  So a square sub-mesh of S x S cells at the
inflow corner of a velocity, with the same initial data and the same inflow
data on its two domain faces, has exactly the full-domain solution on its
cells.  The oracle solves that sub-mesh for every velocity and the GPU's
full-domain sweep is compared there (the dense tiled sweep for the four
diagonal velocities, the chain kernel for the four axis velocities, the
identity for the rest velocity).

Node-local step: S(dt/2) C S(dt/2) is compared on every node.
"""
import numpy as np
import pytest

import workloads as W
from helpers import gpu_initial_state, gpu_to_oracle, inst_dict, oracle_to_gpu, rel_errors, sizes
from oracle import step as ost
from oracle import transport as otr

pytestmark = pytest.mark.gpu

S = 16   # sub-mesh cells per axis at each inflow corner


@pytest.fixture(scope="module")
def lib():
    import paper_1702_00169_amd as P
    return P


def _corner_block(inst, v):
    """(first cell index per axis, physical box) of the S x S block at the
    inflow corner of velocity v."""
    n = np.array(inst.n)
    h = (inst.hi - inst.lo) / n
    first = np.array([0 if inst.vel[v][a] >= 0 else n[a] - S for a in range(inst.dim)])
    lo = inst.lo + first * h
    return first, lo, lo + S * h


def _oracle_corner(inst, v, dt_sub, theta):
    first, lo, hi = _corner_block(inst, v)
    prob = ost.Problem((S, S), lo, hi, inst.degree, inst.vel, inst.m, inst.feq_kind, inst.feq_param)
    x = prob.mesh.node_coords().reshape(-1, inst.dim)
    f0 = prob.feq(inst.w0(x).reshape(-1, prob.mesh.nc, prob.mesh.nd))
    fb = prob.feq(inst.w0(prob.entries(v)["coords"]))[v]
    return first, otr.theta_step_sweep(prob.mesh, inst.vel[v], f0[v], fb, fb, dt_sub, theta, levels=prob.levels(v))


@pytest.mark.parametrize("prec", [0, 2], ids=["fp64", "fp32refine"])
def test_gravity2d_256_sweep_on_corner_blocks(lib, prec):
    torch = pytest.importorskip("torch")
    wl = W.make("gravity2d_256")
    inst = wl.instances[0]
    print(f"gravity2d_256 full-size sweep prec={prec}", flush=True)
    prob = lib.Problem([inst_dict(inst)])
    prob.prepare(wl.dt, theta=wl.theta, omega=wl.omega, scheme=lib.PDG_STRANG_COLLAPSED, precision=prec)
    f, fb = gpu_initial_state(prob, [inst], torch, torch.float64)
    dt_sub = wl.dt / 2
    prob.transport_sweep(f, fb, fb, dt_sub)
    prob.sync_status()
    got = gpu_to_oracle(f.cpu().numpy(), inst)          # (9, 1, nc, nd)
    n = inst.n[0]
    worst = 0.0
    for v in range(inst.vel.shape[0]):
        first, want = _oracle_corner(inst, v, dt_sub, wl.theta)   # (1, S*S, nd)
        ix = first[0] + np.arange(S)
        iy = first[1] + np.arange(S)
        cells = (ix[None, :] + n * iy[:, None]).ravel()            # sub-mesh order: x fastest
        l2, mx = rel_errors(got[v][:, cells, :], want)
        worst = max(worst, l2)
        print(f"  velocity {inst.vel[v]}: rel L2 {l2:.3e} max {mx:.3e}")
        bar = 1e-12 if prec == 0 else 1e-10
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
