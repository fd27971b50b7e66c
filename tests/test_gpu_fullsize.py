"""Parity at the full workload sizes, in the launch configuration bench.py
times (autotuned tiles), on sampled outputs.

After one interior step (one sweep of every velocity + one relaxation) the
values at a cell L depend only on the cells of the lines through L along each
velocity axis (the sweep of an axis-aligned velocity couples a cell only to its
upwind neighbour on that line, Sec. 4.1) and on L itself (the relaxation is
node local).  So the oracle recomputes, for a few sampled cells, each
velocity's sweep on the one-cell-wide line mesh through L, then the
relaxation at L, from its own initial data.
"""
import numpy as np
import pytest

import workloads as W
from helpers import gpu_initial_state, inst_dict, sizes
from oracle import step as ost
from oracle import transport as otr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_1702_00169_amd as P
    return P


def _oracle_cell_after_step(inst, cm, dt, theta, omega):
    """Oracle state (nv, m, nd) at the cell with multi-index cm after one
    transport step of every velocity followed by one relaxation."""
    nv = inst.vel.shape[0]
    h = (inst.hi - inst.lo) / np.array(inst.n)
    _, nd = sizes(inst)
    out = np.zeros((nv, inst.m, nd))
    for v in range(nv):
        a = int(np.nonzero(inst.vel[v])[0][0])
        n_line = [1] * inst.dim
        n_line[a] = inst.n[a]
        lo = inst.lo + np.array(cm) * h
        hi = lo + h
        lo[a], hi[a] = inst.lo[a], inst.hi[a]
        prob = ost.Problem(n_line, lo, hi, inst.degree, inst.vel, inst.m, inst.feq_kind, inst.feq_param)
        x = prob.mesh.node_coords().reshape(-1, inst.dim)
        f0 = prob.feq(inst.w0(x).reshape(inst.m, prob.mesh.nc, prob.mesh.nd))
        ent = prob.entries(v)
        fb = prob.feq(inst.w0(ent["coords"]))[v]
        fv = otr.theta_step_sweep(prob.mesh, inst.vel[v], f0[v], fb, fb, dt, theta)
        out[v] = fv[:, cm[a], :]
    oprob = ost.Problem([1] * inst.dim, inst.lo, inst.hi, inst.degree, inst.vel, inst.m, inst.feq_kind,
                        inst.feq_param)
    return oprob.collide(out[:, :, None, :], omega)[:, :, 0, :]


def _sample_cells(inst, count, seed):
    rng = np.random.default_rng(seed)
    cells = [tuple(0 for _ in inst.n), tuple(k - 1 for k in inst.n)]
    while len(cells) < count:
        cells.append(tuple(int(rng.integers(0, k)) for k in inst.n))
    return cells


def _gpu_cell(f, off, inst, cm):
    nc, nd = sizes(inst)
    c = cm[0] + inst.n[0] * (cm[1] + (inst.n[1] * cm[2] if inst.dim == 3 else 0))
    nv = inst.vel.shape[0]
    idx = off + (np.arange(nv * inst.m * nd) * nc + c)
    import torch
    t = torch.as_tensor(idx, device=f.device)
    return f[t].double().cpu().numpy().reshape(nv, inst.m, nd)


CASES = [("adv2d_16", 0), ("adv3d_64", 0), ("euler2d_256", 0), ("euler2d_256", 2), ("euler3d_128", 0),
         ("euler3d_128", 2), ("batch96", 0), ("batch96", 2)]


@pytest.mark.parametrize("name,prec", CASES, ids=[f"{n}-{['fp64', 'fp32', 'fp32refine'][p]}" for n, p in CASES])
def test_one_step_at_full_size_sampled(lib, name, prec):
    torch = pytest.importorskip("torch")
    print(f"full-size {name} prec={prec}", flush=True)
    wl = W.make(name, seed=0)
    prob = lib.Problem([inst_dict(i) for i in wl.instances])
    prob.prepare(wl.dt, theta=wl.theta, omega=wl.omega, precision=prec)
    f, fb = gpu_initial_state(prob, wl.instances, torch, torch.float64)
    scratch = torch.zeros_like(f)
    tiles = prob.autotune(scratch, fb, reps=1)
    del scratch
    print(f"  tiles {tiles}", flush=True)
    prob.transport_sweep(f, fb, fb, wl.dt)
    prob.relax(f)
    torch.cuda.synchronize()
    picks = [0] if len(wl.instances) == 1 else [0, 17, 58, 95]
    worst = 0.0
    for i in picks:
        inst = wl.instances[i]
        for cm in _sample_cells(inst, 4, seed=i):
            got = _gpu_cell(f, prob.layout["f_off"][i], inst, cm)
            want = _oracle_cell_after_step(inst, cm, wl.dt, wl.theta, wl.omega)
            err = np.linalg.norm(got - want) / np.linalg.norm(want)
            worst = max(worst, err)
    print(f"  worst sampled rel L2 error {worst:.3e}")
    assert worst <= (1e-12 if prec == 0 else 1e-10)
    prob.close()
