"""Parity at the full workload sizes, in the launch configuration bench.py
times (autotuned tiles), on sampled outputs.

After one interior step (one sweep of every velocity + one relaxation) the
values at a cell L depend only on the cells of the lines through L along each
velocity axis (the sweep of an axis-aligned velocity couples a cell only to its
upwind neighbour on that line, Sec. 4.1) and on L itself (the relaxation is
node local).  So the oracle recomputes, for a few sampled cells, each
velocity's sweep on the one-cell-wide line mesh through L, then the
relaxation at L, from its own initial data.

Transport alone is also compared on whole lines: for every velocity, every
cell and node of eight full lines of cells along its axis, chosen at the
boundaries of the work items of the tuned tiles (first and last chain of an
item, the first of the next one) and at the domain corners, so that the
segment combine inside and across workgroups and the row scan across waves
and 256-cell chunks are all on a compared line.
"""
import numpy as np
import pytest

import workloads as W
from helpers import gpu_initial_state, inst_dict, rel_errors, sizes
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
         ("euler3d_128", 2), ("euler3d_128", 3), ("batch96", 0), ("batch96", 2), ("batch96", 3)]
PREC_IDS = ["fp64", "fp32", "fp32refine", "fp32refine48"]


@pytest.mark.parametrize("name,prec", CASES, ids=[f"{n}-{PREC_IDS[p]}" for n, p in CASES])
def test_one_step_at_full_size_sampled(lib, name, prec):
    torch = pytest.importorskip("torch")
    print(f"full-size {name} prec={prec}", flush=True)
    wl = W.make(name, seed=0)
    prob = lib.Problem([inst_dict(i) for i in wl.instances])
    prob.prepare(wl.dt, theta=wl.theta, omega=wl.omega, precision=prec)
    f, fb = gpu_initial_state(prob, wl.instances, torch, None)
    scratch = torch.zeros_like(f)
    tiles = prob.autotune(scratch, fb, reps=1)
    del scratch
    print(f"  tiles {tiles}", flush=True)
    prob.transport_sweep(f, fb, fb, wl.dt)
    prob.relax(f)
    torch.cuda.synchronize()
    f = prob.state_to_f64(f)   # binary64 values on the device
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


def _line_positions(inst, v, tiles, seed):
    """Eight transverse cell positions (tuple per axis, the velocity axis
    marked None) of lines along velocity v's axis: item boundaries of the
    tile of v's launch class, the corners and random ones."""
    a = int(np.nonzero(inst.vel[v])[0][0])
    others = [k for k in range(inst.dim) if k != a]
    ntrans = int(np.prod([inst.n[k] for k in others]))
    x_kind = 1 if a == 0 else 0
    C = [t["C"] for t in tiles if t["np"] == inst.degree + 1 and t["x_kind"] == x_kind][0]
    taus = [0, C - 1, C, 2 * C - 1, 2 * C, ntrans - 1]
    rng = np.random.default_rng(seed)
    taus += [int(rng.integers(0, ntrans)) for _ in range(2)]
    out = []
    for tau in taus:
        tau = min(tau, ntrans - 1)
        cm = [None] * inst.dim
        rem = tau
        for k in others:
            cm[k] = rem % inst.n[k]
            rem //= inst.n[k]
        out.append(tuple(cm))
    return a, out


def _oracle_line_sweep(inst, v, a, cm, dt, theta):
    """Oracle sweep of velocity v on the one-cell-wide line mesh through the
    transverse position cm: (m, n_a, nd), cells in increasing coordinate."""
    h = (inst.hi - inst.lo) / np.array(inst.n)
    n_line = [1] * inst.dim
    n_line[a] = inst.n[a]
    lo = inst.lo + np.array([c if c is not None else 0 for c in cm]) * h
    hi = lo + h
    lo[a], hi[a] = inst.lo[a], inst.hi[a]
    prob = ost.Problem(n_line, lo, hi, inst.degree, inst.vel, inst.m, inst.feq_kind, inst.feq_param)
    x = prob.mesh.node_coords().reshape(-1, inst.dim)
    f0 = prob.feq(inst.w0(x).reshape(-1, prob.mesh.nc, prob.mesh.nd))
    fb = prob.feq(inst.w0(prob.entries(v)["coords"]))[v]
    return otr.theta_step_sweep(prob.mesh, inst.vel[v], f0[v], fb, fb, dt, theta)


def _gpu_line(fvals, off, inst, v, a, cm):
    """GPU values (m, n_a, nd) of velocity v on the cells of the line."""
    nc, nd = sizes(inst)
    cells = []
    for p in range(inst.n[a]):
        c3 = [cm[k] if k != a else p for k in range(inst.dim)] + [0] * (3 - inst.dim)
        cells.append(c3[0] + inst.n[0] * (c3[1] + inst.n[1] * c3[2]))
    import torch
    cells = torch.as_tensor(np.array(cells), device=fvals.device)
    blk = fvals[off + v * inst.m * nd * nc: off + (v + 1) * inst.m * nd * nc].reshape(inst.m, nd, nc)
    return np.transpose(blk[:, :, cells].cpu().numpy(), (0, 2, 1))


LINE_CASES = [("adv3d_64", 0), ("adv3d_64", 3), ("euler3d_128", 0), ("euler3d_128", 2), ("euler3d_128", 3),
              ("batch96", 0), ("batch96", 3)]


@pytest.mark.parametrize("name,prec", LINE_CASES,
                         ids=[f"{n}-{PREC_IDS[p]}" for n, p in LINE_CASES])
def test_transport_on_whole_lines_at_full_size(lib, name, prec):
    torch = pytest.importorskip("torch")
    print(f"full-size lines {name} prec={prec}", flush=True)
    wl = W.make(name, seed=0)
    prob = lib.Problem([inst_dict(i) for i in wl.instances])
    prob.prepare(wl.dt, theta=wl.theta, omega=wl.omega, precision=prec)
    f, fb = gpu_initial_state(prob, wl.instances, torch, None)
    scratch = prob.new_state()
    tiles = prob.autotune(scratch, fb, reps=1)
    del scratch
    print(f"  tiles {tiles}", flush=True)
    prob.transport_sweep(f, fb, fb, wl.dt)
    prob.sync_status()
    fvals = prob.state_to_f64(f)   # binary64 values on the device
    del f
    # batch: the instances whose rows do not fill whole 256-cell chunks
    picks = [0] if len(wl.instances) == 1 else [i for i, ins in enumerate(wl.instances) if 256 % ins.n[0]][:4]
    worst = 0.0
    bar = 1e-12 if prec == 0 else 1e-10
    for i in picks:
        inst = wl.instances[i]
        for v in range(inst.vel.shape[0]):
            a, lines = _line_positions(inst, v, tiles, seed=10 * i + v)
            for cm in lines:
                got = _gpu_line(fvals, prob.layout["f_off"][i], inst, v, a, cm)
                want = _oracle_line_sweep(inst, v, a, cm, wl.dt, wl.theta)
                err = rel_errors(got, want)
                worst = max(worst, err[0])
                assert err[0] <= bar and err[1] <= 10 * bar, (i, v, cm, err)
    print(f"  worst line rel L2 error {worst:.3e} over {len(picks)} instance(s)")
    prob.close()
