"""Edge cases of the transport sweep on the GPU, against the oracle:
single-cell and one-cell-thick meshes (chains of length one, tiles with one
cell), the largest component count (m = 8) on the chain and dense paths, and
the time symmetry of the Crank-Nicolson transport step (Sec. 3.2,
eq. prop_sym: T_2(-dt) T_2(dt) = Id, also with inflow data)."""
import itertools

import numpy as np
import pytest

import workloads as W
from helpers import (gpu_fb_from_function, gpu_to_oracle, inst_dict, oracle_fb_from_function, oracle_problem,
                     oracle_to_gpu, rel_errors, sizes)
from oracle import transport as otr

pytestmark = pytest.mark.gpu

D2Q4, D3Q6 = W.D2Q4, W.D3Q6
D2Q9 = W.D2Q9
D3Q27 = np.array(list(itertools.product([0, 1, -1], repeat=3)), float)


@pytest.fixture(scope="module")
def lib():
    import paper_1702_00169_amd as P
    return P


def _instance(dim, n, degree, vel, m):
    inst = W.Instance(dim, n, degree, 1.0, m, "advection", {"a": [0.1] * dim}, W.uniform_state([1.0] * m),
                      vel=vel)
    inst.hi = np.array([1.0, 1.7, 0.6][:dim])
    return inst


def _sweep_vs_oracle(lib, torch, inst, prec, dt_scale=0.8, seed=0):
    prob = lib.Problem([inst_dict(inst)])
    nc, nd = sizes(inst)
    h = np.min((inst.hi - inst.lo) / np.array(inst.n))
    dt = dt_scale * h / max(1e-300, np.max(np.abs(inst.vel)))
    prob.prepare(dt, theta=0.5, omega=2.0, precision=prec)
    nv, m = inst.vel.shape[0], inst.m
    f_or = W.random_state(seed, (nv, m, nc, nd))
    if prec == 1:
        f_or = f_or.astype(np.float32).astype(np.float64)
    fo, fn = W.smooth_field(seed + 1, inst.dim, m), W.smooth_field(seed + 2, inst.dim, m)
    fbo = torch.tensor(gpu_fb_from_function(prob, [inst], lambda i, v, p: fo(p)), device="cuda")
    fbn = torch.tensor(gpu_fb_from_function(prob, [inst], lambda i, v, p: fn(p)), device="cuda")
    f = torch.tensor(oracle_to_gpu(f_or), dtype=torch.float32 if prec == 1 else torch.float64, device="cuda")
    prob.transport_sweep(f, fbo, fbn, dt)
    prob.sync_status()
    got = gpu_to_oracle(f.double().cpu().numpy(), inst)
    oprob = oracle_problem(inst)
    ofo = oracle_fb_from_function(oprob, 0, lambda i, v, p: fo(p))
    ofn = oracle_fb_from_function(oprob, 0, lambda i, v, p: fn(p))
    want = np.empty_like(f_or)
    for v in range(nv):
        want[v] = otr.theta_step_sweep(oprob.mesh, inst.vel[v], f_or[v], ofo[v], ofn[v], dt, 0.5,
                                       levels=oprob.levels(v))
    prob.close()
    return rel_errors(got, want)


BARS = {0: 1e-12, 2: 1e-10, 1: 1e-5}

THIN = [
    ("2d_1x1_d2_d2q4", 2, (1, 1), 2, D2Q4),
    ("2d_1x7_d3_d2q9", 2, (1, 7), 3, D2Q9),
    ("2d_9x1_d1_d2q9", 2, (9, 1), 1, D2Q9),
    ("3d_1x1x1_d2_d3q27", 3, (1, 1, 1), 2, D3Q27),
    ("3d_1x5x1_d1_d3q27", 3, (1, 5, 1), 1, D3Q27),
    ("3d_6x1x4_d2_d3q6", 3, (6, 1, 4), 2, D3Q6),
]


@pytest.mark.parametrize("case", THIN, ids=[c[0] for c in THIN])
@pytest.mark.parametrize("prec", [0, 2, 1], ids=["fp64", "fp32refine", "fp32"])
def test_single_cell_and_thin_meshes(lib, case, prec):
    torch = pytest.importorskip("torch")
    name, dim, n, degree, vel = case
    print(f"edge case={name} prec={prec}", flush=True)
    (l2, mx) = _sweep_vs_oracle(lib, torch, _instance(dim, n, degree, vel, 1), prec)
    print(f"  rel L2 {l2:.3e} max {mx:.3e}")
    assert l2 <= BARS[prec] and mx <= 10 * BARS[prec]


@pytest.mark.parametrize("vel,n,degree", [(D2Q4, (13, 9), 2), (D2Q9, (11, 6), 2), (D3Q27, (4, 5, 3), 1)],
                         ids=["chains_d2q4", "dense_d2q9", "dense_d3q27"])
def test_largest_component_count(lib, vel, n, degree):
    torch = pytest.importorskip("torch")
    print(f"edge m=8 n={n}", flush=True)
    (l2, mx) = _sweep_vs_oracle(lib, torch, _instance(len(n), n, degree, vel, 8), 0)
    assert l2 <= 1e-12 and mx <= 1e-11


@pytest.mark.parametrize("vel,n,degree", [(D2Q4, (6, 5), 2), (D2Q4, (5, 4), 3), (D2Q9, (4, 3), 2),
                                          (D3Q27, (3, 2, 3), 2), (D3Q27, (5, 4, 6), 1)],
                         ids=["chains_d2q4_d2", "chains_d2q4_d3", "dense_d2q9", "dense_d3q27_d2", "dense_d3q27_d1"])
def test_transport_is_time_symmetric(lib, vel, n, degree):
    """T_2(-dt) T_2(dt) = Id with the same inflow data (the inflow terms
    cancel): forward and backward sweeps return the initial state.  The
    backward (anti-dissipative) sweep amplifies rounding geometrically along
    a chain, so the meshes are short: on them the oracle's own round trip is
    below 1e-14."""
    torch = pytest.importorskip("torch")
    print(f"edge time symmetry n={n}", flush=True)
    inst = _instance(len(n), n, degree, vel, 2)
    h = np.min((inst.hi - inst.lo) / np.array(inst.n))
    dt = 0.25 * h
    nc, nd = sizes(inst)
    f0 = W.random_state(7, (vel.shape[0], 2, nc, nd))
    fbfn = W.smooth_field(8, inst.dim, 2)
    f = torch.tensor(oracle_to_gpu(f0), device="cuda")
    fwd = lib.Problem([inst_dict(inst)])
    fwd.prepare(dt, theta=0.5)
    bwd = lib.Problem([inst_dict(inst)])
    bwd.prepare(-dt, theta=0.5)
    fb = torch.tensor(gpu_fb_from_function(fwd, [inst], lambda i, v, p: fbfn(p)), device="cuda")
    fwd.transport_sweep(f, fb, fb, dt)
    fwd.sync_status()
    moved = rel_errors(gpu_to_oracle(f.cpu().numpy(), inst), f0)[0]
    bwd.transport_sweep(f, fb, fb, -dt)
    bwd.sync_status()
    back = rel_errors(gpu_to_oracle(f.cpu().numpy(), inst), f0)
    print(f"  moved by {moved:.3e}; back to {back[0]:.3e} (max {back[1]:.3e})")
    assert moved > 1e-3
    assert back[0] <= 1e-12 and back[1] <= 1e-11
    fwd.close()
    bwd.close()
