"""GPU parity of one transport sweep (Sec. 4.1-4.2, eq. transport_cn) with
the oracle's level sweep, on seeded arbitrary states.

Bars: binary64 path <= 1e-12 relative (L2 and max), binary32 + binary64
refinement <= 1e-10, plain binary32 reported and held to 1e-5.
"""
import numpy as np
import pytest

import workloads as W
from helpers import (gpu_fb_from_function, gpu_to_oracle, inst_dict, oracle_fb_from_function, oracle_problem,
                     oracle_to_gpu, rel_errors, sizes)
from oracle import transport as otr

pytestmark = pytest.mark.gpu

CASES = [
    # name, dim, n, degree, lambda, m
    ("2d_16x16_d2", 2, (16, 16), 2, 1.0, 1),
    ("2d_37x23_d3_m4", 2, (37, 23), 3, 3.0, 4),
    ("2d_70x130_d1_m2", 2, (70, 130), 1, 1.0, 2),
    ("2d_300x5_d4", 2, (300, 5), 4, 1.0, 1),
    ("3d_9x7x13_d2", 3, (9, 7, 13), 2, 1.0, 1),
    ("3d_5x6x7_d3_m5", 3, (5, 6, 7), 3, 3.0, 5),
    ("3d_17x3x33_d4_m2", 3, (17, 3, 33), 4, 1.0, 2),
]
BARS = {0: 1e-12, 2: 1e-10, 1: 1e-5}


@pytest.fixture(scope="module")
def lib():
    import paper_1702_00169_amd as P  # raises if the HIP library is missing
    return P


def _instance(case):
    name, dim, n, degree, lam, m = case
    inst = W.Instance(dim, n, degree, lam, m, "advection", {"a": [0.1] * dim}, W.uniform_state([1.0] * m))
    # non-unit box to exercise anisotropic cells
    inst.hi = np.array([1.0, 1.7, 0.6][:dim])
    return inst


def _run_case(lib, torch, case, prec, theta, half, seed=0, tiles=None, autotune=False):
    """One sweep on a random state against the oracle; tiles: apply these
    tiles before the sweep; autotune: tune on this context first (the tuned
    tiles are returned with the errors)."""
    inst = _instance(case)
    print(f"sweep case={case[0]} prec={prec} theta={theta} half={half}", flush=True)
    prob = lib.Problem([inst_dict(inst)])
    nc, nd = sizes(inst)
    h = np.min((inst.hi - inst.lo) / np.array(inst.n))
    dt = 0.83 * h / inst.lam
    prob.prepare(dt, theta=theta, omega=2.0, precision=prec)
    if tiles is not None:
        prob.set_tiles(tiles)
    nv, m = inst.vel.shape[0], inst.m
    f_or = W.random_state(seed, (nv, m, nc, nd))
    if prec == lib.PDG_FP32:
        f_or = f_or.astype(np.float32).astype(np.float64)
    fb_old_fn = W.smooth_field(seed + 1, inst.dim, m)
    fb_new_fn = W.smooth_field(seed + 2, inst.dim, m)
    fbo = gpu_fb_from_function(prob, [inst], lambda i, v, p: fb_old_fn(p))
    fbn = gpu_fb_from_function(prob, [inst], lambda i, v, p: fb_new_fn(p))
    dtype = torch.float32 if prec == lib.PDG_FP32 else torch.float64
    f = torch.tensor(oracle_to_gpu(f_or), dtype=dtype, device="cuda")
    fbo_t = torch.tensor(fbo, device="cuda")
    fbn_t = torch.tensor(fbn, device="cuda")
    dsub = 0.5 * dt if half else dt
    if autotune:
        tiles = prob.autotune(torch.zeros_like(f), fbo_t, reps=1)
    used = prob.tiles()
    prob.transport_sweep(f, fbo_t, fbn_t, dsub)
    torch.cuda.synchronize()
    got = gpu_to_oracle(f.double().cpu().numpy(), inst)
    oprob = oracle_problem(inst)
    want = np.empty_like(f_or)
    ofbo = oracle_fb_from_function(oprob, 0, lambda i, v, p: fb_old_fn(p))
    ofbn = oracle_fb_from_function(oprob, 0, lambda i, v, p: fb_new_fn(p))
    for v in range(nv):
        want[v] = otr.theta_step_sweep(oprob.mesh, inst.vel[v], f_or[v], ofbo[v], ofbn[v], dsub, theta,
                                       levels=oprob.levels(v))
    corr = prob.last_refine_correction() if prec == lib.PDG_FP32_REFINE else None
    prob.close()
    if autotune or tiles is not None:
        return rel_errors(got, want), corr, used
    return rel_errors(got, want), corr


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", [0, 2, 1], ids=["fp64", "fp32refine", "fp32"])
def test_sweep_matches_oracle(lib, case, prec):
    torch = pytest.importorskip("torch")
    (l2, mx), corr = _run_case(lib, torch, case, prec, 0.5, False)
    print(f"  rel L2 {l2:.3e}  rel max {mx:.3e}  refine correction {corr}")
    assert l2 <= BARS[prec] and mx <= BARS[prec] * 10


@pytest.mark.parametrize("case", [CASES[1], CASES[5]], ids=[CASES[1][0], CASES[5][0]])
@pytest.mark.parametrize("theta,half", [(1.0, False), (0.5, True), (0.7, True)])
def test_sweep_theta_and_half_step(lib, case, theta, half):
    torch = pytest.importorskip("torch")
    (l2, mx), _ = _run_case(lib, torch, case, 0, theta, half, seed=3)
    assert l2 <= 1e-12 and mx <= 1e-11


def test_sweep_tile_shapes_agree(lib, monkeypatch):
    """Every tile shape solves the same block-triangular system."""
    torch = pytest.importorskip("torch")
    case = ("2d_70x130_d1_m2", 2, (70, 130), 1, 1.0, 2)
    base, _ = _run_case(lib, torch, case, 0, 0.5, False, seed=5)
    for tile in ["8,1", "16,2", "32,4", "64,8", "4,8", "1,2", "2,4", "8,8"]:
        monkeypatch.setenv("PDG_TILE", tile)
        (l2, mx), _ = _run_case(lib, torch, case, 0, 0.5, False, seed=5)
        assert l2 <= 1e-12 and mx <= 1e-11, tile


@pytest.mark.parametrize("case", [CASES[4], CASES[1]], ids=[CASES[4][0], CASES[1][0]])
def test_autotuned_tiles_solve_the_same_system(lib, case):
    """The autotuner only changes the work decomposition: parity on the
    context that was tuned, with the tiles it chose; the same tiles applied to
    a fresh context through pdg_set_tiles give the same result."""
    torch = pytest.importorskip("torch")
    (l2, mx), _, tuned = _run_case(lib, torch, case, 0, 0.5, False, seed=8, autotune=True)
    print(f"  tuned tiles {tuned}: rel L2 {l2:.3e} max {mx:.3e}")
    assert {t["np"] for t in tuned} == {case[3] + 1}
    assert l2 <= 1e-12 and mx <= 1e-11
    (l2b, mxb), _, used = _run_case(lib, torch, case, 0, 0.5, False, seed=8, tiles=tuned)
    assert used == tuned
    assert l2b <= 1e-12 and mxb <= 1e-11
    inst = _instance(case)
    prob = lib.Problem([inst_dict(inst)])
    prob.prepare(0.05)
    with pytest.raises(lib.PdgError):
        prob.set_tiles([dict(np=case[3] + 1, x_kind=0, C=7, S=1)])
    prob.close()
