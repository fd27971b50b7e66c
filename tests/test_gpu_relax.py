"""GPU parity of the collision step (eq. collision_cn) and the equilibrium
helpers with the oracle.  Bars as for the sweep."""
import numpy as np
import pytest

import workloads as W
from helpers import (gpu_fb_from_function, gpu_initial_state, gpu_to_oracle, inst_dict, oracle_fb_from_function,
                     oracle_initial_state, oracle_problem, oracle_to_gpu, rel_errors, sizes)
from oracle import relax as orx

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_1702_00169_amd as P
    return P


def _insts():
    return [
        W.make("adv2d_16", seed=1).instances[0],
        W.make("euler2d_256", seed=2, scale=12).instances[0],
        W.make("euler3d_128", seed=3, scale=5).instances[0],
        W.make("adv3d_64", seed=4, scale=6).instances[0],
    ]


@pytest.mark.parametrize("idx", range(4), ids=["adv2d", "euler2d", "euler3d", "adv3d"])
@pytest.mark.parametrize("prec", [0, 2, 1], ids=["fp64", "fp32refine", "fp32"])
@pytest.mark.parametrize("omega", [2.0, 1.37])
def test_relax_matches_oracle(lib, idx, prec, omega):
    torch = pytest.importorskip("torch")
    inst = _insts()[idx]
    print(f"relax {inst.name} prec={prec} omega={omega}", flush=True)
    prob = lib.Problem([inst_dict(inst)])
    prob.prepare(0.01, omega=omega, precision=prec)
    oprob = oracle_problem(inst)
    f0, _ = oracle_initial_state(oprob, inst)
    rng = np.random.default_rng(idx)
    f_or = f0 * (1.0 + 0.05 * rng.standard_normal(f0.shape))
    if prec == 1:
        f_or = f_or.astype(np.float32).astype(np.float64)
    f = torch.tensor(oracle_to_gpu(f_or), dtype=torch.float32 if prec == 1 else torch.float64, device="cuda")
    w_out = torch.zeros(prob.layout["w_elems"], dtype=torch.float64, device="cuda")
    prob.relax(f, w_out)
    torch.cuda.synchronize()
    got = gpu_to_oracle(f.double().cpu().numpy(), inst)
    want = oprob.collide(f_or, omega)
    l2, mx = rel_errors(got, want)
    bar = {0: 1e-13, 2: 1e-13, 1: 1e-6}[prec]
    print(f"  f rel L2 {l2:.3e} max {mx:.3e}")
    assert l2 <= bar and mx <= 10 * bar
    nc, nd = sizes(inst)
    w_got = np.transpose(w_out.cpu().numpy().reshape(inst.m, nd, nc), (0, 2, 1))
    w_want = orx.moments_fsum(f_or)
    assert rel_errors(w_got, w_want)[1] <= 1e-15 * inst.vel.shape[0]
    prob.close()


@pytest.mark.parametrize("idx", range(4), ids=["adv2d", "euler2d", "euler3d", "adv3d"])
def test_equilibrium_helpers_match_oracle(lib, idx):
    torch = pytest.importorskip("torch")
    inst = _insts()[idx]
    prob = lib.Problem([inst_dict(inst)])
    prob.prepare(0.01)
    f, fb = gpu_initial_state(prob, [inst], torch, torch.float64)
    oprob = oracle_problem(inst)
    f0, fb0 = oracle_initial_state(oprob, inst)
    l2, mx = rel_errors(gpu_to_oracle(f.cpu().numpy(), inst), f0)
    assert l2 <= 1e-14 and mx <= 1e-13
    # fb: compare per velocity by matching inflow points by position
    got = fb.cpu().numpy()
    off = 0
    _, inflow = prob.node_coords(0)
    ioff = 0
    for v in range(oprob.nv):
        ent = oprob.entries(v)
        npts = ent["coords"].shape[0]
        pts = inflow[ioff:ioff + inst.dim * npts].reshape(inst.dim, npts).T
        vals = got[off:off + inst.m * npts].reshape(inst.m, npts)
        key_g = np.lexsort(np.round(pts, 12).T[::-1])
        key_o = np.lexsort(np.round(ent["coords"], 12).T[::-1])
        np.testing.assert_allclose(pts[key_g], ent["coords"][key_o], atol=1e-13)
        assert rel_errors(vals[:, key_g], fb0[v][:, key_o])[1] <= 1e-13
        off += inst.m * npts
        ioff += inst.dim * npts
    prob.close()
