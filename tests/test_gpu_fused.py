"""GPU parity of the fused collision + x transport pass (opt-in, PDG_FUSED=1:
the collapsed Strang step T(dt/2) [C T(dt)]^(N-1) C T(dt/2), Sec. 5.1, with
each C T pair run as one pass over the state for the velocities along x and
a sweep of the others): whole steps against the oracle, and against the same
steps with separate collision and sweep launches.  Rows shorter than a wave,
rows of several waves, rows with padding lanes, every precision."""
import numpy as np
import pytest

import workloads as W
from helpers import gpu_initial_state, gpu_to_oracle, inst_dict, oracle_initial_state, oracle_problem, rel_errors
from oracle import step as ost

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_1702_00169_amd as P
    return P


def _adv(dim, n, degree, m, seed):
    rng = np.random.default_rng(seed)
    a = list(rng.uniform(-0.4, 0.4, dim))
    centre = rng.uniform(0.3, 0.7, dim)
    g = W.gaussian_bump(0.6, centre, 18.0)
    w0 = (lambda x: 0.4 + g(x)) if m == 1 else (lambda x: np.concatenate([0.4 + (k + 1) * g(x) for k in range(m)]))
    return W.Instance(dim, n, degree, 1.0, m, "advection", {"a": a}, w0)


def _euler(dim, n, degree, seed):
    rng = np.random.default_rng(seed)
    if dim == 2:
        return W.Instance(2, n, degree, 3.0, 4, "euler", {"gamma": W.GAMMA},
                          W.isentropic_vortex(rng.uniform(0.4, 0.6, 2), 0.15, 0.8))
    bump = W.gaussian_bump(0.1, rng.uniform(0.3, 0.7, 3), 30.0)
    return W.Instance(3, n, degree, 3.0, 5, "euler", {"gamma": W.GAMMA},
                      W.euler_at_rest(lambda x: 1.0 + bump(x)[0], lambda x: 1.0 + 0.5 * bump(x)[0], 3))


CASES = [
    # name, instance factory (rows: nx cells, (d+1) blocks of ceil(nx/64) waves)
    ("adv3d_7x6x5_d2", lambda: _adv(3, (7, 6, 5), 2, 1, 1)),
    ("euler3d_9x7x6_d2", lambda: _euler(3, (9, 7, 6), 2, 2)),
    ("euler2d_20x17_d3", lambda: _euler(2, (20, 17), 3, 3)),
    ("adv2d_100x5_d1", lambda: _adv(2, (100, 5), 1, 1, 4)),         # a row of two waves, padding
    ("adv2d_130x4_d1", lambda: _adv(2, (130, 4), 1, 1, 5)),         # three waves per row
    ("euler2d_200x3_d1", lambda: _euler(2, (200, 3), 1, 6)),        # four waves per row, m = 4
    ("adv2d_64x6_d4", lambda: _adv(2, (64, 6), 4, 1, 7)),           # five nodes per cell
    ("euler3d_5x4x3_d4", lambda: _euler(3, (5, 4, 3), 4, 8)),
]
BARS = {0: 1e-12, 2: 1e-10, 3: 1e-10, 1: 1e-5}


@pytest.fixture(autouse=True)
def fused_on(monkeypatch):
    """The fused pass is opt-in: PDG_FUSED=1, read when a problem is prepared."""
    monkeypatch.setenv("PDG_FUSED", "1")


def _run(lib, torch, insts, prec, steps, dt, omega):
    prob = lib.Problem([inst_dict(i) for i in insts])
    prob.prepare(dt, theta=0.5, omega=omega, scheme=2, precision=prec)
    f, fb = gpu_initial_state(prob, insts, torch, None)
    prob.step(f, fb, steps)
    prob.sync_status()
    out = prob.state_to_f64(f).cpu().numpy()
    corr = prob.last_refine_correction() if prec in (2, 3) else None
    layout = prob.layout
    prob.close()
    return out, layout, corr


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", [0, 2, 3, 1], ids=["fp64", "fp32refine", "fp32refine48", "fp32"])
def test_fused_steps_match_oracle(lib, case, prec):
    torch = pytest.importorskip("torch")
    name, make = case
    print(f"fused steps case={name} prec={prec}", flush=True)
    inst = make()
    h = np.min((inst.hi - inst.lo) / np.array(inst.n))
    dt = 0.7 * h / inst.lam
    omega = 1.7
    out, layout, corr = _run(lib, torch, [inst], prec, 3, dt, omega)
    got = gpu_to_oracle(out, inst)
    oprob = oracle_problem(inst)
    f0, fb0 = oracle_initial_state(oprob, inst)
    want = ost.run(oprob, f0, fb0, dt, 0.5, omega, 2, 3)
    l2, mx = rel_errors(got, want)
    print(f"  rel L2 {l2:.3e} max {mx:.3e} refine correction {corr}")
    assert l2 <= BARS[prec] and mx <= 10 * BARS[prec]


@pytest.mark.parametrize("prec", [0, 3], ids=["fp64", "fp32refine48"])
def test_fused_equals_separate_passes(lib, prec, monkeypatch):
    """The fused pass against separate collision and sweep launches on a
    batch of instances of different degrees and row lengths (one fused
    launch group per (d+1, n_v, m, nx))."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(11)
    insts = [W.adv2d_instance(rng, n, int(rng.integers(1, 5)), rng.uniform(-0.45, 0.45, 2)) for n in (9, 40, 17, 70)]
    insts.append(_euler(2, (33, 12), 2, 12))
    outs = []
    for fused in ("1", "0"):
        monkeypatch.setenv("PDG_FUSED", fused)
        out, _, _ = _run(lib, torch, insts, prec, 4, 0.01, 1.8)
        outs.append(out)
    d = np.max(np.abs(outs[0] - outs[1])) / np.max(np.abs(outs[1]))
    print(f"  fused vs separate: max rel diff {d:.3e}")
    assert d <= (1e-13 if prec == 0 else 1e-10)
