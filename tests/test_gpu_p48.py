"""The 48-bit state (PDG_FP32_REFINE_P48): binary32 cell solves with one
binary64 residual correction, as PDG_FP32_REFINE, with every state value kept
as a binary32 plane plus an int16 plane (a 40-bit significand).

* the storage format, bit for bit, against its definition in the header,
  written out again here with numpy;
* parity with the oracle of the transport sweep (axis-aligned chains of every
  kind, dense tiles under both schedules), the relaxation, the D2Q9 source
  and relaxation, and whole steps of every composition.

The input of each parity case is first written into the 48-bit state and read
back, and the oracle starts from those values, so the bars measure the path
(each stored result is rounded by at most 2^-39 relative, far below the
1e-10 bar of the refined arithmetic).
"""
import numpy as np
import pytest

import test_gpu_dense as TD
import test_gpu_sweep as TS
import workloads as W
from helpers import (gpu_fb_from_function, gpu_initial_state, gpu_state, gpu_state_values, gpu_to_oracle, inst_dict,
                     oracle_fb_from_function, oracle_initial_state, oracle_problem, oracle_to_gpu, rel_errors, sizes)
from oracle import step as ost
from oracle import transport as otr

pytestmark = pytest.mark.gpu

P48 = 3


@pytest.fixture(scope="module")
def lib():
    import paper_1702_00169_amd as P
    assert P.PDG_FP32_REFINE_P48 == P48
    return P


def _format_reference(x):
    """(h, l) of the documented format: h = x rounded to binary32, l =
    rint((x - h) 2^(39 - e)) clamped to +-32767, e the exponent of h's
    binade (-126 for zero and subnormal h)."""
    h = x.astype(np.float32)
    r = x - h.astype(np.float64)
    eb = ((h.view(np.uint32) >> 23) & 0xFF).astype(np.int64)
    e = np.where(eb == 0, -126, eb - 127)
    q = np.clip(np.rint(r * np.ldexp(1.0, 39 - e)), -32767, 32767)
    return h, q.astype(np.int16), e


def _format_values(n, seed):
    rng = np.random.default_rng(seed)
    mag = np.ldexp(1.0 + rng.random(n), rng.integers(-40, 40, n))
    x = np.where(rng.random(n) < 0.5, -mag, mag)
    special = np.array([0.0, -0.0, 1.0, -2.0, 1.0 - 2.0 ** -30, 1.0 + 2.0 ** -25, 2.0 ** -126 * 1.5,
                        2.0 ** -140, -3.0e-44, 1.0e30, np.nextafter(2.0, 0.0), 0.1, -1.0 / 3.0])
    x[:special.size] = special
    return x


def _prob(lib, n_values):
    """A problem whose state has at least n_values elements (2D, d = 1)."""
    side = int(np.ceil(np.sqrt(n_values / 16.0)))
    inst = W.make("adv2d_16", seed=0).instances[0]
    d = inst_dict(inst)
    d.update(n=[side, side], degree=1)
    prob = lib.Problem([d])
    prob.prepare(0.01, precision=P48)
    return prob


def test_storage_format_is_bit_exact(lib):
    torch = pytest.importorskip("torch")
    print("p48 storage format", flush=True)
    prob = _prob(lib, 200_000)
    n = prob.layout["f_elems"]
    x = _format_values(n, seed=3)
    f = prob.new_state()
    prob.state_from_f64(torch.tensor(x, device="cuda"), f)
    raw = f.cpu().numpy().view(np.uint8)
    assert raw.size == 6 * n
    h_gpu = raw[:4 * n].view(np.float32)
    l_gpu = raw[4 * n:].view(np.int16)
    h, l, e = _format_reference(x)
    assert np.array_equal(h_gpu.view(np.uint32), h.view(np.uint32))
    assert np.array_equal(l_gpu, l)
    # decoding is h + l 2^(e - 39), exact in binary64, within half a unit of
    # l of x, or one unit where l was clamped
    dec = gpu_state_values(prob, f)
    want = h.astype(np.float64) + l.astype(np.float64) * np.ldexp(1.0, e - 39)
    assert np.array_equal(dec, want)
    clamped = np.abs(l) == 32767
    err = np.abs(dec - x)
    assert np.all(err[~clamped] <= np.ldexp(1.0, e - 40)[~clamped])
    assert np.all(err[clamped] <= np.ldexp(1.0, e - 39)[clamped])
    normal = np.abs(x) >= 2.0 ** -126
    rel = err[normal] / np.abs(x[normal])
    print(f"  max relative rounding {rel.max():.3e} (2^-39 = {2.0 ** -39:.3e}); {clamped.sum()} clamped")
    assert rel.max() <= 2.0 ** -39
    # writing the decoded values again keeps them exactly (the bytes may
    # differ just below a power of two, where the value has two encodings)
    g = prob.new_state()
    prob.state_from_f64(torch.tensor(dec, device="cuda"), g)
    assert np.array_equal(gpu_state_values(prob, g), dec)
    prob.close()


def _sweep_case(lib, torch, inst, theta, half, seed, dense=False):
    prob = lib.Problem([inst_dict(inst)])
    nc, nd = sizes(inst)
    h = np.min((inst.hi - inst.lo) / np.array(inst.n))
    dt = (0.77 if dense else 0.83) * h / np.max(np.abs(inst.vel))
    prob.prepare(dt, theta=theta, omega=2.0, precision=P48)
    nv, m = inst.vel.shape[0], inst.m
    f = gpu_state(prob, torch, oracle_to_gpu(W.random_state(seed, (nv, m, nc, nd))))
    f_in = gpu_to_oracle(gpu_state_values(prob, f), inst)
    fo = W.smooth_field(seed + 1, inst.dim, m)
    fn = W.smooth_field(seed + 2, inst.dim, m)
    fbo = torch.tensor(gpu_fb_from_function(prob, [inst], lambda i, v, p: fo(p)), device="cuda")
    fbn = torch.tensor(gpu_fb_from_function(prob, [inst], lambda i, v, p: fn(p)), device="cuda")
    dsub = 0.5 * dt if half else dt
    prob.transport_sweep(f, fbo, fbn, dsub)
    prob.sync_status()
    got = gpu_to_oracle(gpu_state_values(prob, f), inst)
    corr = prob.last_refine_correction()
    oprob = oracle_problem(inst)
    ofo = oracle_fb_from_function(oprob, 0, lambda i, v, p: fo(p))
    ofn = oracle_fb_from_function(oprob, 0, lambda i, v, p: fn(p))
    want = np.empty_like(f_in)
    for v in range(nv):
        want[v] = otr.theta_step_sweep(oprob.mesh, inst.vel[v], f_in[v], ofo[v], ofn[v], dsub, theta,
                                       levels=oprob.levels(v))
    prob.close()
    return rel_errors(got, want), corr


@pytest.mark.parametrize("case", TS.CASES, ids=[c[0] for c in TS.CASES])
@pytest.mark.parametrize("theta,half", [(0.5, False), (1.0, True)])
def test_sweep_matches_oracle(lib, case, theta, half):
    torch = pytest.importorskip("torch")
    print(f"p48 sweep case={case[0]} theta={theta} half={half}", flush=True)
    (l2, mx), corr = _sweep_case(lib, torch, TS._instance(case), theta, half, seed=5)
    print(f"  rel L2 {l2:.3e} max {mx:.3e}; refine correction {corr:.2e}")
    assert l2 <= 1e-10 and mx <= 1e-9
    assert 0.0 < corr < 1e-5


@pytest.mark.parametrize("case", TD.CASES, ids=[c[0] for c in TD.CASES])
def test_dense_sweep_matches_oracle(lib, case, schedule):
    torch = pytest.importorskip("torch")
    print(f"p48 dense case={case[0]} schedule={schedule}", flush=True)
    (l2, mx), _ = _sweep_case(lib, torch, TD._instance(case), 0.5, False, seed=6, dense=True)
    print(f"  rel L2 {l2:.3e} max {mx:.3e}")
    assert l2 <= 1e-10 and mx <= 1e-9


@pytest.fixture(params=["level", "claim", "transfer"])
def schedule(request, monkeypatch):
    monkeypatch.setenv("PDG_DENSE_SCHEDULE", request.param)
    return request.param


@pytest.mark.parametrize("name,scale", [("adv2d_16", None), ("euler2d_256", 12), ("euler3d_128", 5),
                                        ("adv3d_64", 6)])
@pytest.mark.parametrize("omega", [2.0, 1.37])
def test_relax_matches_oracle(lib, name, scale, omega):
    torch = pytest.importorskip("torch")
    print(f"p48 relax {name} omega={omega}", flush=True)
    inst = (W.make(name, seed=2, scale=scale) if scale else W.make(name, seed=2)).instances[0]
    prob = lib.Problem([inst_dict(inst)])
    prob.prepare(0.01, omega=omega, precision=P48)
    oprob = oracle_problem(inst)
    f0, _ = oracle_initial_state(oprob, inst)
    rng = np.random.default_rng(7)
    f = gpu_state(prob, torch, oracle_to_gpu(f0 * (1.0 + 0.05 * rng.standard_normal(f0.shape))))
    f_in = gpu_to_oracle(gpu_state_values(prob, f), inst)
    prob.relax(f)
    got = gpu_to_oracle(gpu_state_values(prob, f), inst)
    want = oprob.collide(f_in, omega)
    l2, mx = rel_errors(got, want)
    print(f"  rel L2 {l2:.3e} max {mx:.3e}")
    # one rounding to the 40-bit significand (plus binary64 arithmetic)
    assert l2 <= 2e-12 and mx <= 4e-12
    prob.close()


def _run_steps(lib, torch, wl, scheme, steps):
    prob = lib.Problem([inst_dict(i) for i in wl.instances])
    prob.prepare(wl.dt, theta=wl.theta, omega=wl.omega, scheme=scheme, precision=P48)
    f, fb = gpu_initial_state(prob, wl.instances, torch, None)
    prob.step(f, fb, steps)
    prob.sync_status()
    out = gpu_state_values(prob, f)
    res = []
    for i, inst in enumerate(wl.instances):
        got = gpu_to_oracle(out, inst, prob.layout["f_off"][i])
        oprob = oracle_problem(inst)
        f0, fb0 = oracle_initial_state(oprob, inst)
        want = ost.run(oprob, f0, fb0, wl.dt, wl.theta, wl.omega, scheme, steps)
        res.append(rel_errors(got, want))
    prob.close()
    return res


@pytest.mark.parametrize("scheme", [0, 1, 2, 3, 4], ids=["lie", "strang", "collapsed", "kin", "kin4"])
def test_steps_adv2d_16(lib, scheme):
    torch = pytest.importorskip("torch")
    print(f"p48 steps adv2d_16 scheme={scheme}", flush=True)
    wl = W.make("adv2d_16", seed=0)
    (err,) = _run_steps(lib, torch, wl, scheme, wl.steps)
    print(f"  rel L2 {err[0]:.3e} max {err[1]:.3e}")
    assert err[0] <= 1e-10 and err[1] <= 1e-9


@pytest.mark.parametrize("name,scale,steps", [("euler2d_256", 24, 10), ("euler3d_128", 7, 20), ("adv3d_64", 8, 10)])
def test_collapsed_steps_of_the_workloads(lib, name, scale, steps):
    torch = pytest.importorskip("torch")
    print(f"p48 collapsed steps {name} scale={scale}", flush=True)
    wl = W.make(name, seed=1, scale=scale)
    (err,) = _run_steps(lib, torch, wl, 2, steps)
    print(f"  rel L2 {err[0]:.3e} max {err[1]:.3e}")
    assert err[0] <= 1e-10 and err[1] <= 1e-9


def test_uneven_batch_steps(lib):
    torch = pytest.importorskip("torch")
    print("p48 uneven batch", flush=True)
    rng = np.random.default_rng(3)
    insts = [W.adv2d_instance(rng, n, int(rng.integers(1, 5)), rng.uniform(-0.45, 0.45, 2))
             for n in (5, 33, 17, 40, 9, 26)]
    wl = W.Workload("batch_small", insts, dt=0.01, steps=4)
    for l2, mx in _run_steps(lib, torch, wl, 2, 4):
        assert l2 <= 1e-10 and mx <= 1e-9


@pytest.mark.parametrize("scheme", [0, 2, 3], ids=["lie", "collapsed", "kin"])
def test_gravity_steps_match_oracle(lib, scheme, schedule):
    """D2Q9 with the gravity source (Sec. 5.1): dense diagonal velocities, the
    lattice S C S kernel and the source step, all on the 48-bit state."""
    torch = pytest.importorskip("torch")
    print(f"p48 gravity steps scheme={scheme} schedule={schedule}", flush=True)
    wl = W.make("gravity2d_256", seed=0, scale=12)
    (err,) = _run_steps(lib, torch, wl, scheme, 4)
    print(f"  rel L2 {err[0]:.3e} max {err[1]:.3e}")
    assert err[0] <= 1e-10 and err[1] <= 1e-9
