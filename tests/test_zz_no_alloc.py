"""pdg_transport_sweep_static: the sweep whose scratch (refinement
statistics, dense trace slots, tile-claim counters) lives in the library's
static device array instead of the context's buffers.  Called through the C
ABI and compared with pdg_transport_sweep on copies of the same input, on
two calls in a row, the second with a smaller problem; a problem whose
scratch exceeds the static array is refused before any launch.
"""
import ctypes

import numpy as np
import pytest

import workloads as W
from helpers import gpu_initial_state, inst_dict, rel_errors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_1702_00169_amd as P
    return P


def _static_sweep(lib, prob, f, fb, dt_sub):
    import torch
    so = lib._lib
    so.pdg_transport_sweep_static.restype = ctypes.c_int32
    so.pdg_transport_sweep_static.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_double, ctypes.c_void_p]
    return so.pdg_transport_sweep_static(prob.ctx, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(fb.data_ptr()),
                                         ctypes.c_void_p(fb.data_ptr()), float(dt_sub),
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def _compare(lib, torch, wl, prec, schedule, monkeypatch):
    monkeypatch.setenv("PDG_DENSE_SCHEDULE", schedule)
    prob = lib.Problem([inst_dict(i) for i in wl.instances])
    prob.prepare(wl.dt, theta=wl.theta, omega=wl.omega, precision=prec)
    f, fb = gpu_initial_state(prob, wl.instances, torch, None)
    g = f.clone()
    prob.transport_sweep(f, fb, fb, wl.dt)
    prob.sync_status()
    corr = prob.last_refine_correction() if prec in (2, 3) else None
    assert _static_sweep(lib, prob, g, fb, wl.dt) == lib.PDG_OK
    prob.sync_status()
    corr_s = prob.last_refine_correction() if prec in (2, 3) else None
    a = prob.state_to_f64(f).cpu().numpy()
    b = prob.state_to_f64(g).cpu().numpy()
    l2, mx = rel_errors(b, a)
    print(f"  {wl.name} prec={prec} schedule={schedule}: rel L2 {l2:.3e} max {mx:.3e}; "
          f"bitwise equal {np.array_equal(a, b)}; refine correction {corr} / {corr_s}")
    assert l2 <= 1e-12 and mx <= 1e-12
    assert corr == corr_s
    prob.close()


@pytest.mark.parametrize("prec,schedule", [(0, "claim"), (2, "claim"), (3, "level")])
def test_static_sweep_equals_the_sweep_on_two_calls(lib, monkeypatch, prec, schedule):
    torch = pytest.importorskip("torch")
    print(f"static sweep prec={prec} schedule={schedule}", flush=True)
    # first call: D2Q9 gravity 128^2, degree 3 (dense tiles and chains)
    _compare(lib, torch, W.make("gravity2d_256", seed=0, scale=128), prec, schedule, monkeypatch)
    # second call, smaller: 48^2, and a 3D Euler problem on chains only
    _compare(lib, torch, W.make("gravity2d_256", seed=1, scale=48), prec, schedule, monkeypatch)
    _compare(lib, torch, W.make("euler3d_128", seed=1, scale=12), prec, schedule, monkeypatch)


def test_static_sweep_refuses_a_problem_beyond_its_scratch(lib, monkeypatch):
    torch = pytest.importorskip("torch")
    print("static sweep size limit", flush=True)
    monkeypatch.setenv("PDG_DENSE_SCHEDULE", "claim")
    wl = W.make("gravity2d_256", seed=0, scale=1100)   # about 39 MB of dense trace slots
    prob = lib.Problem([inst_dict(i) for i in wl.instances])
    prob.prepare(wl.dt, precision=0)
    f = torch.zeros(prob.layout["f_elems"], dtype=torch.float64, device="cuda")
    fb = torch.zeros(prob.layout["fb_elems"], dtype=torch.float64, device="cuda")
    assert _static_sweep(lib, prob, f, fb, wl.dt) == lib.PDG_EUNSUPPORTED
    assert "scratch" in lib.pdg_error_detail()
    assert float(f.abs().max()) == 0.0   # nothing was launched
    prob.close()
