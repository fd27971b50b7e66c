"""Failure paths of the device entry points.

* PDG_EDEVICE from the dense sweep: the bound of the trace waits is set to
  zero ticks from the host (PDG_DENSE_WAIT_TICKS=0, read at prepare), so the
  first wait that is not served at once gives up, substitutes zeros and
  reports.  Every wave still runs to its end; only the result is invalid.
  pdg_sync_status reports it, and until then every entry point that would
  build on the invalid state refuses with PDG_EDEVICE.
* PDG_ESINGULAR: a time step of negative size at which I + theta dt Gamma has
  an eigenvalue 0 (Gamma has a real eigenvalue for d = 2), for the line blocks
  of an axis-aligned velocity and for the dense block of a diagonal velocity.
"""
import numpy as np
import pytest

import workloads as W
from helpers import gpu_initial_state, inst_dict

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_1702_00169_amd as P
    return P


def test_dense_wait_give_up_is_reported(lib, monkeypatch):
    torch = pytest.importorskip("torch")
    print("dense wait bound 0 ticks, claimed schedule, gravity2d 128^2", flush=True)
    monkeypatch.setenv("PDG_DENSE_SCHEDULE", "claim")
    monkeypatch.setenv("PDG_DENSE_WAIT_TICKS", "0")
    wl = W.make("gravity2d_256", seed=0, scale=128)
    prob = lib.Problem([inst_dict(i) for i in wl.instances])
    prob.prepare(wl.dt, precision=lib.PDG_FP64)
    f, fb = gpu_initial_state(prob, wl.instances, torch, torch.float64)
    prob.transport_sweep(f, fb, fb, wl.dt)
    torch.cuda.synchronize()
    # the kernels have finished: the host-visible flag is set, so the next
    # calls refuse before launching anything
    with pytest.raises(lib.PdgError) as ei:
        prob.step(f, fb, 1)
    assert ei.value.status == lib.PDG_EDEVICE
    with pytest.raises(lib.PdgError) as ei:
        prob.relax(f)
    assert ei.value.status == lib.PDG_EDEVICE
    with pytest.raises(lib.PdgError) as ei:
        prob.transport_sweep(f, fb, fb, wl.dt)
    assert ei.value.status == lib.PDG_EDEVICE
    with pytest.raises(lib.PdgError) as ei:
        prob.sync_status()
    assert ei.value.status == lib.PDG_EDEVICE and "timed out" in str(ei.value)
    # reported once: the flags are clear again and the context works
    prob.sync_status()
    prob.relax(f)
    prob.sync_status()
    prob.close()
    # the default bound (1 s) on the same problem: no failure
    monkeypatch.delenv("PDG_DENSE_WAIT_TICKS")
    prob = lib.Problem([inst_dict(i) for i in wl.instances])
    prob.prepare(wl.dt, precision=lib.PDG_FP64)
    f, fb = gpu_initial_state(prob, wl.instances, torch, torch.float64)
    prob.step(f, fb, 2)
    prob.sync_status()
    prob.close()


def _real_eigenvalue(G):
    ev = np.linalg.eigvals(G)
    re = ev[np.abs(ev.imag) < 1e-9 * np.abs(ev).max()].real
    assert re.size > 0
    return float(re.max())


@pytest.mark.parametrize("kind", ["line", "dense"])
def test_singular_cell_block_is_reported(lib, kind):
    torch = pytest.importorskip("torch")  # noqa: F841  (the inversion runs on the device)
    print(f"singular {kind} block", flush=True)
    vel = [[1.0, 0.0]] if kind == "line" else [[1.0, 1.0]]
    desc = dict(dim=2, n=[4, 3], degree=2, v=vel, m=1, feq="advection", feq_param=[0.1, 0.1])
    prob = lib.Problem([desc])
    N = 3 if kind == "line" else 9
    g = np.zeros(N * N)
    if kind == "line":
        lib.pdg_line_operator(prob.ctx, 0, 0, g)
    else:
        lib.pdg_cell_operator(prob.ctx, 0, 0, g, np.zeros(3))
    lam = _real_eigenvalue(g.reshape(N, N))
    theta = 0.5
    dt = -1.0 / (theta * lam)   # I + theta dt Gamma is singular
    with pytest.raises(lib.PdgError) as ei:
        prob.prepare(dt, theta=theta)
    assert ei.value.status == lib.PDG_ESINGULAR
    # the context is left unprepared, and a regular step size works
    with pytest.raises(lib.PdgError) as ei:
        prob.relax(torch.zeros(prob.layout["f_elems"], dtype=torch.float64, device="cuda"))
    assert ei.value.status == lib.PDG_ESTATE
    prob.prepare(0.9 * dt, theta=theta)
    prob.prepare(-dt, theta=theta)
    prob.close()
