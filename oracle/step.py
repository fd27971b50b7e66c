"""Kinetic problems and the splitting compositions of transport and collision.

Oracle (test infrastructure only).

A problem is a mesh, a velocity set {v_i} (nv x D), m components per
velocity, and an equilibrium model.  The state F has shape (nv, m, nc, nd)
in the oracle's numbering (cells lexicographic x fastest, nodes tensor with
the first index fastest).

Compositions (Sec. 3.2 and Sec. 5.1), with T = theta-scheme transport of every
velocity and C = collision:
* LIE:               [T(dt) C]^N
* STRANG:            [T(dt/2) C T(dt/2)]^N     (the three-stage M_2)
* STRANG_COLLAPSED:  T(dt/2) C [T(dt) C]^{N-1} T(dt/2), the collapsed Strang
                     scheme of Sec. 5.1 in which the last half transport of a
                     step and the first of the next are fused.
The inflow data f^b is time independent (Sec. 2).

Pins: a constant equilibrium state is preserved over several steps (scalar
and Euler), second-order convergence in dt of the collapsed scheme for scalar
advection, and the involution C(C(f)) = f at omega = 2.
"""

import numpy as np

from . import mesh as _mesh
from . import relax as _relax
from . import transport as _tr

LIE, STRANG, STRANG_COLLAPSED = 0, 1, 2


class Problem:
    def __init__(self, n, lo, hi, degree, vel, m, feq_kind, feq_param):
        self.mesh = _mesh.Mesh(n, lo, hi, degree)
        self.vel = np.asarray(vel, dtype=float).reshape(-1, self.mesh.dim)
        self.nv = self.vel.shape[0]
        self.m = int(m)
        self.feq_kind = feq_kind            # "advection" or "euler"
        self.feq_param = dict(feq_param)
        self._levels = {}
        self._entries = {}

    # ---- equilibrium ----------------------------------------------------
    @property
    def lam(self):
        return float(np.max(np.abs(self.vel)))

    def flux(self, w):
        if self.feq_kind == "advection":
            return _relax.advection_flux(w, self.feq_param["a"])
        if self.feq_kind == "euler":
            return _relax.euler_flux(w, self.feq_param["gamma"])
        raise ValueError(self.feq_kind)

    def feq(self, w):
        return _relax.equilibrium(w, self.vel, self.flux(w), self.lam)

    # ---- per-velocity data ----------------------------------------------
    def levels(self, i):
        if i not in self._levels:
            self._levels[i] = _tr.topological_levels(self.mesh, self.vel[i])
        return self._levels[i]

    def entries(self, i):
        if i not in self._entries:
            self._entries[i] = _tr.inflow_entries(self.mesh, self.vel[i])
        return self._entries[i]

    def inflow_from_w(self, w_of_x):
        """f^b_i = f^eq_i(w(x)) at the inflow points of every velocity i.

        w_of_x: callable (E, D) -> (m, E).  Returns a list of (m, E_i).
        """
        out = []
        for i in range(self.nv):
            pts = self.entries(i)["coords"]
            w = w_of_x(pts)
            out.append(self.feq(w)[i])
        return out

    # ---- steps ------------------------------------------------------------
    def transport(self, f, fb_old, fb_new, dt, theta, method="sweep"):
        out = np.empty_like(f)
        for i in range(self.nv):
            if method == "direct":
                out[i] = _tr.theta_step_direct(self.mesh, self.vel[i], f[i], fb_old[i], fb_new[i], dt, theta)
            else:
                out[i] = _tr.theta_step_sweep(self.mesh, self.vel[i], f[i], fb_old[i], fb_new[i], dt, theta,
                                              levels=self.levels(i))
        return out

    def collide(self, f, omega):
        return _relax.relax(f, omega, self.feq)


def run(prob, f0, fb, dt, theta, omega, scheme, nsteps, method="sweep"):
    """Apply ``nsteps`` steps of the given composition; fb is time independent."""
    f = np.array(f0, dtype=float, copy=True)
    if nsteps <= 0:
        return f
    if scheme == LIE:
        for _ in range(nsteps):
            f = prob.transport(f, fb, fb, dt, theta, method)
            f = prob.collide(f, omega)
    elif scheme == STRANG:
        for _ in range(nsteps):
            f = prob.transport(f, fb, fb, dt / 2, theta, method)
            f = prob.collide(f, omega)
            f = prob.transport(f, fb, fb, dt / 2, theta, method)
    elif scheme == STRANG_COLLAPSED:
        f = prob.transport(f, fb, fb, dt / 2, theta, method)
        f = prob.collide(f, omega)
        for _ in range(nsteps - 1):
            f = prob.transport(f, fb, fb, dt, theta, method)
            f = prob.collide(f, omega)
        f = prob.transport(f, fb, fb, dt / 2, theta, method)
    else:
        raise ValueError("unknown scheme")
    return f
