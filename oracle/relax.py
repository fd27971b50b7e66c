"""Moments, equilibria and the Crank-Nicolson collision update.

Oracle (test infrastructure only).

* Moments (eq. micro_to_macro, Sec. 2): w = P f.  For the kinetic models used
  here every velocity carries all m components and P sums over velocities:
  w_k = sum_i f_{i,k}.
* Equilibrium (Sec. 2): f^eq depends on w only, has the same moments
  (P f^eq = P f) and reproduces the flux, q^k(w) = P V^k f^eq.  For the
  D_dQ_{2D} sets {+-lambda e_k} the paper gives no formula; the reading used is
  f_i^eq = w / (2D) + v_i . Q(w) / (2 lambda^2), Q = (q^1, ..., q^D), which
  satisfies both moment conditions exactly.  Two fluxes are provided: linear
  advection q^k = a_k w (scalar) and the compressible Euler flux (m = D+2).
* Collision (eq. collision_cn): C_2(dt) F = F + omega (F^eq(F) - F) with
  omega = 2 dt / (2 tau + dt); omega = 2 is the tau = 0 limit.

Pins (tests/test_oracle_relax.py): the moments of f^eq equal w and Q(w), the
collision leaves w unchanged, f^eq is a fixed point, omega = 2 is an
involution, the scalar form reduces to the printed w/4 + (v_i.a) w/2 of the
2D advection workload, and the Euler flux of a state at rest is (0, p I, 0).
Euler values after several steps are parity unpinned beyond these invariants.
"""

import math

import numpy as np


def moments(f):
    """w[k, ...] = sum_i f[i, k, ...] for f of shape (nv, m, ...)."""
    return np.sum(np.asarray(f, dtype=float), axis=0)


def moments_fsum(f):
    """Same as ``moments`` but each sum with math.fsum (exactly rounded)."""
    f = np.asarray(f, dtype=float)
    flat = f.reshape(f.shape[0], -1)
    out = np.array([math.fsum(flat[:, q]) for q in range(flat.shape[1])])
    return out.reshape(f.shape[1:])


def euler_flux(w, gamma):
    """q[k] of the compressible Euler equations for w = (rho, rho u_1..D, E).

    Returns array of shape (D, m, ...): q[k] = (rho u_k, rho u_k u + p e_k,
    (E + p) u_k), p = (gamma - 1)(E - |rho u|^2 / (2 rho)).
    """
    w = np.asarray(w, dtype=float)
    m = w.shape[0]
    dim = m - 2
    rho = w[0]
    mom = w[1:1 + dim]
    energy = w[1 + dim]
    u = mom / rho
    p = (gamma - 1.0) * (energy - 0.5 * np.sum(mom * u, axis=0))
    q = np.empty((dim,) + w.shape)
    for k in range(dim):
        q[k, 0] = mom[k]
        for l in range(dim):
            q[k, 1 + l] = mom[k] * u[l] + (p if l == k else 0.0)
        q[k, 1 + dim] = (energy + p) * u[k]
    return q


def advection_flux(w, a):
    """q[k] = a_k w for linear advection, shape (D, m, ...)."""
    w = np.asarray(w, dtype=float)
    a = np.asarray(a, dtype=float)
    return np.stack([a[k] * w for k in range(a.size)])


def equilibrium(w, vel, flux, lam):
    """f^eq[i] = w/(2D) + v_i . Q(w) / (2 lambda^2) for the set {+-lambda e_k}.

    w: (m, ...); vel: (nv, D) with nv = 2D; flux: Q(w) of shape (D, m, ...).
    """
    vel = np.asarray(vel, dtype=float)
    nv, dim = vel.shape
    if nv != 2 * dim:
        raise ValueError("equilibrium defined for the 2D-velocity sets {+-lambda e_k}")
    out = np.empty((nv,) + np.shape(w))
    for i in range(nv):
        acc = np.asarray(w, dtype=float) / (2.0 * dim)
        for k in range(dim):
            acc = acc + vel[i, k] * flux[k] / (2.0 * lam * lam)
        out[i] = acc
    return out


def relax(f, omega, feq_of_w):
    """C_2 update f + omega (f^eq(P f) - f) (eq. collision_cn)."""
    f = np.asarray(f, dtype=float)
    w = moments(f)
    return f + omega * (feq_of_w(w) - f)
