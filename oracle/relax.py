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

* D2Q9 lattice model of the isothermal Euler equations with gravity
  (Sec. 5.1): one scalar f_i per velocity, the nine velocities lambda x
  {0, +-e_x, +-e_y, (+-1, +-1)}, moments w = P f = (rho, rho u_x, rho u_y) with
  the 3 x 9 matrix P of that section, and the second-order polynomial
  equilibrium f_i^eq = w_i rho (1 + u.v_i/c^2 + (u.v_i)^2/(2 c^4) - u.u/(2 c^2)),
  c = lambda / sqrt(3), weights 4/9 (rest), 1/9 (axis), 1/36 (diagonal).
* Source step S_2(h) (Sec. 3.2, Sec. 5.1): the Crank-Nicolson integrator of
  the source, applied to the equilibrium part of f: the moments follow
  w' = w + h/2 (S(w) + S(w')) with S(w) = (0, 0, -g rho) (constant gravity
  -g e_y), which keeps rho and so is solved exactly, w'_y = w_y - h g rho; the
  distribution function moves by f^eq(w') - f^eq(w), so its non-equilibrium
  part is untouched.

Pins (tests/test_oracle_relax.py, tests/test_oracle_d2q9.py): the moments of
f^eq equal w and Q(w), the collision leaves w unchanged, f^eq is a fixed
point, omega = 2 is an involution, the scalar form reduces to the printed
w/4 + (v_i.a) w/2 of the 2D advection workload, and the Euler flux of a state
at rest is (0, p I, 0); for D2Q9: P f^eq(w) = w, the second moment of f^eq is
the isothermal Euler flux rho c^2 I + rho u u, the weights reproduce the
lattice isotropy sums, S(0) = Id, S(-h) S(h) = Id, and the source moves the
momentum by -h g rho exactly.  Euler values after several steps are parity
unpinned beyond these invariants.
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


# ---- D2Q9 isothermal model (Sec. 5.1) ---------------------------------------

def d2q9_weights(vel, lam):
    """Lattice weight of each velocity from |v_i|^2 / lambda^2 in {0, 1, 2}."""
    vel = np.asarray(vel, dtype=float)
    r = np.rint(np.sum(vel * vel, axis=1) / (lam * lam)).astype(int)
    table = {0: 4.0 / 9.0, 1: 1.0 / 9.0, 2: 1.0 / 36.0}
    if vel.shape != (9, 2) or sorted(r.tolist()) != [0, 1, 1, 1, 1, 2, 2, 2, 2]:
        raise ValueError("not a D2Q9 velocity set")
    return np.array([table[k] for k in r])


def d2q9_moments(f, vel):
    """w = P f = (sum f_i, sum f_i v_ix, sum f_i v_iy); f of shape (9, 1, ...)."""
    f = np.asarray(f, dtype=float)[:, 0]
    vel = np.asarray(vel, dtype=float)
    return np.stack([np.sum(f, axis=0),
                     np.tensordot(vel[:, 0], f, axes=(0, 0)),
                     np.tensordot(vel[:, 1], f, axes=(0, 0))])


def d2q9_equilibrium(w, vel, lam):
    """f^eq of the isothermal D2Q9 model for w = (rho, rho u_x, rho u_y);
    returns shape (9, 1, ...)."""
    w = np.asarray(w, dtype=float)
    vel = np.asarray(vel, dtype=float)
    wt = d2q9_weights(vel, lam)
    c2 = lam * lam / 3.0
    rho = w[0]
    ux = w[1] / rho
    uy = w[2] / rho
    uu = ux * ux + uy * uy
    out = np.empty((9, 1) + rho.shape)
    for i in range(9):
        uv = ux * vel[i, 0] + uy * vel[i, 1]
        out[i, 0] = wt[i] * rho * (1.0 + uv / c2 + uv * uv / (2.0 * c2 * c2) - uu / (2.0 * c2))
    return out


def gravity_source_moments(w, h, g):
    """Crank-Nicolson source step on the moments: rho and rho u_x unchanged,
    rho u_y - h g rho (exact, since the source keeps rho)."""
    w = np.array(w, dtype=float, copy=True)
    w[2] = w[2] - h * g * w[0]
    return w


def source_step(f, h, g, moments_of_f, feq_of_w):
    """S_2(h) applied to the equilibrium part of f: f + f^eq(w') - f^eq(w)."""
    f = np.asarray(f, dtype=float)
    w = moments_of_f(f)
    w2 = gravity_source_moments(w, h, g)
    return f + feq_of_w(w2) - feq_of_w(w)
