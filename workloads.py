"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and bench.

This module holds problem data only: velocity sets, mesh sizes, time steps,
and the initial macroscopic fields w_0(x) as closed-form functions of the
physical position.  It contains none of the method's arithmetic (no
quadrature, no transport operator, no equilibrium); each side evaluates the
functions below at its own Gauss-Lobatto points and builds f^0 = f^eq(w_0)
and f^b = f^eq(w_0) on the inflow boundary with its own code.

The paper's meshes and physics runs are not available, so these workloads
stand in for them: 2D and 3D uniform or graded (tensor-product) box meshes,
the {+-lambda e_k} velocity sets
(the first 2D / 6 points of the paper's D2Q9 / D3Q27 lists), scalar advection
and compressible Euler equilibria, and smooth seeded data; and the D2Q9
isothermal gravity test of Sec. 5.1 (the paper's velocity list and its
hydrostatic steady state rho_0 exp(-g y / c^2), c^2 = lambda^2 / 3).
"""

import math

import numpy as np

D2Q4 = np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [0.0, -1.0]])
D3Q6 = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [-1.0, 0.0, 0.0],
                 [0.0, -1.0, 0.0], [0.0, 0.0, -1.0], [0.0, 0.0, 1.0]])

D2Q9 = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [0.0, -1.0],
                 [1.0, 1.0], [-1.0, 1.0], [-1.0, -1.0], [1.0, -1.0]])

GAMMA = 1.4


class Instance:
    """One independent kinetic problem on the unit box."""

    def __init__(self, dim, n, degree, lam, m, feq_kind, feq_param, w0, name="", vel=None):
        self.dim = dim
        self.n = tuple(n)
        self.degree = degree
        self.lam = float(lam)
        base = (D2Q4 if dim == 2 else D3Q6) if vel is None else np.asarray(vel, dtype=float)
        self.vel = base * self.lam
        self.m = m
        self.feq_kind = feq_kind        # "advection" | "euler" | "d2q9"
        self.feq_param = feq_param      # {"a": [...]}, {"gamma": g} or {"g": gravity}
        self.w0 = w0                    # callable (N, dim) -> (m, N)
        self.lo = np.zeros(dim)
        self.hi = np.ones(dim)
        self.edges = None               # optional per-axis cell edges (graded mesh)
        self.name = name

    @property
    def n_dof(self):
        return self.vel.shape[0] * self.m * int(np.prod(self.n)) * (self.degree + 1) ** self.dim


class Workload:
    def __init__(self, name, instances, dt, steps, theta=0.5, omega=2.0, description=""):
        self.name = name
        self.instances = instances
        self.dt = dt
        self.steps = steps
        self.theta = theta
        self.omega = omega
        self.description = description

    @property
    def n_dof(self):
        return sum(i.n_dof for i in self.instances)


# ---------------------------------------------------------------------------
# initial fields
# ---------------------------------------------------------------------------
def gaussian_bump(amplitude, centre, width2):
    """w(x) = amplitude * exp(-|x - centre|^2 * width2), scalar."""
    centre = np.asarray(centre, dtype=float)

    def w0(x):
        r2 = np.sum((np.asarray(x, dtype=float) - centre) ** 2, axis=1)
        return (amplitude * np.exp(-width2 * r2))[None, :]
    return w0


def gaussian_sum(amps, centres, sigmas, offset=0.0):
    amps = np.asarray(amps, float)
    centres = np.asarray(centres, float)
    sigmas = np.asarray(sigmas, float)

    def g(x):
        x = np.asarray(x, dtype=float)
        out = np.full(x.shape[0], offset)
        for a, c, s in zip(amps, centres, sigmas):
            out = out + a * np.exp(-np.sum((x - c) ** 2, axis=1) / (2.0 * s * s))
        return out
    return g


def isentropic_vortex(centre, radius, rho_min, gamma=GAMMA):
    """Conservative (rho, rho u, rho v, E) of a Shu-type isentropic vortex.

    Background rho = 1, p = 1, u = 0.  With r = |x - centre| / radius the
    temperature dip is dT = -(gamma-1) eps^2 / (8 gamma pi^2) exp(1 - r^2) and
    the velocity is eps / (2 pi) exp((1 - r^2)/2) (-y', x') with (x', y') =
    (x - centre) / radius; rho = (1 + dT)^(1/(gamma-1)), p = rho^gamma.
    eps is chosen so that rho(centre) = rho_min.
    """
    centre = np.asarray(centre, dtype=float)
    t_min = rho_min ** (gamma - 1.0)
    eps = math.sqrt((1.0 - t_min) * 8.0 * gamma * math.pi ** 2 / ((gamma - 1.0) * math.e))

    def w0(x):
        xp = (np.asarray(x, dtype=float) - centre) / radius
        r2 = np.sum(xp ** 2, axis=1)
        dtemp = -(gamma - 1.0) * eps ** 2 / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
        amp = eps / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
        u = -amp * xp[:, 1]
        v = amp * xp[:, 0]
        rho = (1.0 + dtemp) ** (1.0 / (gamma - 1.0))
        p = rho ** gamma
        energy = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
        return np.stack([rho, rho * u, rho * v, energy])
    return w0


def euler_at_rest(rho_fn, p_fn, dim, gamma=GAMMA):
    def w0(x):
        rho = rho_fn(x)
        p = p_fn(x)
        zeros = [np.zeros_like(rho)] * dim
        return np.stack([rho] + zeros + [p / (gamma - 1.0)])
    return w0


def hydrostatic_d2q9(rho0, g, lam, bump=0.0, centre=(0.5, 0.5), width2=40.0):
    """(rho, rho u_x, rho u_y) of the fluid at rest in gravity -g e_y,
    rho = rho0 exp(-g y / c^2), c^2 = lambda^2 / 3 (Sec. 5.1), times an
    optional density bump 1 + bump exp(-|x - centre|^2 width2)."""
    c2 = lam * lam / 3.0
    centre = np.asarray(centre, dtype=float)

    def w0(x):
        x = np.asarray(x, dtype=float)
        rho = rho0 * np.exp(-g * x[:, 1] / c2)
        if bump:
            rho = rho * (1.0 + bump * np.exp(-width2 * np.sum((x - centre) ** 2, axis=1)))
        return np.stack([rho, np.zeros_like(rho), np.zeros_like(rho)])
    return w0


def gravity2d_instance(n, degree, lam=1.0, g=1.0, rho0=1.0, bump=0.0):
    """The D2Q9 isothermal gravity problem of Sec. 5.1 on the unit square."""
    return Instance(2, (n, n), degree, lam, 1, "d2q9", {"g": g}, hydrostatic_d2q9(rho0, g, lam, bump),
                    name=f"gravity2d_n{n}_d{degree}", vel=D2Q9)


def graded_edges(n, lo, hi, stretch=1.5, jitter=0.0, seed=0):
    """n + 1 increasing cell edges on [lo, hi]: exponentially stretched
    (cells grow by about exp(stretch / n) from one to the next; 0 = uniform),
    optionally with seeded random jitter of each interior edge by up to
    jitter x the local cell size."""
    s = np.arange(n + 1) / n
    if stretch:
        s = np.expm1(stretch * s) / np.expm1(stretch)
    e = lo + (hi - lo) * s
    if jitter and n > 1:
        rng = np.random.default_rng(seed)
        h = np.diff(e)
        e[1:-1] += jitter * np.minimum(h[:-1], h[1:]) * rng.uniform(-1.0, 1.0, n - 1)
    return e


def uniform_state(values):
    values = np.asarray(values, dtype=float)

    def w0(x):
        return np.repeat(values[:, None], np.asarray(x).shape[0], axis=1)
    return w0


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------
def adv2d_instance(rng, n, degree, a, lam=1.0):
    amp = 1.0 + 0.1 * rng.uniform(-1.0, 1.0)
    return Instance(2, (n, n), degree, lam, 1, "advection", {"a": list(a)},
                    gaussian_bump(amp, (0.5, 0.5), 50.0), name=f"adv2d_n{n}_d{degree}")


def make(name, seed=0, scale=None):
    """Build a workload by name.  ``scale`` overrides the cells per axis
    (used by tests to shrink a workload while keeping its physics)."""
    rng = np.random.default_rng(seed)
    if name == "adv2d_16":
        n = scale or 16
        inst = adv2d_instance(rng, n, 2, (0.5, 0.25))
        return Workload(name, [inst], dt=0.01, steps=10,
                        description="2D scalar advection, D2Q4 lambda=1, a=(0.5,0.25), 16x16 cells, degree 2")
    if name == "adv3d_64":
        n = scale or 64
        amps = rng.uniform(0.5, 1.0, 8)
        cents = rng.uniform(0.2, 0.8, (8, 3))
        sig = rng.uniform(0.05, 0.15, 8)
        g = gaussian_sum(amps, cents, sig)
        inst = Instance(3, (n, n, n), 2, 1.0, 1, "advection", {"a": [0.3, 0.2, 0.1]},
                        lambda x: g(x)[None, :], name=f"adv3d_n{n}_d2")
        return Workload(name, [inst], dt=0.01, steps=50,
                        description="3D scalar advection, D3Q6 lambda=1, a=(0.3,0.2,0.1), 64^3 cells, degree 2")
    if name == "euler2d_256":
        n = scale or 256
        centre = rng.uniform(0.4, 0.6, 2)
        inst = Instance(2, (n, n), 3, 3.0, 4, "euler", {"gamma": GAMMA},
                        isentropic_vortex(centre, 0.1, 0.8), name=f"euler2d_n{n}_d3")
        return Workload(name, [inst], dt=(1.0 / n) / 3.0, steps=10,
                        description="2D Euler, D2Q4 lambda=3, m=4, 256^2 cells, degree 3, isentropic vortex")
    if name == "euler3d_128":
        n = scale or 128
        ar = rng.uniform(0.5, 1.0, 4)
        ap = rng.uniform(0.5, 1.0, 4)
        cr = rng.uniform(0.2, 0.8, (4, 3))
        cp = rng.uniform(0.2, 0.8, (4, 3))
        sgr = rng.uniform(0.05, 0.15, 4)
        sgp = rng.uniform(0.05, 0.15, 4)
        # amplitudes normalised to sum 1, so each bump field stays in [0, 1]
        grho = gaussian_sum(ar / ar.sum(), cr, sgr)
        gpr = gaussian_sum(ap / ap.sum(), cp, sgp)
        inst = Instance(3, (n, n, n), 2, 3.0, 5, "euler", {"gamma": GAMMA},
                        euler_at_rest(lambda x: 1.0 + 0.1 * grho(x), lambda x: 1.0 + 0.1 * gpr(x), 3),
                        name=f"euler3d_n{n}_d2")
        return Workload(name, [inst], dt=(1.0 / n) / 3.0, steps=20,
                        description="3D Euler, D3Q6 lambda=3, m=5, 128^3 cells, degree 2, density/pressure bumps")
    if name == "adv3d_64_graded":
        # the adv3d_64 problem on a graded mesh: cells stretched along every
        # axis (sizes from about 0.4 to 1.9 times the uniform size, jittered)
        wl = make("adv3d_64", seed=seed, scale=scale)
        inst = wl.instances[0]
        inst.edges = [graded_edges(inst.n[k], 0.0, 1.0, 1.0, 0.2, seed=seed + k) for k in range(3)]
        inst.name += "_graded"
        return Workload(name, [inst], dt=wl.dt, steps=wl.steps,
                        description="3D scalar advection, D3Q6 lambda=1, a=(0.3,0.2,0.1), 64^3 cells graded along "
                                    "every axis (stretch 1.0, jitter 0.2), degree 2")
    if name == "gravity2d_256":
        n = scale or 256
        inst = gravity2d_instance(n, 3, lam=1.0, g=1.0, bump=0.05)
        return Workload(name, [inst], dt=1.0 / n, steps=10,
                        description="2D isothermal Euler with gravity, D2Q9 lambda=1 (c^2=1/3), g=1, "
                                    "256^2 cells, degree 3, hydrostatic state with a 5% density bump")
    if name == "batch96":
        count = 96 if scale is None else scale
        insts = []
        for _ in range(count):
            n = int(rng.integers(32, 513))
            d = int(rng.integers(1, 5))
            a = rng.uniform(-0.45, 0.45, 2)
            insts.append(adv2d_instance(rng, n, d, a))
        return Workload(name, insts, dt=0.01, steps=10,
                        description="96 uneven 2D scalar D2Q4 instances, n~U{32..512}, degree~U{1..4}")
    raise KeyError(name)


WORKLOADS = ("adv2d_16", "adv3d_64", "euler2d_256", "euler3d_128", "batch96", "gravity2d_256", "adv3d_64_graded")


# ---------------------------------------------------------------------------
# generic seeded arrays for parity tests
# ---------------------------------------------------------------------------
def random_state(seed, shape, low=0.5, high=1.5):
    """Uniform random values (no smoothness); used as arbitrary transport input."""
    return np.random.default_rng(seed).uniform(low, high, size=shape)


def smooth_field(seed, dim, m, modes=3):
    """A seeded smooth function x -> (m, N): sums of low Fourier modes."""
    rng = np.random.default_rng(seed)
    k = rng.integers(0, modes + 1, size=(m, 4, dim))
    ph = rng.uniform(0, 2 * np.pi, size=(m, 4))
    am = rng.uniform(0.05, 0.2, size=(m, 4))

    def f(x):
        x = np.asarray(x, dtype=float)
        out = np.ones((m, x.shape[0]))
        for c in range(m):
            for t in range(4):
                out[c] += am[c, t] * np.cos(2 * np.pi * (x @ k[c, t]) + ph[c, t])
        return out
    return f
