"""Cartesian meshes of hexahedral (box) cells with affine maps.

Oracle (test infrastructure only).  The paper maps the reference cell
]-1,1[^D onto each cell L by tau_L with positive Jacobian determinant and
places the Gauss-Lobatto points and weights of eq. map_GL in it (Sec. 3.1).
On the axis-aligned box meshes used here, tau_L is affine:
tau_L(xh) = corner_L + (xh + 1) h_L / 2.  The cells are uniform on [lo, hi]
unless per-axis cell edges are given (a tensor-product graded mesh: cell
sizes vary along each axis, every cell stays a box).

Numbering used by the oracle (its own; the GPU library has another):
cells are lexicographic with x fastest, nodes in a cell are tensor indices
(i_0, ..., i_{D-1}) with i_0 fastest, i.e. node = sum_k i_k (d+1)^k.
"""

import itertools

import numpy as np

from . import gl


class Mesh:
    """Mesh of n[0] x ... x n[D-1] box cells, degree d: uniform on [lo, hi],
    or with cell edges edges[k] (n[k] + 1 increasing values) along axis k."""

    def __init__(self, n, lo, hi, degree, edges=None):
        self.n = tuple(int(v) for v in n)
        self.dim = len(self.n)
        if self.dim not in (1, 2, 3):
            raise ValueError("dimension must be 1, 2 or 3")
        if edges is None:
            lo = np.asarray(lo, dtype=float).reshape(self.dim)
            hi = np.asarray(hi, dtype=float).reshape(self.dim)
            edges = [lo[k] + (hi[k] - lo[k]) * np.arange(self.n[k] + 1) / self.n[k] for k in range(self.dim)]
        self.edges = [np.asarray(e, dtype=float) for e in edges]
        for k in range(self.dim):
            if self.edges[k].shape != (self.n[k] + 1,) or not np.all(np.diff(self.edges[k]) > 0):
                raise ValueError("edges must hold n[k] + 1 increasing values per axis")
        self.lo = np.array([e[0] for e in self.edges])
        self.hi = np.array([e[-1] for e in self.edges])
        # smallest cell size per axis (a length scale for tolerances)
        self.h = np.array([np.min(np.diff(e)) for e in self.edges])
        self.degree = int(degree)
        self.np1 = self.degree + 1
        self.nc = int(np.prod(self.n))
        self.nd = self.np1 ** self.dim
        self.xi, self.wi = gl.gauss_lobatto(self.degree)
        self.dmat = gl.lagrange_derivative_matrix(self.xi)
        # tensor index of every node: node_idx[i, k] = i_k
        self.node_idx = np.array(
            [tuple(reversed(t)) for t in itertools.product(range(self.np1), repeat=self.dim)],
            dtype=np.int64)
        # reference coordinates and weights of the tensor nodes (eq. map_GL)
        self.xhat = self.xi[self.node_idx]                      # (nd, D)
        self.what = np.prod(self.wi[self.node_idx], axis=1)     # (nd,)

    # ---- cells -----------------------------------------------------------
    def cell_multi(self, cells):
        """(len(cells), D) integer coordinates of flat cell indices."""
        cells = np.asarray(cells, dtype=np.int64)
        out = np.empty((cells.size, self.dim), dtype=np.int64)
        rem = cells.copy()
        for k in range(self.dim):
            out[:, k] = rem % self.n[k]
            rem //= self.n[k]
        return out

    def cell_flat(self, multi):
        multi = np.asarray(multi, dtype=np.int64)
        flat = np.zeros(multi.shape[0], dtype=np.int64)
        stride = 1
        for k in range(self.dim):
            flat += multi[:, k] * stride
            stride *= self.n[k]
        return flat

    def jacobian(self, cells):
        """tau_L' for each cell (affine: constant over the cell), shape (N, D, D).

        Computed from the cell's own corner coordinates, as a general affine
        map would be: column k is (corner + h_k e_k - corner) / 2.
        """
        multi = self.cell_multi(cells)
        corner = self.corner(multi)
        jac = np.zeros((len(multi), self.dim, self.dim))
        for k in range(self.dim):
            far = corner.copy()
            far[:, k] = self.edges[k][multi[:, k] + 1]
            jac[:, :, k] = (far - corner) / 2.0
        return jac

    def corner(self, multi):
        """Lower corner of the cells with integer coordinates multi, (N, D)."""
        return np.stack([self.edges[k][multi[:, k]] for k in range(self.dim)], axis=1)

    def node_coords(self, cells=None):
        """Physical GL points x_{L,i} = tau_L(xhat_i), shape (N, nd, D)."""
        if cells is None:
            cells = np.arange(self.nc)
        multi = self.cell_multi(cells)
        corner = self.corner(multi)                               # (N, D)
        jac = self.jacobian(cells)                                # (N, D, D)
        return corner[:, None, :] + np.einsum("nkl,jl->njk", jac, self.xhat + 1.0)

    def neighbour(self, cells, axis, side):
        """Flat index of the face neighbour across (axis, side), -1 on the boundary."""
        multi = self.cell_multi(cells)
        multi[:, axis] += side
        inside = (multi[:, axis] >= 0) & (multi[:, axis] < self.n[axis])
        out = np.full(len(multi), -1, dtype=np.int64)
        out[inside] = self.cell_flat(multi[inside])
        return out
