"""Structured meshes of hexahedral cells with affine maps.

Oracle (test infrastructure only).  The paper maps the reference cell
]-1,1[^D onto each cell L by tau_L with positive Jacobian determinant and
places the Gauss-Lobatto points and weights of eq. map_GL in it (Sec. 3.1).
Every map here is affine, tau_L(xh) = corner_L + J_L (xh + 1), on three kinds
of meshes: uniform box cells on [lo, hi]; tensor-product graded box cells
(per-axis cell edges: sizes vary along each axis); and a uniform affine
lattice (cell edge vectors a_k, the columns of `axes`): every cell is the same
parallelogram / parallelepiped, corner_L = lo + sum_k i_k a_k, J_L = A / 2.

Numbering used by the oracle (its own; the GPU library has another):
cells are lexicographic with x fastest, nodes in a cell are tensor indices
(i_0, ..., i_{D-1}) with i_0 fastest, i.e. node = sum_k i_k (d+1)^k.
"""

import itertools

import numpy as np

from . import gl


class Mesh:
    """Mesh of n[0] x ... x n[D-1] cells, degree d: uniform boxes on [lo, hi],
    boxes with cell edges edges[k] (n[k] + 1 increasing values) along axis k,
    or the affine lattice of cell edge vectors axes[:, k] (D x D, positive
    determinant) from the corner lo (hi is then ignored)."""

    def __init__(self, n, lo, hi, degree, edges=None, axes=None):
        self.n = tuple(int(v) for v in n)
        self.dim = len(self.n)
        if self.dim not in (1, 2, 3):
            raise ValueError("dimension must be 1, 2 or 3")
        self.axes = None
        if axes is not None:
            if edges is not None:
                raise ValueError("a mesh has either cell edges or lattice axes")
            self.axes = np.asarray(axes, dtype=float).reshape(self.dim, self.dim)
            if not np.linalg.det(self.axes) > 0:
                raise ValueError("the lattice axes must have a positive determinant")
            lo = np.asarray(lo, dtype=float).reshape(self.dim)
            # box-equivalent edges: only used for the extent of each axis index
            edges = [np.arange(self.n[k] + 1, dtype=float) for k in range(self.dim)]
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
        if self.axes is not None:
            self.lo = lo
            self.hi = lo + self.axes @ np.array(self.n, dtype=float)   # the far corner
            self.h = np.linalg.norm(self.axes, axis=0)
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
        if self.axes is not None:
            return np.broadcast_to(self.axes / 2.0, (len(multi), self.dim, self.dim)).copy()
        corner = self.corner(multi)
        jac = np.zeros((len(multi), self.dim, self.dim))
        for k in range(self.dim):
            far = corner.copy()
            far[:, k] = self.edges[k][multi[:, k] + 1]
            jac[:, :, k] = (far - corner) / 2.0
        return jac

    def corner(self, multi):
        """Lower corner of the cells with integer coordinates multi, (N, D)."""
        if self.axes is not None:
            return self.lo[None, :] + np.asarray(multi, dtype=float) @ self.axes.T
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
