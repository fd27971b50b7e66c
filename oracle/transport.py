"""Upwind nodal DG transport operator and the implicit theta-scheme step.

Oracle (test infrastructure only).  Written from Sec. 3.1 and Sec. 4.1 of the
paper, for one constant velocity v and uniform affine Cartesian cells.

Per-cell blocks (Sec. 4.1, split of eq. DG_reduit).  The semi-discrete scheme
is d/dt f_L + Gamma_{L<-L} f_L + sum_R Gamma_{L<-R} f_R = 0 with

  (Gamma_{L<-L})_{ij} = -(1/omega_{L,i}) v . c_{L,j} gradhat phihat_i(xhat_j) omegahat_j
                        + delta_ij (1/omega_{L,i}) sum_eps mu_i^eps (v . c_{L,i} nhat_eps)^+
  (Gamma_{L<-R})_{i,i'} = (1/omega_{L,i}) mu_i^eps (v . c_{L,i} nhat_eps)^-

where c = co(tau_L') = det(tau_L') tau_L'^{-T} (eq. co_mat), omega_{L,i} =
omegahat_i det(tau_L') (eq. map_GL), mu_i^eps is the face weight of node i on
face eps (zero off the face), and i' is the node of the neighbour R at the
same physical point (found by matching coordinates).  On a boundary face the
neighbour value is the imposed inflow value f^b (eq. boundary_conditions),
held in a fictitious cell with d/dt f^b = 0 (eq. fictitious_ODE).

Global form (eq. linear_ODE).  d/dt F = L_h F + b with L_h = -Gamma over the
real cells and b = -Gamma_{L<-boundary} f^b.

Theta-scheme step (eq. transport_cn; the garbled eq. crank_nicolson is read
as the theta-scheme, theta = 1/2 giving T_2):
  (I - theta dt L_h) F^{n+1} = (I + (1-theta) dt L_h) F^n + dt (theta b^{n+1} + (1-theta) b^n).
It is solved two ways: ``theta_step_direct`` (global sparse LU, the plain
definition) and ``theta_step_sweep`` (cell blocks in topological levels of the
upwind dependency graph, Sec. 4.1-4.2).

Dependency graph (Sec. 4.1): edge L -> R when the face normal n_LR (oriented
from L to R) has n_LR . v > 0 at some Gauss-Lobatto point of the common face.
Levels are the layers of Kahn's algorithm: level = longest upwind path.

Pins (tests/test_oracle_transport.py): L_h 1 + b(1) = 0; L_h p + b(p) =
-v . grad p for p in Q_d; F^T W L_h F <= 0; a hand-derived 1D d=1 example;
the 3x3 dependency-graph levels of the paper's figure; block triangularity in
topological order; sweep == direct solve; the discrete mass identity;
T(-dt) T(dt) = I; exact translation of polynomial profiles.
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# ---------------------------------------------------------------------------
# reference-cell quantities
# ---------------------------------------------------------------------------
def reference_gradients(mesh):
    """grad[i, j, k] = d/dxhat_k of phihat_i at xhat_j.

    For the tensor Lagrange basis phihat_i(xhat) = prod_l l_{i_l}(xhat_l):
    component k is l'_{i_k}(xi_{j_k}) prod_{l != k} delta(i_l, j_l).
    """
    idx = mesh.node_idx
    nd, dim = mesh.nd, mesh.dim
    grad = np.zeros((nd, nd, dim))
    for i in range(nd):
        for j in range(nd):
            for k in range(dim):
                same = all(idx[i, l] == idx[j, l] for l in range(dim) if l != k)
                if same:
                    grad[i, j, k] = mesh.dmat[idx[j, k], idx[i, k]]
    return grad


def reference_faces(mesh):
    """List of faces eps = (axis, side, nhat, on_face mask, mu)."""
    out = []
    idx = mesh.node_idx
    for axis in range(mesh.dim):
        for side in (-1, 1):
            nhat = np.zeros(mesh.dim)
            nhat[axis] = side
            target = mesh.degree if side > 0 else 0
            on = idx[:, axis] == target
            mu = np.zeros(mesh.nd)
            for i in np.nonzero(on)[0]:
                mu[i] = np.prod([mesh.wi[idx[i, l]] for l in range(mesh.dim) if l != axis])
            out.append((axis, side, nhat, on, mu))
    return out


def _cofactor(jac):
    """co(A) = det(A) (A^{-1})^T, batched (eq. co_mat)."""
    det = np.linalg.det(jac)
    return det[:, None, None] * np.transpose(np.linalg.inv(jac), (0, 2, 1)), det


# ---------------------------------------------------------------------------
# per-cell blocks
# ---------------------------------------------------------------------------
class CellBlocks:
    """Gamma_{L<-L} and the upwind couplings of a batch of cells.

    Attributes
      cells   : (N,) flat cell indices
      gll     : (N, nd, nd) Gamma_{L<-L}
      faces   : list of dicts, one per reference face eps, with
                nbr   (N,)     neighbour cell or -1 on the boundary
                nodes (nf,)    node indices i of the face
                partner (N,nf) matching node index i' in the neighbour (-1 on the boundary)
                coef  (N, nf)  (1/omega_{L,i}) mu_i (v . c nhat)^-   (<= 0)
    """


def cell_blocks(mesh, v, cells, grad=None, rfaces=None):
    v = np.asarray(v, dtype=float).reshape(mesh.dim)
    cells = np.asarray(cells, dtype=np.int64)
    if grad is None:
        grad = reference_gradients(mesh)
    if rfaces is None:
        rfaces = reference_faces(mesh)
    jac = mesh.jacobian(cells)
    cof, det = _cofactor(jac)                                  # (N, D, D), (N,)
    omega = mesh.what[None, :] * det[:, None]                  # omega_{L,i}
    # volume part: v . c gradhat phihat_i(xhat_j)  (c constant on affine cells)
    cv = np.einsum("k,nkl->nl", v, cof)                          # v . c (row form)
    vcg = np.einsum("nl,ijl->nij", cv, grad)                   # v . c gradhat phihat_i(xhat_j)
    gll = -(vcg * mesh.what[None, None, :]) / omega[:, :, None]
    coords = mesh.node_coords(cells)
    faces = []
    for axis, side, nhat, on, mu in rfaces:
        vn = np.einsum("nkl,l,k->n", cof, nhat, v)              # v . c nhat
        plus = np.maximum(vn, 0.0)
        minus = np.minimum(vn, 0.0)
        nodes = np.nonzero(on)[0]
        diag = (mu[None, :] * plus[:, None]) / omega
        gll[:, np.arange(mesh.nd), np.arange(mesh.nd)] += diag
        coef = (mu[nodes][None, :] * minus[:, None]) / omega[:, nodes]
        nbr = mesh.neighbour(cells, axis, side)
        partner = np.full((len(cells), len(nodes)), -1, dtype=np.int64)
        inside = nbr >= 0
        if inside.any():
            rcoords = mesh.node_coords(nbr[inside])                         # (M, nd, D)
            lc = coords[inside][:, nodes, :]                                 # (M, nf, D)
            dist = np.linalg.norm(lc[:, :, None, :] - rcoords[:, None, :, :], axis=3)
            best = np.argmin(dist, axis=2)
            if np.max(np.take_along_axis(dist, best[:, :, None], axis=2)) > 1e-9 * np.min(mesh.h):
                raise RuntimeError("non-conformal face: no matching Gauss-Lobatto point")
            partner[inside] = best
        faces.append(dict(axis=axis, side=side, nbr=nbr, nodes=nodes, partner=partner,
                          coef=coef, vn=vn))
    blk = CellBlocks()
    blk.cells, blk.gll, blk.faces, blk.omega = cells, gll, faces, omega
    return blk


# ---------------------------------------------------------------------------
# inflow boundary entries (fictitious cells)
# ---------------------------------------------------------------------------
def inflow_entries(mesh, v):
    """Boundary coupling entries of velocity v.

    Returns dict with arrays cell, node, face (index into reference_faces),
    coef ((1/omega) mu (v.c n)^-, < 0) and coords (E, D) of the boundary GL
    points at which f^b is needed.  One entry per (cell, node, boundary face)
    with a non-zero inflow coefficient.
    """
    multi = mesh.cell_multi(np.arange(mesh.nc))
    on_bnd = np.zeros(mesh.nc, dtype=bool)
    for k in range(mesh.dim):
        on_bnd |= (multi[:, k] == 0) | (multi[:, k] == mesh.n[k] - 1)
    blk = cell_blocks(mesh, v, np.nonzero(on_bnd)[0])
    cells, nodes, faces, coefs = [], [], [], []
    for e, fc in enumerate(blk.faces):
        bnd = fc["nbr"] < 0
        for col, i in enumerate(fc["nodes"]):
            sel = bnd & (fc["coef"][:, col] != 0.0)
            c = blk.cells[sel]
            cells.append(c)
            nodes.append(np.full(c.size, i, dtype=np.int64))
            faces.append(np.full(c.size, e, dtype=np.int64))
            coefs.append(fc["coef"][sel, col])
    cell = np.concatenate(cells) if cells else np.zeros(0, np.int64)
    node = np.concatenate(nodes) if nodes else np.zeros(0, np.int64)
    face = np.concatenate(faces) if faces else np.zeros(0, np.int64)
    coef = np.concatenate(coefs) if coefs else np.zeros(0)
    coords = mesh.node_coords(cell)[np.arange(cell.size), node] if cell.size else np.zeros((0, mesh.dim))
    return dict(cell=cell, node=node, face=face, coef=coef, coords=coords)


# ---------------------------------------------------------------------------
# global matrix (eq. linear_ODE)
# ---------------------------------------------------------------------------
def assemble(mesh, v):
    """Return (L_h, Bb, entries): d/dt F = L_h F + Bb fb.

    F is indexed cell * nd + node; fb holds one value per inflow entry (see
    ``inflow_entries``).  Only for small meshes.
    """
    nd, nc = mesh.nd, mesh.nc
    blk = cell_blocks(mesh, v, np.arange(nc))
    rows, cols, vals = [], [], []
    base = np.arange(nc)[:, None, None] * nd
    ii = np.broadcast_to(np.arange(nd)[None, :, None], (nc, nd, nd))
    jj = np.broadcast_to(np.arange(nd)[None, None, :], (nc, nd, nd))
    rows.append((base + ii).ravel())
    cols.append((base + jj).ravel())
    vals.append(-blk.gll.ravel())
    for fc in blk.faces:
        inside = fc["nbr"] >= 0
        for col, i in enumerate(fc["nodes"]):
            sel = inside & (fc["coef"][:, col] != 0.0)
            rows.append(blk.cells[sel] * nd + i)
            cols.append(fc["nbr"][sel] * nd + fc["partner"][sel, col])
            vals.append(-fc["coef"][sel, col])
    lh = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(nc * nd, nc * nd))
    ent = inflow_entries(mesh, v)
    bb = sp.csr_matrix((-ent["coef"], (ent["cell"] * nd + ent["node"], np.arange(ent["cell"].size))),
                       shape=(nc * nd, ent["cell"].size))
    return lh, bb, ent


def theta_step_direct(mesh, v, f_old, fb_old, fb_new, dt, theta):
    """Theta-scheme transport step by a global sparse direct solve.

    f_old: (m, nc, nd); fb_old, fb_new: (m, E) inflow values per entry.
    """
    lh, bb, _ = assemble(mesh, v)
    n = mesh.nc * mesh.nd
    eye = sp.identity(n, format="csr")
    lhs = (eye - theta * dt * lh).tocsc()
    rhs_op = eye + (1.0 - theta) * dt * lh
    f_old = np.asarray(f_old, dtype=float)
    out = np.empty_like(f_old)
    lu = spla.splu(lhs)
    for k in range(f_old.shape[0]):
        rhs = rhs_op @ f_old[k].ravel() + dt * (bb @ (theta * fb_new[k] + (1.0 - theta) * fb_old[k]))
        out[k] = lu.solve(rhs).reshape(mesh.nc, mesh.nd)
    return out


# ---------------------------------------------------------------------------
# dependency graph and topological levels (Sec. 4.1)
# ---------------------------------------------------------------------------
def dependency_edges(mesh, v):
    """Edges (L, R) with n_LR . v > 0 at some GL point of the common face."""
    cells = np.arange(mesh.nc)
    blk = cell_blocks(mesh, v, cells)
    src, dst = [], []
    for fc in blk.faces:
        inside = fc["nbr"] >= 0
        out_flow = fc["vn"] > 0.0          # n_LR . v, constant on an affine face
        sel = inside & out_flow
        src.append(cells[sel])
        dst.append(fc["nbr"][sel])
    return np.concatenate(src), np.concatenate(dst)


def topological_levels(mesh, v):
    """Kahn's algorithm by layers; returns level[cell].  Raises on a cycle."""
    src, dst = dependency_edges(mesh, v)
    nc = mesh.nc
    indeg = np.bincount(dst, minlength=nc)
    order = np.argsort(src, kind="stable")
    src_s, dst_s = src[order], dst[order]
    start = np.searchsorted(src_s, np.arange(nc + 1))
    level = np.full(nc, -1, dtype=np.int64)
    frontier = np.nonzero(indeg == 0)[0]
    lev = 0
    done = 0
    while frontier.size:
        level[frontier] = lev
        done += frontier.size
        targets = np.concatenate([dst_s[start[c]:start[c + 1]] for c in frontier]) \
            if frontier.size else np.zeros(0, np.int64)
        np.subtract.at(indeg, targets, 1)
        cand = np.unique(targets)
        frontier = cand[indeg[cand] == 0]
        lev += 1
    if done != nc:
        raise ValueError("dependency graph has a cycle")
    return level


# ---------------------------------------------------------------------------
# level sweep
# ---------------------------------------------------------------------------
def theta_step_sweep(mesh, v, f_old, fb_old, fb_new, dt, theta, levels=None):
    """Theta-scheme transport step solved cell block by cell block.

    Cells are visited level by level; each cell solves
      (I + theta dt G_LL) x_L = (I - (1-theta) dt G_LL) f_L^n
                                - dt sum_R G_LR [theta x_R + (1-theta) f_R^n]
    with x_R already known for every upwind R (and f^b on the boundary),
    using numpy.linalg.solve on the block itself (no stored inverse).
    f_old: (m, nc, nd); fb_*: (m, E) per inflow entry of ``inflow_entries``.
    """
    f_old = np.asarray(f_old, dtype=float)
    m, nc, nd = f_old.shape
    if levels is None:
        levels = topological_levels(mesh, v)
    ent = inflow_entries(mesh, v)
    # boundary value lookup: (cell, node, face) -> entry index
    bkey = {(int(c), int(n), int(e)): k
            for k, (c, n, e) in enumerate(zip(ent["cell"], ent["node"], ent["face"]))}
    grad = reference_gradients(mesh)
    rfaces = reference_faces(mesh)
    f_new = np.zeros_like(f_old)
    solved = np.zeros(nc, dtype=bool)
    eye = np.eye(nd)
    order = np.argsort(levels, kind="stable")
    bounds = np.searchsorted(levels[order], np.arange(levels.max() + 2))
    for lev in range(levels.max() + 1):
        cells = order[bounds[lev]:bounds[lev + 1]]
        blk = cell_blocks(mesh, v, cells, grad, rfaces)
        a = eye[None] + theta * dt * blk.gll
        bmat = eye[None] - (1.0 - theta) * dt * blk.gll
        rhs = np.einsum("nij,knj->kni", bmat, f_old[:, cells, :])
        for e, fc in enumerate(blk.faces):
            for col, i in enumerate(fc["nodes"]):
                coef = fc["coef"][:, col]
                nz = coef != 0.0
                if not nz.any():
                    continue
                inside = nz & (fc["nbr"] >= 0)
                if inside.any():
                    r = fc["nbr"][inside]
                    ip = fc["partner"][inside, col]
                    if not solved[r].all():
                        raise RuntimeError("upwind cell not solved before its downwind cell")
                    up_new = f_new[:, r, ip]
                    rhs[:, inside, i] -= dt * coef[inside] * (theta * up_new + (1.0 - theta) * f_old[:, r, ip])
                bnd = nz & (fc["nbr"] < 0)
                if bnd.any():
                    idx = np.array([bkey[(int(c), int(i), e)] for c in cells[bnd]])
                    rhs[:, bnd, i] -= dt * coef[bnd] * (theta * fb_new[:, idx] + (1.0 - theta) * fb_old[:, idx])
        sol = np.linalg.solve(a[None], rhs[..., None])[..., 0]   # (m, N, nd)
        f_new[:, cells, :] = sol
        solved[cells] = True
    return f_new
