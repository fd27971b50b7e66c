"""Shared test plumbing: build matching GPU and oracle problems from a
``workloads.Instance`` and move data between the two layouts.

GPU layout (library):  f[v][k][j][c] per instance (node-major).
Oracle layout:         f[v][k][c][j] per instance (cell-major).
Both sides evaluate the seeded w_0(x) of ``workloads`` at their own
Gauss-Lobatto points; nothing computed by one side is fed to the other.
"""
import numpy as np

from oracle import step as ost


def inst_dict(inst):
    if inst.feq_kind == "advection":
        par = list(inst.feq_param["a"])
    elif inst.feq_kind == "d2q9":
        par = [inst.feq_param["g"]]
    else:
        par = [inst.feq_param["gamma"]]
    return dict(dim=inst.dim, n=list(inst.n), degree=inst.degree, v=np.asarray(inst.vel, float), m=inst.m,
                lo=list(inst.lo), hi=list(inst.hi), feq=inst.feq_kind, feq_param=par,
                edges=getattr(inst, "edges", None), axes=getattr(inst, "axes", None))


def oracle_problem(inst):
    edges = getattr(inst, "edges", None)
    if edges is not None:
        edges = [np.asarray(e, float) if e is not None else np.linspace(inst.lo[k], inst.hi[k], inst.n[k] + 1)
                 for k, e in enumerate(edges)]
    return ost.Problem(inst.n, inst.lo, inst.hi, inst.degree, inst.vel, inst.m, inst.feq_kind, inst.feq_param,
                       edges, getattr(inst, "axes", None))


def sizes(inst):
    nc = int(np.prod(inst.n))
    nd = (inst.degree + 1) ** inst.dim
    return nc, nd


def index_velocity(inst, v):
    """Velocity v in the frame of the cell index axes: A^{-1} v on an affine
    lattice of edge vectors A (columns), v itself on a box mesh."""
    axes = getattr(inst, "axes", None)
    vel = np.asarray(inst.vel[v], float)
    if axes is None:
        return vel
    vt = np.linalg.solve(np.asarray(axes, float), vel)
    return np.where(np.abs(vt) <= 1e-13 * np.max(np.abs(vt)), 0.0, vt)   # rounding-level components are zero


def inflow_faces(inst, v):
    """[(axis, tnodes, ntc)] of the inflow face blocks of velocity v (one per
    non-zero component in the index frame, increasing axis)."""
    nc, _ = sizes(inst)
    tn = (inst.degree + 1) ** (inst.dim - 1)
    vt = index_velocity(inst, v)
    return [(a, tn, nc // inst.n[a]) for a in range(inst.dim) if vt[a] != 0]


def gpu_inflow_points(prob, i, inst):
    """Per velocity, the list of (npts, D) coordinate arrays of its face blocks."""
    _, inflow = prob.node_coords(i)
    out = []
    off = 0
    for v in range(inst.vel.shape[0]):
        faces = []
        for a, tn, ntc in inflow_faces(inst, v):
            blk = inflow[off:off + inst.dim * tn * ntc].reshape(inst.dim, tn * ntc)
            faces.append(blk.T.copy())
            off += inst.dim * tn * ntc
        out.append(faces)
    return out


def gpu_fb_from_function(prob, insts, fn_of_inst_v):
    """fb (numpy, fb layout [v][k][face][t][tau]) with value fn(i, v, pts) -> (m, npts)."""
    fb = np.zeros(prob.layout["fb_elems"])
    for i, inst in enumerate(insts):
        off = prob.layout["fb_off"][i]
        for v, faces in enumerate(gpu_inflow_points(prob, i, inst)):
            if not faces:
                continue
            vals = [fn_of_inst_v(i, v, pts) for pts in faces]   # each (m, npts_face)
            blk = np.concatenate(vals, axis=1)                  # (m, sum npts)
            fb[off:off + blk.size] = blk.ravel()
            off += blk.size
    return fb


def oracle_fb_from_function(oprob, i, fn_of_inst_v):
    return [fn_of_inst_v(i, v, oprob.entries(v)["coords"]) for v in range(oprob.nv)]


def gpu_w_inflow_from_function(prob, insts, fn_of_inst_v, nw):
    """w_inflow (numpy) for pdg_inflow_equilibrium: per instance and velocity,
    nw blocks of the velocity's inflow points; fn(i, v, pts) -> (nw_i, npts)."""
    blocks = []
    for i, inst in enumerate(insts):
        for v, faces in enumerate(gpu_inflow_points(prob, i, inst)):
            if not faces:
                continue
            vals = [fn_of_inst_v(i, v, pts) for pts in faces]
            blocks.append(np.concatenate(vals, axis=1).ravel())
    return np.concatenate(blocks) if blocks else np.zeros(0)


def gpu_to_oracle(f_flat, inst, f_off=0):
    nc, nd = sizes(inst)
    nv, m = inst.vel.shape[0], inst.m
    blk = np.asarray(f_flat[f_off:f_off + nv * m * nd * nc]).reshape(nv, m, nd, nc)
    return np.transpose(blk, (0, 1, 3, 2)).copy()


def oracle_to_gpu(f_or):
    return np.ascontiguousarray(np.transpose(f_or, (0, 1, 3, 2))).ravel()


def rel_errors(got, want):
    got = np.asarray(got, float)
    want = np.asarray(want, float)
    l2 = np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)
    mx = np.max(np.abs(got - want)) / max(np.max(np.abs(want)), 1e-300)
    return l2, mx


def gpu_initial_state(prob, insts, torch, dtype):
    """f = f^eq(w0), fb = f^eq(w0 on the inflow points), built by the library
    (w0 gives m moments per point, or 3 for the D2Q9 model)."""
    w = np.zeros(prob.layout["w_elems"])
    for i, inst in enumerate(insts):
        vol, _ = prob.node_coords(i)
        pts = vol.reshape(inst.dim, -1).T
        vals = inst.w0(pts)                            # (m, nd*nc)
        w[prob.layout["w_off"][i]:prob.layout["w_off"][i + 1]] = vals.ravel()
    fbw = gpu_w_inflow_from_function(prob, insts, lambda i, v, pts: insts[i].w0(pts), None)
    dev = "cuda"
    w_t = torch.tensor(w, device=dev)
    fbw_t = torch.tensor(fbw, device=dev)
    # dtype None: the prepared precision's own storage (e.g. the 48-bit state)
    f = prob.new_state() if dtype is None else torch.empty(prob.layout["f_elems"], dtype=dtype, device=dev)
    fb = torch.empty(prob.layout["fb_elems"], dtype=torch.float64, device=dev)
    prob.equilibrium(w_t, f)
    prob.inflow_equilibrium(fbw_t, fb)
    torch.cuda.synchronize()
    return f, fb


def oracle_initial_state(oprob, inst):
    x = oprob.mesh.node_coords().reshape(-1, oprob.mesh.dim)
    w = inst.w0(x).reshape(-1, oprob.mesh.nc, oprob.mesh.nd)
    return oprob.feq(w), oprob.inflow_from_w(inst.w0)


def gpu_state(prob, torch, x_flat):
    """Device state in the prepared precision holding the binary64 values
    x_flat (GPU layout), written by the library's conversion."""
    f = prob.new_state()
    prob.state_from_f64(torch.as_tensor(np.asarray(x_flat, np.float64), device="cuda"), f)
    return f


def gpu_state_values(prob, f):
    """The state's values as binary64 numpy (GPU layout)."""
    return prob.state_to_f64(f).cpu().numpy()
