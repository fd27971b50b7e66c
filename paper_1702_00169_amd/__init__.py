"""Python binding of the PDG transport-sweep + relaxation library (``libpdg.so``).

A thin ctypes layer over the C ABI of ``include/pdg.h``: every entry point
keeps its C name, arguments are marshalled (torch tensors become device
pointers, ``torch.cuda.current_stream()`` the stream) and every step of the
method runs in the HIP library.  There is no fallback: if the library has
not been built, importing this package raises.

Layouts are those of the header: f[v][k][j][c] per instance, j the
Gauss-Lobatto tensor index (x fastest), c the cell index (x fastest).
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libpdg.so")

PDG_OK, PDG_EINVAL, PDG_EUNSUPPORTED, PDG_ENOTDAG, PDG_ESINGULAR, PDG_ENOMEM, PDG_EDEVICE, PDG_ESTATE = range(8)
PDG_FP64, PDG_FP32, PDG_FP32_REFINE, PDG_FP32_REFINE_P48 = 0, 1, 2, 3
# bytes of one state value per precision (the 48-bit state: a binary32 plane, then an int16 plane)
STATE_BYTES = {PDG_FP64: 8, PDG_FP32: 4, PDG_FP32_REFINE: 8, PDG_FP32_REFINE_P48: 6}
PDG_FEQ_ADVECTION, PDG_FEQ_EULER, PDG_FEQ_D2Q9 = 0, 1, 2
PDG_LIE, PDG_STRANG, PDG_STRANG_COLLAPSED, PDG_KIN, PDG_KIN4 = 0, 1, 2, 3, 4

EXPORTED = ("pdg_setup_mesh", "pdg_layout", "pdg_node_coords", "pdg_levels", "pdg_topo_levels", "pdg_line_operator", "pdg_cell_operator",
            "pdg_prepare", "pdg_equilibrium", "pdg_state_to_f64", "pdg_state_from_f64", "pdg_inflow_equilibrium", "pdg_transport_sweep", "pdg_transport_sweep_static",
            "pdg_relax", "pdg_source", "pdg_step", "pdg_autotune", "pdg_get_tiles", "pdg_set_tiles", "pdg_last_refine_correction", "pdg_sync_status", "pdg_status_string", "pdg_error_detail", "pdg_destroy")


class PdgError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        detail = pdg_error_detail() if status in (PDG_EDEVICE, PDG_ENOMEM) else ""
        super().__init__(f"{where}: {pdg_status_string(status)}" + (f" [{detail}]" if detail else ""))


class pdg_instance_desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("degree", ctypes.c_int32),
                ("nv", ctypes.c_int32), ("m", ctypes.c_int32), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("v", ctypes.POINTER(ctypes.c_double)),
                ("feq", ctypes.c_int32), ("feq_param", ctypes.c_double * 4),
                ("edges", ctypes.POINTER(ctypes.c_double) * 3), ("axes", ctypes.c_double * 9)]


def _load():
    # torch ships its own HIP runtime (soname libamdhip64.so.7).  Importing it
    # first makes the dynamic linker bind libpdg.so to that same runtime, so
    # the process holds one HIP/HSA runtime and torch tensors, streams and the
    # library's launches share one device context.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1702_00169_amd/build.py` "
                          "(the library has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    p, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "pdg_setup_mesh": (i32, [ctypes.POINTER(pdg_instance_desc), i32, ctypes.POINTER(p)]),
        "pdg_layout": (i32, [p, p, p, p, p, p, p]),
        "pdg_node_coords": (i32, [p, i32, p, p]),
        "pdg_levels": (i32, [p, i32, i32, p]),
        "pdg_topo_levels": (i32, [i32, i64, p, p, p]),
        "pdg_line_operator": (i32, [p, i32, i32, p, ctypes.POINTER(d)]),
        "pdg_cell_operator": (i32, [p, i32, i32, p, p]),
        "pdg_prepare": (i32, [p, d, d, d, i32, i32, p]),
        "pdg_equilibrium": (i32, [p, p, p, p]),
        "pdg_state_to_f64": (i32, [p, p, p, p]),
        "pdg_state_from_f64": (i32, [p, p, p, p]),
        "pdg_inflow_equilibrium": (i32, [p, p, p, p]),
        "pdg_transport_sweep": (i32, [p, p, p, p, d, p]),
        "pdg_transport_sweep_static": (i32, [p, p, p, p, d, p]),
        "pdg_relax": (i32, [p, p, p, p]),
        "pdg_source": (i32, [p, p, d, p]),
        "pdg_step": (i32, [p, p, p, i32, p]),
        "pdg_autotune": (i32, [p, p, p, i32, p]),
        "pdg_get_tiles": (i32, [p, ctypes.POINTER(i32), p]),
        "pdg_set_tiles": (i32, [p, i32, p]),
        "pdg_last_refine_correction": (i32, [p, ctypes.POINTER(d)]),
        "pdg_sync_status": (i32, [p]),
        "pdg_status_string": (ctypes.c_char_p, [i32]),
        "pdg_error_detail": (ctypes.c_char_p, []),
        "pdg_destroy": (None, [p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def pdg_status_string(status):
    return _lib.pdg_status_string(int(status)).decode()


def pdg_error_detail():
    return _lib.pdg_error_detail().decode()


def _check(status, where):
    if status != PDG_OK:
        raise PdgError(status, where)


def _ptr(t):
    """Device (or host numpy) pointer of a tensor/array; None stays NULL."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return ctypes.c_void_p(t.data_ptr())
    return t.ctypes.data_as(ctypes.c_void_p)


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------------------
# C-named entry points
# ---------------------------------------------------------------------------
def pdg_setup_mesh(instances):
    """instances: list of dicts with dim, n, degree, v (nv x dim), m, lo, hi,
    feq ('advection'|'euler'|'d2q9'), feq_param and optionally edges (per
    axis None or n[k] + 1 cell edges) or axes (D x D array whose column k is
    the cell edge vector a_k of a uniform affine lattice).  Returns an opaque
    context handle."""
    import numpy as np
    arr = (pdg_instance_desc * len(instances))()
    keep = []
    for i, ins in enumerate(instances):
        v = np.ascontiguousarray(np.asarray(ins["v"], dtype=np.float64))
        keep.append(v)
        dim = int(ins["dim"])
        n = (list(ins["n"]) + [1, 1, 1])[:3]
        lo = (list(ins.get("lo", [0.0] * 3)) + [0.0] * 3)[:3]
        hi = (list(ins.get("hi", [1.0] * 3)) + [1.0] * 3)[:3]
        par = (list(ins.get("feq_param", [])) + [0.0] * 4)[:4]
        feq = ins.get("feq", "advection")
        feq = {"advection": PDG_FEQ_ADVECTION, "euler": PDG_FEQ_EULER, "d2q9": PDG_FEQ_D2Q9}.get(feq, feq)
        nv = v.shape[0] if v.ndim == 2 else 0
        # optional per-axis cell edges (graded mesh); None = uniform on [lo, hi]
        edges = (list(ins.get("edges") or []) + [None] * 3)[:3]
        eptr = (ctypes.POINTER(ctypes.c_double) * 3)()
        for k, e in enumerate(edges):
            if e is not None:
                e = np.ascontiguousarray(np.asarray(e, dtype=np.float64))
                keep.append(e)
                eptr[k] = e.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        ax9 = [0.0] * 9
        if ins.get("axes") is not None:
            a = np.asarray(ins["axes"], dtype=np.float64).reshape(dim, dim)
            for k in range(dim):
                for r in range(dim):
                    ax9[3 * k + r] = float(a[r, k])
        arr[i] = pdg_instance_desc(dim, (ctypes.c_int32 * 3)(*n), int(ins["degree"]), nv, int(ins["m"]),
                                   (ctypes.c_double * 3)(*lo), (ctypes.c_double * 3)(*hi),
                                   v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(feq),
                                   (ctypes.c_double * 4)(*par), eptr, (ctypes.c_double * 9)(*ax9))
    ctx = ctypes.c_void_p()
    _check(_lib.pdg_setup_mesh(arr, len(instances), ctypes.byref(ctx)), "pdg_setup_mesh")
    return ctx


def pdg_layout(ctx, n_inst):
    import numpy as np
    fe, we, be = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    fo = np.zeros(n_inst + 1, np.int64)
    wo = np.zeros(n_inst + 1, np.int64)
    bo = np.zeros(n_inst + 1, np.int64)
    _check(_lib.pdg_layout(ctx, ctypes.byref(fe), ctypes.byref(we), ctypes.byref(be), _ptr(fo), _ptr(wo),
                           _ptr(bo)), "pdg_layout")
    return dict(f_elems=fe.value, w_elems=we.value, fb_elems=be.value, f_off=fo, w_off=wo, fb_off=bo)


def pdg_node_coords(ctx, inst, vol_xyz, inflow_xyz):
    _check(_lib.pdg_node_coords(ctx, int(inst), _ptr(vol_xyz), _ptr(inflow_xyz)), "pdg_node_coords")


def pdg_levels(ctx, inst, vel, level):
    _check(_lib.pdg_levels(ctx, int(inst), int(vel), _ptr(level)), "pdg_levels")


def pdg_topo_levels(n_nodes, src, dst, level):
    """Returns the status (PDG_OK or PDG_ENOTDAG) instead of raising."""
    return _lib.pdg_topo_levels(int(n_nodes), int(len(src)), _ptr(src), _ptr(dst), _ptr(level))


def pdg_line_operator(ctx, inst, vel, gamma):
    kappa = ctypes.c_double()
    _check(_lib.pdg_line_operator(ctx, int(inst), int(vel), _ptr(gamma), ctypes.byref(kappa)), "pdg_line_operator")
    return kappa.value


def pdg_cell_operator(ctx, inst, vel, gamma, kappa):
    _check(_lib.pdg_cell_operator(ctx, int(inst), int(vel), _ptr(gamma), _ptr(kappa)), "pdg_cell_operator")


def pdg_prepare(ctx, dt, theta, omega, scheme, precision, stream=None):
    _check(_lib.pdg_prepare(ctx, float(dt), float(theta), float(omega), int(scheme), int(precision),
                            _stream(stream)), "pdg_prepare")


def pdg_equilibrium(ctx, w, f, stream=None):
    _check(_lib.pdg_equilibrium(ctx, _ptr(w), _ptr(f), _stream(stream)), "pdg_equilibrium")


def pdg_state_to_f64(ctx, f, x, stream=None):
    _check(_lib.pdg_state_to_f64(ctx, _ptr(f), _ptr(x), _stream(stream)), "pdg_state_to_f64")


def pdg_state_from_f64(ctx, x, f, stream=None):
    _check(_lib.pdg_state_from_f64(ctx, _ptr(x), _ptr(f), _stream(stream)), "pdg_state_from_f64")


def pdg_inflow_equilibrium(ctx, w_inflow, fb, stream=None):
    _check(_lib.pdg_inflow_equilibrium(ctx, _ptr(w_inflow), _ptr(fb), _stream(stream)), "pdg_inflow_equilibrium")


def pdg_transport_sweep(ctx, f, fb_old, fb_new, dt_sub, stream=None):
    _check(_lib.pdg_transport_sweep(ctx, _ptr(f), _ptr(fb_old), _ptr(fb_new), float(dt_sub), _stream(stream)),
           "pdg_transport_sweep")


def pdg_transport_sweep_static(ctx, f, fb_old, fb_new, dt_sub, stream=None):
    _check(_lib.pdg_transport_sweep_static(ctx, _ptr(f), _ptr(fb_old), _ptr(fb_new), float(dt_sub),
                                           _stream(stream)), "pdg_transport_sweep_static")


def pdg_relax(ctx, f, w_out=None, stream=None):
    _check(_lib.pdg_relax(ctx, _ptr(f), _ptr(w_out), _stream(stream)), "pdg_relax")


def pdg_source(ctx, f, h, stream=None):
    _check(_lib.pdg_source(ctx, _ptr(f), float(h), _stream(stream)), "pdg_source")


def pdg_step(ctx, f, fb, n_steps, stream=None):
    _check(_lib.pdg_step(ctx, _ptr(f), _ptr(fb), int(n_steps), _stream(stream)), "pdg_step")


def pdg_autotune(ctx, f_scratch, fb, reps=3, stream=None):
    _check(_lib.pdg_autotune(ctx, _ptr(f_scratch), _ptr(fb), int(reps), _stream(stream)), "pdg_autotune")


def pdg_get_tiles(ctx):
    """List of dicts {np, x_kind, C, S}, one per launch class."""
    import numpy as np
    n = ctypes.c_int32(0)
    _check(_lib.pdg_get_tiles(ctx, ctypes.byref(n), None), "pdg_get_tiles")
    buf = np.zeros(4 * max(1, n.value), np.int32)
    _check(_lib.pdg_get_tiles(ctx, ctypes.byref(n), _ptr(buf)), "pdg_get_tiles")
    return [dict(np=int(buf[4 * i]), x_kind=int(buf[4 * i + 1]), C=int(buf[4 * i + 2]), S=int(buf[4 * i + 3]))
            for i in range(n.value)]


def pdg_set_tiles(ctx, tiles):
    import numpy as np
    buf = np.array([[t["np"], t["x_kind"], t["C"], t["S"]] for t in tiles], np.int32).ravel()
    _check(_lib.pdg_set_tiles(ctx, len(tiles), _ptr(buf)), "pdg_set_tiles")


def pdg_last_refine_correction(ctx):
    out = ctypes.c_double()
    _check(_lib.pdg_last_refine_correction(ctx, ctypes.byref(out)), "pdg_last_refine_correction")
    return out.value


def pdg_sync_status(ctx):
    _check(_lib.pdg_sync_status(ctx), "pdg_sync_status")


def pdg_destroy(ctx):
    if ctx is not None and ctx.value:
        _lib.pdg_destroy(ctx)


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------
class Problem:
    """Owns a context for a list of instances (dicts as for pdg_setup_mesh)."""

    def __init__(self, instances):
        self.instances = list(instances)
        self.ctx = pdg_setup_mesh(self.instances)
        self.layout = pdg_layout(self.ctx, len(self.instances))

    def close(self):
        pdg_destroy(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def node_coords(self, i):
        import numpy as np
        ins = self.instances[i]
        dim = int(ins["dim"])
        nc = int(np.prod(ins["n"][:dim]))
        nd = (int(ins["degree"]) + 1) ** dim
        vol = np.zeros((dim, nd, nc))
        nb = (self.layout["fb_off"][i + 1] - self.layout["fb_off"][i]) // int(ins["m"])
        inflow = np.zeros(dim * nb)
        pdg_node_coords(self.ctx, i, vol, inflow)
        return vol, inflow

    def prepare(self, dt, theta=0.5, omega=2.0, scheme=PDG_STRANG_COLLAPSED, precision=PDG_FP64, stream=None):
        pdg_prepare(self.ctx, dt, theta, omega, scheme, precision, stream)
        self.dt = dt
        self.precision = precision

    def equilibrium(self, w, f, stream=None):
        pdg_equilibrium(self.ctx, w, f, stream)

    def new_state(self):
        """An uninitialised device buffer for f in the prepared precision
        (binary64 / binary32 elements; for the 48-bit state, 6 bytes per value
        as int16 triples holding the binary32 plane and then the int16 plane)."""
        import torch
        n = self.layout["f_elems"]
        if self.precision == PDG_FP32_REFINE_P48:
            return torch.empty(3 * n, dtype=torch.int16, device="cuda")
        return torch.empty(n, dtype=torch.float32 if self.precision == PDG_FP32 else torch.float64, device="cuda")

    def state_to_f64(self, f, x=None, stream=None):
        """Binary64 copy of the state (x: optional device float64 tensor)."""
        import torch
        if x is None:
            x = torch.empty(self.layout["f_elems"], dtype=torch.float64, device="cuda")
        pdg_state_to_f64(self.ctx, f, x, stream)
        return x

    def state_from_f64(self, x, f, stream=None):
        pdg_state_from_f64(self.ctx, x, f, stream)

    def inflow_equilibrium(self, w_inflow, fb, stream=None):
        pdg_inflow_equilibrium(self.ctx, w_inflow, fb, stream)

    def transport_sweep(self, f, fb_old, fb_new, dt_sub, stream=None):
        pdg_transport_sweep(self.ctx, f, fb_old, fb_new, dt_sub, stream)

    def relax(self, f, w_out=None, stream=None):
        pdg_relax(self.ctx, f, w_out, stream)

    def source(self, f, h, stream=None):
        pdg_source(self.ctx, f, h, stream)

    def step(self, f, fb, n_steps, stream=None):
        pdg_step(self.ctx, f, fb, n_steps, stream)

    def autotune(self, f_scratch, fb, reps=3, stream=None):
        pdg_autotune(self.ctx, f_scratch, fb, reps, stream)
        return pdg_get_tiles(self.ctx)

    def tiles(self):
        return pdg_get_tiles(self.ctx)

    def set_tiles(self, tiles):
        pdg_set_tiles(self.ctx, tiles)

    def sync_status(self):
        pdg_sync_status(self.ctx)

    def last_refine_correction(self):
        return pdg_last_refine_correction(self.ctx)
