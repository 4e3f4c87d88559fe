"""Python binding of libgdg (include/gdg.h): the same entry points, argument
marshalling only.  Every step of the scheme runs in the HIP kernels of
libgdg.so; there is no other code path.  PyTorch supplies device memory (the
workspace) and the stream.

Raises ``GdgError`` when the built library is missing or a call fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgdg.so")

(GDG_OK, GDG_E_INVALID, GDG_E_INADMISSIBLE, GDG_E_CFL, GDG_E_NOMEM, GDG_E_DEVICE, GDG_E_BUDGET,
 GDG_E_BOUNDARY) = (0, -1, -2, -3, -4, -5, -6, -7)
GDG_REQ_PENDING, GDG_REQ_RUNNING, GDG_REQ_DONE, GDG_REQ_FAILED = 0, 1, 2, 3
GDG_BC_PERIODIC, GDG_BC_OUTFLOW, GDG_BC_SLIP, GDG_BC_DIRICHLET, GDG_BC_SUPERSONIC, GDG_BC_INOUTFLOW = 0, 1, 2, 3, 4, 5
GDG_DATA_CONSTANT, GDG_DATA_VORTEX, GDG_DATA_STEP_START = 0, 1, 2
GDG_LOW_ORDER, GDG_HIGH_ORDER, GDG_LIMITED = 0, 1, 2
GDG_FLAG_NO_QUIET_ROWS = 1
GDG_FP64, GDG_MIXED = 0, 1
GDG_SSPRK3, GDG_SSPRK54 = 0, 1
(GDG_FIELD_STATE, GDG_FIELD_EV_N, GDG_FIELD_BOUNDS, GDG_FIELD_UL, GDG_FIELD_DUH,
 GDG_FIELD_U1) = range(6)
_FIELD_PLANES = {GDG_FIELD_EV_N: 1, GDG_FIELD_BOUNDS: 3}

_NAMES = {0: "GDG_OK", -1: "GDG_E_INVALID", -2: "GDG_E_INADMISSIBLE", -3: "GDG_E_CFL",
          -4: "GDG_E_NOMEM", -5: "GDG_E_DEVICE", -6: "GDG_E_BUDGET", -7: "GDG_E_BOUNDARY"}


class GdgError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__("%s%s" % (_NAMES.get(status, str(status)), (": " + msg) if msg else ""))


class gdg_mesh_desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("degree", C.c_int32), ("cells", C.c_int64 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("bc", C.c_int32 * 6),
                ("bc_state", (C.c_double * 5) * 6), ("data_kind", C.c_int32), ("map_degree", C.c_int32),
                ("vortex", C.c_double * 6), ("vertices", C.POINTER(C.c_double)),
                ("bc_cells", C.POINTER(C.c_int8)), ("ucells", C.c_int64), ("npoints", C.c_int64),
                ("ucell_points", C.POINTER(C.c_int64)), ("uface_bc", C.POINTER(C.c_int8)),
                ("continuous", C.c_int32), ("reserved", C.c_int32)]


class gdg_params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("cfl", C.c_double), ("c_ev", C.c_double),
                ("c_k", C.c_double), ("c_r", C.c_double), ("p_r", C.c_double),
                ("limiter_passes", C.c_int32), ("scheme", C.c_int32), ("precision", C.c_int32),
                ("flags", C.c_int32), ("integrator", C.c_int32), ("reserved", C.c_int32)]


class gdg_stats(C.Structure):
    _fields_ = [("t", C.c_double), ("steps", C.c_int64), ("restarts", C.c_int64),
                ("last_dt", C.c_double), ("min_rho", C.c_double), ("min_eps", C.c_double),
                ("total", C.c_double * 5), ("bound_violations", C.c_int64),
                ("limited_pairs", C.c_int64), ("quiet_rows", C.c_int64)]


class gdg_server_desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("degree", C.c_int32), ("precision", C.c_int32),
                ("max_slots", C.c_int32), ("steps_per_graph", C.c_int32), ("solo_dofs", C.c_int32)]


class gdg_request_info(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("t", C.c_double), ("steps", C.c_int64),
                ("restarts", C.c_int64), ("ndofs", C.c_int64), ("submit_s", C.c_double),
                ("admit_s", C.c_double), ("done_s", C.c_double)]


_lib = None
_P = C.c_void_p
_DP = C.POINTER(C.c_double)


def load():
    """Loads libgdg.so; fails loudly if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise GdgError(GDG_E_DEVICE, "libgdg.so not built (run __graft_entry__.build())")
    # torch ships its own HIP runtime under the same soname; loading it first
    # makes libgdg bind to that one runtime instead of a second copy
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    L.gdg_default_params.argtypes = [C.c_int32, C.POINTER(gdg_params)]
    L.gdg_workspace_bytes.argtypes = [C.POINTER(gdg_mesh_desc), C.POINTER(gdg_params),
                                      C.POINTER(C.c_size_t)]
    L.gdg_create.argtypes = [C.POINTER(gdg_mesh_desc), C.POINTER(gdg_params), _P, C.c_size_t, _P,
                             C.POINTER(_P)]
    L.gdg_destroy.argtypes = [_P]
    L.gdg_destroy.restype = None
    L.gdg_num_dofs.argtypes = [_P]
    L.gdg_num_dofs.restype = C.c_int64
    L.gdg_node_coords.argtypes = [_P, _DP]
    L.gdg_upload_state.argtypes = [_P, _P, C.c_int32]
    L.gdg_download_state.argtypes = [_P, _P, C.c_int32]
    L.gdg_step.argtypes = [_P, C.c_double, C.c_double, _DP]
    L.gdg_run_to.argtypes = [_P, C.c_double, C.c_int64, C.POINTER(gdg_stats)]
    L.gdg_stage.argtypes = [_P, C.c_double, _DP]
    L.gdg_read_field.argtypes = [_P, C.c_int32, _P, C.c_int32]
    L.gdg_get_stats.argtypes = [_P, C.POINTER(gdg_stats)]
    L.gdg_profile.argtypes = [_P, C.c_int32]
    L.gdg_profile_read.argtypes = [_P, _DP, C.POINTER(C.c_int64)]
    L.gdg_last_error.argtypes = [_P]
    L.gdg_last_error.restype = C.c_char_p
    L.gdg_server_overhead_bytes.argtypes = [C.POINTER(gdg_server_desc), C.POINTER(C.c_size_t)]
    L.gdg_server_create.argtypes = [C.POINTER(gdg_server_desc), _P, C.c_size_t, _P, C.POINTER(_P)]
    L.gdg_server_submit.argtypes = [_P, C.POINTER(gdg_mesh_desc), C.POINTER(gdg_params), _DP, C.c_double,
                                    C.POINTER(C.c_uint64)]
    L.gdg_server_pump.argtypes = [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.gdg_server_sync.argtypes = [_P]
    L.gdg_server_poll.argtypes = [_P, C.c_uint64, C.POINTER(gdg_request_info)]
    L.gdg_server_result.argtypes = [_P, C.c_uint64, _DP]
    L.gdg_server_destroy.argtypes = [_P]
    L.gdg_server_destroy.restype = None
    L.gdg_server_last_error.argtypes = [_P]
    L.gdg_server_last_error.restype = C.c_char_p
    L.gdg_solve_noalloc.argtypes = [C.POINTER(gdg_mesh_desc), C.POINTER(gdg_params), _P, _P, C.c_double,
                                    C.c_int64, _P, C.POINTER(gdg_stats)]
    for fn in ("gdg_default_params", "gdg_workspace_bytes", "gdg_create", "gdg_node_coords",
               "gdg_upload_state", "gdg_download_state", "gdg_step", "gdg_run_to", "gdg_stage",
               "gdg_read_field", "gdg_get_stats", "gdg_profile", "gdg_profile_read",
               "gdg_server_overhead_bytes", "gdg_server_create", "gdg_server_submit", "gdg_server_pump",
               "gdg_server_sync", "gdg_server_poll", "gdg_server_result", "gdg_solve_noalloc"):
        getattr(L, fn).restype = C.c_int
    _lib = L
    return L


def _check(st, ctx=None):
    if st != GDG_OK:
        msg = load().gdg_last_error(ctx).decode()
        raise GdgError(st, msg)


def mesh_desc(dim, degree, cells, lo, hi, bc, bstate=None, vortex=None, vertices=None,
              bc_cells=None, map_degree=1, continuous=False, step_start_data=False) -> gdg_mesh_desc:
    """bstate: per face the conserved Dirichlet data of the DIRICHLET,
    SUPERSONIC and INOUTFLOW kinds (None, or None entries, elsewhere); vortex:
    (beta, x0_1, x0_2, u_1, u_2, gamma) to take that data from the isentropic
    vortex instead.  vertices: general cells, the lattice's points as an array
    of shape (prod(cells + 1), dim), the first axis fastest; the descriptor
    keeps a reference to its float64 copy (``m._vx``); map_degree 2: curved
    cells, vertices the lattice of 2 cells + 1 points per axis of their
    quadratic maps.  bc_cells: a kind per
    boundary cell face (for each non-periodic box face in order, its cells
    lexicographically over the other axes, the lowest axis fastest).
    step_start_data: the data of those kinds are the node's own state at the
    start of the step (GDG_DATA_STEP_START)."""
    m = gdg_mesh_desc()
    m.dim, m.degree = dim, degree
    m.continuous = 1 if continuous else 0
    if step_start_data:
        m.data_kind = GDG_DATA_STEP_START
    for e in range(3):
        m.cells[e] = int(cells[e]) if e < dim else 1
        m.lo[e] = float(lo[e]) if e < dim else 0.0
        m.hi[e] = float(hi[e]) if e < dim else 1.0
    for f in range(6):
        m.bc[f] = int(bc[f]) if f < 2 * dim else GDG_BC_OUTFLOW
        if bstate is not None and f < 2 * dim and bstate[f] is not None:
            for q, v in enumerate(bstate[f]):
                m.bc_state[f][q] = float(v)
    if vortex is not None:
        m.data_kind = GDG_DATA_VORTEX
        for k, v in enumerate(vortex):
            m.vortex[k] = float(v)
    if vertices is not None:
        vx = np.ascontiguousarray(vertices, dtype=np.float64)
        m.map_degree = int(map_degree)
        npts = int(np.prod([int(map_degree) * int(c) + 1 for c in cells[:dim]]))
        if vx.shape != (npts, dim):
            raise ValueError(f"vertices must have shape ({npts}, {dim})")
        m._vx = vx
        m.vertices = vx.ctypes.data_as(C.POINTER(C.c_double))
    if bc_cells is not None:
        k = np.ascontiguousarray(bc_cells, dtype=np.int8).ravel()
        n = sum(int(np.prod([int(cells[g]) for g in range(dim) if g != f // 2]))
                for f in range(2 * dim) if int(bc[f]) != GDG_BC_PERIODIC)
        if k.size != n:
            raise ValueError(f"bc_cells needs {n} entries, not {k.size}")
        m._bcc = k
        m.bc_cells = k.ctypes.data_as(C.POINTER(C.c_int8))
    return m


def umesh_desc(dim, degree, cell_points, points, face_bc, bstate=None, map_degree=1,
               step_start_data=False) -> gdg_mesh_desc:
    """Unstructured mesh: cell q is the image of the reference cell under its
    map of degree map_degree through points[cell_points[q, v]]; face_bc[q, f]
    is the kind + 8 * data slot of a face on no other cell (0 elsewhere).  The
    descriptor keeps references to its arrays."""
    m = gdg_mesh_desc()
    m.dim, m.degree = dim, degree
    cp = np.ascontiguousarray(cell_points, dtype=np.int64)
    pts = np.ascontiguousarray(points, dtype=np.float64)
    fb = np.ascontiguousarray(face_bc, dtype=np.int8)
    if cp.ndim != 2 or cp.shape[1] != (int(map_degree) + 1) ** dim or pts.ndim != 2 or pts.shape[1] != dim \
            or fb.shape != (cp.shape[0], 2 * dim):
        raise ValueError("unstructured mesh arrays of the wrong shape")
    for e in range(3):
        m.cells[e] = 1
        m.hi[e] = 1.0
    for f in range(6):
        m.bc[f] = GDG_BC_OUTFLOW
        if bstate is not None and f < len(bstate) and bstate[f] is not None:
            for q, v in enumerate(bstate[f]):
                m.bc_state[f][q] = float(v)
    m.map_degree = int(map_degree)
    m.ucells, m.npoints = cp.shape[0], pts.shape[0]
    m._keep = (cp, pts, fb)
    m.vertices = pts.ctypes.data_as(C.POINTER(C.c_double))
    m.ucell_points = cp.ctypes.data_as(C.POINTER(C.c_int64))
    m.uface_bc = fb.ctypes.data_as(C.POINTER(C.c_int8))
    if step_start_data:
        m.data_kind = GDG_DATA_STEP_START
    return m


# -- the C entry points -------------------------------------------------------
def gdg_default_params(degree: int) -> gdg_params:
    p = gdg_params()
    _check(load().gdg_default_params(degree, C.byref(p)))
    return p


def gdg_workspace_bytes(mesh: gdg_mesh_desc, prm: gdg_params) -> int:
    n = C.c_size_t(0)
    _check(load().gdg_workspace_bytes(C.byref(mesh), C.byref(prm), C.byref(n)))
    return n.value


def gdg_create(mesh, prm, workspace_ptr: int, ws_bytes: int, stream_ptr: int):
    ctx = _P()
    _check(load().gdg_create(C.byref(mesh), C.byref(prm), _P(workspace_ptr), ws_bytes,
                             _P(stream_ptr), C.byref(ctx)), None)
    return ctx


def gdg_destroy(ctx):
    load().gdg_destroy(ctx)


def gdg_num_dofs(ctx) -> int:
    return load().gdg_num_dofs(ctx)


def gdg_node_coords(ctx, dim: int) -> np.ndarray:
    x = np.zeros((gdg_num_dofs(ctx), dim))
    _check(load().gdg_node_coords(ctx, x.ctypes.data_as(_DP)), ctx)
    return x


def _ptr(arr):
    """(pointer, is_device) of a C-contiguous float64 numpy array or torch tensor."""
    if isinstance(arr, np.ndarray):
        assert arr.dtype == np.float64 and arr.flags.c_contiguous
        return arr.ctypes.data, 0
    assert arr.dtype.itemsize == 8 and arr.is_contiguous()
    return arr.data_ptr(), int(arr.is_cuda)


def gdg_upload_state(ctx, U):
    p, dev = _ptr(U)
    _check(load().gdg_upload_state(ctx, _P(p), dev), ctx)


def gdg_download_state(ctx, out):
    p, dev = _ptr(out)
    _check(load().gdg_download_state(ctx, _P(p), dev), ctx)
    return out


def gdg_step(ctx, dt_cap: float = 0.0, dt_fixed: float = 0.0) -> float:
    dt = C.c_double(0.0)
    _check(load().gdg_step(ctx, dt_cap, dt_fixed, C.byref(dt)), ctx)
    return dt.value


def gdg_run_to(ctx, t_final: float, max_steps: int = 2 ** 62) -> gdg_stats:
    s = gdg_stats()
    _check(load().gdg_run_to(ctx, t_final, max_steps, C.byref(s)), ctx)
    return s


def gdg_stage(ctx, tau: float = 0.0) -> float:
    t = C.c_double(0.0)
    _check(load().gdg_stage(ctx, tau, C.byref(t)), ctx)
    return t.value


def gdg_read_field(ctx, field: int, out):
    p, dev = _ptr(out)
    _check(load().gdg_read_field(ctx, field, _P(p), dev), ctx)
    return out


def gdg_get_stats(ctx) -> gdg_stats:
    s = gdg_stats()
    _check(load().gdg_get_stats(ctx, C.byref(s)))
    return s


KERNEL_NAMES = ("prim", "sweep1", "sweep2", "limit1", "limit2")


def gdg_profile(ctx, enable: bool):
    _check(load().gdg_profile(ctx, int(bool(enable))), ctx)


def gdg_profile_read(ctx):
    """{kernel name: (summed ms, launches)} since the last gdg_profile()."""
    ms = np.zeros(len(KERNEL_NAMES))
    n = np.zeros(len(KERNEL_NAMES), dtype=np.int64)
    _check(load().gdg_profile_read(ctx, ms.ctypes.data_as(_DP), n.ctypes.data_as(C.POINTER(C.c_int64))), ctx)
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_NAMES)}


def gdg_last_error(ctx) -> str:
    return load().gdg_last_error(ctx).decode()


def gdg_solve_noalloc(mesh, prm, U0, out, t_final: float, max_steps: int = 2 ** 62,
                      stream_ptr: int = 0) -> gdg_stats:
    """The whole solve in the library's static device workspace (no device
    allocation): U0 and out are float64 SoA arrays, numpy or torch (host or
    device)."""
    s = gdg_stats()
    p0, _ = _ptr(U0)
    p1, _ = _ptr(out)
    _check(load().gdg_solve_noalloc(C.byref(mesh), C.byref(prm), _P(p0), _P(p1), t_final, max_steps,
                                    _P(stream_ptr), C.byref(s)), None)
    return s


# -- convenience owner of workspace + context ----------------------------------
class Solver:
    """A context whose device workspace is a torch uint8 tensor on ``device``
    and whose stream is torch's current stream there (or ``stream``)."""

    def __init__(self, dim, degree, cells, lo, hi, bc, params: gdg_params | None = None,
                 device="cuda:0", stream=None, bstate=None, vortex=None, vertices=None, bc_cells=None,
                 map_degree=1, desc=None, continuous=False, step_start_data=False):
        import torch
        self.torch = torch
        self.dim, self.m = dim, dim + 2
        # desc: a ready descriptor (an unstructured mesh's, umesh_desc)
        self.mesh = desc if desc is not None else mesh_desc(dim, degree, cells, lo, hi, bc, bstate, vortex,
                                                            vertices, bc_cells, map_degree, continuous,
                                                            step_start_data)
        self.params = params if params is not None else gdg_default_params(degree)
        self.device = torch.device(device)
        nbytes = gdg_workspace_bytes(self.mesh, self.params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self.ws_ptr = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = gdg_create(self.mesh, self.params, self.ws_ptr, nbytes, self.stream.cuda_stream)
        self.ndofs = gdg_num_dofs(self.ctx)

    @classmethod
    def from_spec(cls, ms, params=None, **kw):
        return cls(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc, params,
                   bstate=getattr(ms, "bstate", None), vortex=getattr(ms, "vortex", None),
                   vertices=getattr(ms, "vertices", None), bc_cells=getattr(ms, "bc_cells", None),
                   map_degree=getattr(ms, "map_degree", 1), **kw)

    @classmethod
    def unstructured(cls, dim, degree, cell_points, points, face_bc, params=None, bstate=None, map_degree=1,
                     step_start_data=False, **kw):
        desc = umesh_desc(dim, degree, cell_points, points, face_bc, bstate, map_degree, step_start_data)
        return cls(dim, degree, None, None, None, None, params, desc=desc, **kw)

    def close(self):
        if getattr(self, "ctx", None):
            gdg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        self.close()

    def coords(self):
        return gdg_node_coords(self.ctx, self.dim)

    def upload(self, U):
        if isinstance(U, np.ndarray):
            U = np.ascontiguousarray(U, dtype=np.float64).reshape(self.m, self.ndofs)
        gdg_upload_state(self.ctx, U)

    def download(self) -> np.ndarray:
        out = np.zeros((self.m, self.ndofs))
        return gdg_download_state(self.ctx, out)

    def step(self, dt_cap=0.0, dt_fixed=0.0) -> float:
        return gdg_step(self.ctx, dt_cap, dt_fixed)

    def run_to(self, t_final, max_steps=2 ** 62):
        return gdg_run_to(self.ctx, t_final, max_steps)

    def stage(self, tau=0.0) -> float:
        return gdg_stage(self.ctx, tau)

    def field(self, field: int) -> np.ndarray:
        planes = _FIELD_PLANES.get(field, self.m)
        out = np.zeros((planes, self.ndofs))
        return gdg_read_field(self.ctx, field, out)

    def stats(self) -> gdg_stats:
        return gdg_get_stats(self.ctx)


# -- serving -------------------------------------------------------------------
def _scheck(st, srv):
    if st != GDG_OK:
        raise GdgError(st, load().gdg_server_last_error(srv).decode())


def server_desc(dim, degree, precision=GDG_FP64, max_slots=64, steps_per_graph=8, solo_dofs=0) -> gdg_server_desc:
    d = gdg_server_desc()
    d.dim, d.degree, d.precision, d.max_slots, d.steps_per_graph = dim, degree, precision, max_slots, steps_per_graph
    d.solo_dofs = solo_dofs
    return d


def gdg_server_overhead_bytes(desc: gdg_server_desc) -> int:
    n = C.c_size_t(0)
    _check(load().gdg_server_overhead_bytes(C.byref(desc), C.byref(n)))
    return n.value


def gdg_server_create(desc, pool_ptr: int, pool_bytes: int, stream_ptr: int):
    srv = _P()
    st = load().gdg_server_create(C.byref(desc), _P(pool_ptr), pool_bytes, _P(stream_ptr), C.byref(srv))
    if st != GDG_OK:
        raise GdgError(st, "server creation failed")
    return srv


def gdg_server_submit(srv, mesh, prm, U0: np.ndarray, t_final: float) -> int:
    U0 = np.ascontiguousarray(U0, dtype=np.float64)
    t = C.c_uint64(0)
    _scheck(load().gdg_server_submit(srv, C.byref(mesh), C.byref(prm), U0.ctypes.data_as(_DP), t_final,
                                     C.byref(t)), srv)
    return t.value


def gdg_server_pump(srv):
    r, p = C.c_int32(0), C.c_int32(0)
    _scheck(load().gdg_server_pump(srv, C.byref(r), C.byref(p)), srv)
    return r.value, p.value


def gdg_server_sync(srv):
    _scheck(load().gdg_server_sync(srv), srv)


def gdg_server_poll(srv, ticket: int) -> gdg_request_info:
    info = gdg_request_info()
    _scheck(load().gdg_server_poll(srv, ticket, C.byref(info)), srv)
    return info


def gdg_server_result(srv, ticket: int, out: np.ndarray) -> np.ndarray:
    assert out.dtype == np.float64 and out.flags.c_contiguous
    _scheck(load().gdg_server_result(srv, ticket, out.ctypes.data_as(_DP)), srv)
    return out


def gdg_server_destroy(srv):
    load().gdg_server_destroy(srv)


def gdg_server_last_error(srv) -> str:
    return load().gdg_server_last_error(srv).decode()


class Server:
    """A request server whose memory pool (the HBM budget) is a torch uint8
    tensor on ``device`` and whose stream is torch's current stream there."""

    def __init__(self, dim, degree, precision=GDG_FP64, budget_bytes=4 << 30, max_slots=64,
                 steps_per_graph=8, device="cuda:0", stream=None, solo_dofs=0):
        import torch
        self.desc = server_desc(dim, degree, precision, max_slots, steps_per_graph, solo_dofs)
        self.device = torch.device(device)
        self.pool = torch.empty(budget_bytes + 256, dtype=torch.uint8, device=self.device)
        self.pool_ptr = (self.pool.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.srv = gdg_server_create(self.desc, self.pool_ptr, budget_bytes, self.stream.cuda_stream)
        self.m = dim + 2

    def submit(self, ms, U0, t_final, params=None) -> int:
        prm = params if params is not None else gdg_default_params(ms.degree)
        if params is None:
            prm.precision = self.desc.precision
        mesh = mesh_desc(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc, getattr(ms, "bstate", None),
                         getattr(ms, "vortex", None), getattr(ms, "vertices", None),
                         getattr(ms, "bc_cells", None), getattr(ms, "map_degree", 1))
        return gdg_server_submit(self.srv, mesh, prm, U0, t_final)

    def pump(self):
        return gdg_server_pump(self.srv)

    def sync(self):
        gdg_server_sync(self.srv)

    def poll(self, ticket) -> gdg_request_info:
        return gdg_server_poll(self.srv, ticket)

    def result(self, ticket) -> np.ndarray:
        info = self.poll(ticket)
        out = np.zeros((self.m, info.ndofs))
        return gdg_server_result(self.srv, ticket, out)

    def close(self):
        if getattr(self, "srv", None):
            gdg_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        self.close()
