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

GDG_OK, GDG_E_INVALID, GDG_E_INADMISSIBLE, GDG_E_CFL, GDG_E_NOMEM, GDG_E_DEVICE = 0, -1, -2, -3, -4, -5
GDG_BC_PERIODIC, GDG_BC_OUTFLOW, GDG_BC_SLIP = 0, 1, 2
GDG_LOW_ORDER, GDG_HIGH_ORDER, GDG_LIMITED = 0, 1, 2
GDG_FP64, GDG_MIXED = 0, 1
(GDG_FIELD_STATE, GDG_FIELD_EV_N, GDG_FIELD_BOUNDS, GDG_FIELD_UL, GDG_FIELD_DUH,
 GDG_FIELD_U1) = range(6)
_FIELD_PLANES = {GDG_FIELD_EV_N: 1, GDG_FIELD_BOUNDS: 3}

_NAMES = {0: "GDG_OK", -1: "GDG_E_INVALID", -2: "GDG_E_INADMISSIBLE", -3: "GDG_E_CFL",
          -4: "GDG_E_NOMEM", -5: "GDG_E_DEVICE"}


class GdgError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__("%s%s" % (_NAMES.get(status, str(status)), (": " + msg) if msg else ""))


class gdg_mesh_desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("degree", C.c_int32), ("cells", C.c_int64 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("bc", C.c_int32 * 6)]


class gdg_params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("cfl", C.c_double), ("c_ev", C.c_double),
                ("c_k", C.c_double), ("c_r", C.c_double), ("p_r", C.c_double),
                ("limiter_passes", C.c_int32), ("scheme", C.c_int32), ("precision", C.c_int32),
                ("reserved", C.c_int32)]


class gdg_stats(C.Structure):
    _fields_ = [("t", C.c_double), ("steps", C.c_int64), ("restarts", C.c_int64),
                ("last_dt", C.c_double)]


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
    for fn in ("gdg_default_params", "gdg_workspace_bytes", "gdg_create", "gdg_node_coords",
               "gdg_upload_state", "gdg_download_state", "gdg_step", "gdg_run_to", "gdg_stage",
               "gdg_read_field", "gdg_get_stats", "gdg_profile", "gdg_profile_read"):
        getattr(L, fn).restype = C.c_int
    _lib = L
    return L


def _check(st, ctx=None):
    if st != GDG_OK:
        msg = load().gdg_last_error(ctx).decode()
        raise GdgError(st, msg)


def mesh_desc(dim, degree, cells, lo, hi, bc) -> gdg_mesh_desc:
    m = gdg_mesh_desc()
    m.dim, m.degree = dim, degree
    for e in range(3):
        m.cells[e] = int(cells[e]) if e < dim else 1
        m.lo[e] = float(lo[e]) if e < dim else 0.0
        m.hi[e] = float(hi[e]) if e < dim else 1.0
    for f in range(6):
        m.bc[f] = int(bc[f]) if f < 2 * dim else GDG_BC_OUTFLOW
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


# -- convenience owner of workspace + context ----------------------------------
class Solver:
    """A context whose device workspace is a torch uint8 tensor on ``device``
    and whose stream is torch's current stream there (or ``stream``)."""

    def __init__(self, dim, degree, cells, lo, hi, bc, params: gdg_params | None = None,
                 device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.dim, self.m = dim, dim + 2
        self.mesh = mesh_desc(dim, degree, cells, lo, hi, bc)
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
        return cls(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc, params, **kw)

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
