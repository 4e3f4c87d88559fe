"""Python face of the CPU FP64 oracle (``gdg_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow, literal CPU
implementation of the graph-based DG scheme of arXiv 2402.04514 that the GPU
library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import it.  It shares no code with
the GPU library.

Conventions (the same interface conventions as the library, written
independently): dofs are numbered cell-major, cells lexicographic with x
fastest, local nodes lexicographic with x fastest; states are SoA arrays of
shape ``(dim + 2, ndofs)`` holding ``rho, m_1..m_d, E``; box face ``f = 2*axis
+ side`` (side 0 = low); boundary kinds 0 periodic, 1 outflow, 2 slip,
3 Dirichlet, 4 supersonic in/outflow (the last two with per-face data).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gdg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_PERIODIC, BC_OUTFLOW, BC_SLIP, BC_DIRICHLET, BC_SUPERSONIC, BC_INOUTFLOW = 0, 1, 2, 3, 4, 5
LOW_ORDER, HIGH_ORDER, LIMITED = 0, 1, 2
SSPRK3, SSPRK54 = 0, 1
KIND_CELL, KIND_FACE_COLLOC, KIND_FACE = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc at -O2, no fast-math (OpenMP over rows)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("cfl", C.c_double), ("c_ev", C.c_double),
                ("c_k", C.c_double), ("c_r", C.c_double), ("p_r", C.c_double),
                ("passes", C.c_int), ("scheme", C.c_int), ("integrator", C.c_int)]


_DP = C.POINTER(C.c_double)


class _Diag(C.Structure):
    _fields_ = [("tau_max", C.c_double), ("N", _DP), ("rho_min", _DP), ("rho_max", _DP),
                ("s_min", _DP), ("UL", _DP), ("dUH", _DP), ("U1", _DP), ("dij", _DP),
                ("lij", _DP), ("lbd", _DP), ("Aij", _DP), ("Abd", _DP), ("Ncond", _DP)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        # GDG_ORACLE_LIB points the pins at another build of this same source
        # (used to check that planted mistakes make the pins fail)
        _lib = C.CDLL(os.environ.get("GDG_ORACLE_LIB") or build())
        L = _lib
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_long), _DP, _DP, C.POINTER(C.c_int)]
        L.or_create_mapped.restype = C.c_void_p
        L.or_create_mapped.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_long), _DP, C.POINTER(C.c_int)]
        L.or_create_curved.restype = C.c_void_p
        L.or_create_curved.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_long), _DP, C.POINTER(C.c_int), C.c_int]
        L.or_create_cg_curved.restype = C.c_void_p
        L.or_create_cg_curved.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_long), _DP, C.POINTER(C.c_int), C.c_int]
        L.or_create_cg.restype = C.c_void_p
        L.or_create_cg.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_long), _DP, _DP, C.POINTER(C.c_int)]
        L.or_create_unstructured.restype = C.c_void_p
        L.or_create_unstructured.argtypes = [C.c_int, C.c_int, C.c_long, C.POINTER(C.c_long), C.c_long, _DP, C.c_int,
                                             C.POINTER(C.c_byte)]
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_num_threads.restype = C.c_int
        L.or_num_threads.argtypes = []
        L.or_default_cev.restype = C.c_double
        L.or_default_cev.argtypes = [C.c_int]
        L.or_set_num_threads.restype = None
        L.or_set_num_threads.argtypes = [C.c_int]
        for fn in ("or_num_dofs", "or_nnz", "or_nbnd"):
            getattr(L, fn).restype = C.c_long
            getattr(L, fn).argtypes = [C.c_void_p]
        L.or_volume.restype = C.c_double
        L.or_volume.argtypes = [C.c_void_p]
        L.or_set_reference_volume.restype = None
        L.or_set_reference_volume.argtypes = [C.c_void_p, C.c_double]
        L.or_set_boundary_kinds.restype = C.c_int
        L.or_set_boundary_kinds.argtypes = [C.c_void_p, C.POINTER(C.c_byte)]
        L.or_set_boundary_state.restype = None
        L.or_set_boundary_state.argtypes = [C.c_void_p, C.c_int, _DP]
        L.or_inoutflow_state.restype = C.c_int
        L.or_inoutflow_state.argtypes = [C.c_int, C.c_double, _DP, _DP, _DP, _DP]
        L.or_set_time.restype = None
        L.or_set_time.argtypes = [C.c_void_p, C.c_double]
        L.or_set_vortex_data.restype = C.c_int
        L.or_set_vortex_data.argtypes = [C.c_void_p, _DP]
        L.or_csr.argtypes = [C.c_void_p, C.POINTER(C.c_long), C.POINTER(C.c_long), _DP, _DP,
                             C.POINTER(C.c_int)]
        L.or_lumped.argtypes = [C.c_void_p, _DP]
        L.or_boundary.argtypes = [C.c_void_p, C.POINTER(C.c_long), C.POINTER(C.c_int), _DP]
        L.or_node_coords.argtypes = [C.c_void_p, _DP]
        L.or_literal_cij.argtypes = [C.c_void_p, C.c_long, C.c_long, _DP]
        L.or_lambda_max.restype = C.c_double
        L.or_lambda_max.argtypes = [C.c_double, C.c_int, _DP, _DP, _DP]
        L.or_exact_riemann.restype = C.c_int
        L.or_exact_riemann.argtypes = [C.c_double] * 7 + [_DP, _DP]
        L.or_exact_lambda.restype = C.c_double
        L.or_exact_lambda.argtypes = [C.c_double] * 7
        L.or_riemann_sample.argtypes = [C.c_double] * 8 + [_DP]
        L.or_stage.restype = C.c_int
        L.or_stage.argtypes = [C.c_void_p, C.POINTER(_Params), _DP, C.c_double, _DP,
                               C.POINTER(_Diag)]
        L.or_tau_rows.argtypes = [C.c_void_p, C.POINTER(_Params), _DP, _DP]
        L.or_set_step_start_data.restype = None
        L.or_set_step_start_data.argtypes = [C.c_void_p]
        L.or_ssprk54_table.restype = None
        L.or_ssprk54_table.argtypes = [_DP, _DP]
        L.or_step.restype = C.c_int
        L.or_step.argtypes = [C.c_void_p, C.POINTER(_Params), _DP, C.c_double, C.c_double, _DP,
                              C.POINTER(C.c_int)]
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


def params(gamma=1.4, cfl=0.5, degree=1, c_ev=None, c_k=1.0, c_r=4.0, p_r=1.5, passes=2,
           scheme=LIMITED, integrator=SSPRK3) -> _Params:
    """Scheme constants of Sec. 5 (c_ev = 1, 0.5, 0.25 for k = 1, 2, 3);
    integrator SSPRK3 or SSPRK54 (the fourth-order SSP method of Sec. 6.2)."""
    if c_ev is None:
        c_ev = lib().or_default_cev(degree)
    return _Params(gamma, cfl, c_ev, c_k, c_r, p_r, passes, scheme, integrator)


def ssprk54_table():
    """(alpha, beta): the Shu-Osher coefficients of the oracle's SSPRK(5,4),
    rows i = 0..5 (stage u(i)), columns k = 0..4."""
    a = np.zeros(30)
    b = np.zeros(30)
    lib().or_ssprk54_table(_dp(a), _dp(b))
    return a.reshape(6, 5), b.reshape(6, 5)


class Mesh:
    """Uniform Cartesian DG Q_k mesh with the stencil of Sec. 2.3."""

    def __init__(self, dim, degree, cells, lo, hi, bc, bstate=None, vortex=None, vertices=None, bc_cells=None,
                 map_degree=1, continuous=False, step_start_data=False):
        """bc: kinds per box face 2*axis+side (0 periodic, 1 outflow, 2 slip,
        3 Dirichlet, 4 supersonic in/outflow, 5 sub- and supersonic
        in/outflow).  bstate: per face the conserved Dirichlet data U^d of
        kinds 3-5 (None elsewhere).  vortex: (beta, x0_1, x0_2, u_1, u_2,
        gamma) to take the data of kinds 3-5 from the isentropic vortex at the
        node and the stage time instead (2D).  vertices: the cell lattice's
        vertices, shape ((n_0+1)(n_1+1)..., dim), x fastest, for general
        (multilinearly mapped) cells; lo and hi are then ignored.
        map_degree 2: curved cells, vertices then holds the lattice of
        2 n_e + 1 points per axis (corners, edge and face midpoints, centres)
        of quadratic cell maps.  continuous: continuous Q_k elements on the
        box (App. B): one dof per lattice node, c_ij and c_i^d of
        eq. cijcidefCg; the low-order scheme only.  bc_cells:
        a kind per boundary cell face (kinds 1-5): for each non-periodic box
        face in order, its cells lexicographically over the other axes, the
        lowest axis fastest; data kinds take that box face's data.
        step_start_data: the data of kinds 3-5 are the node's own state at
        the start of the step (strategy (d) of Sec. 6.3)."""
        self.dim, self.degree = dim, degree
        self.cells = tuple(int(c) for c in cells)
        self.lo = tuple(float(x) for x in lo)
        self.hi = tuple(float(x) for x in hi)
        self.bc = tuple(int(b) for b in bc)
        L = lib()
        c = (C.c_long * 3)(*(list(self.cells) + [1] * (3 - dim)))
        lo_ = (C.c_double * 3)(*(list(self.lo) + [0.0] * (3 - dim)))
        hi_ = (C.c_double * 3)(*(list(self.hi) + [1.0] * (3 - dim)))
        b = (C.c_int * 6)(*(list(self.bc) + [1] * (6 - len(self.bc))))
        if vertices is not None:
            vx = np.ascontiguousarray(vertices, dtype=np.float64)
            nv = int(np.prod([map_degree * n + 1 for n in self.cells]))
            assert vx.shape == (nv, dim), (vx.shape, nv, dim)
            self._vx = vx
            if continuous:
                self._h = L.or_create_cg_curved(dim, degree, c, _dp(vx), b, int(map_degree))
            else:
                self._h = L.or_create_curved(dim, degree, c, _dp(vx), b, int(map_degree))
        elif continuous:
            self._h = L.or_create_cg(dim, degree, c, lo_, hi_, b)
        else:
            self._h = L.or_create(dim, degree, c, lo_, hi_, b)
        if not self._h:
            raise ValueError("invalid mesh description")
        self.ndofs = L.or_num_dofs(self._h)
        self.m = dim + 2
        if vortex is not None:
            v = np.ascontiguousarray(vortex, dtype=np.float64)
            assert v.shape == (6,)
            if L.or_set_vortex_data(self._h, _dp(v)) != 0:
                raise ValueError("vortex boundary data needs a 2D mesh")
        if step_start_data:
            L.or_set_step_start_data(self._h)
        kinds = [{self.bc[f]} for f in range(2 * dim)]
        if bc_cells is not None:
            k = np.ascontiguousarray(bc_cells, dtype=np.int8).ravel()
            pos = 0
            for f in range(2 * dim):
                if self.bc[f] == 0:
                    continue
                cnt = int(np.prod([self.cells[g] for g in range(dim) if g != f // 2]))
                kinds[f] = set(int(x) for x in k[pos:pos + cnt])
                pos += cnt
            if pos != k.size:
                raise ValueError("bc_cells needs %d entries, not %d" % (pos, k.size))
            self._bcc = k
            if L.or_set_boundary_kinds(self._h, k.ctypes.data_as(C.POINTER(C.c_byte))) != 0:
                raise ValueError("bc_cells holds a periodic or unknown kind")
        for f in range(2 * dim):
            if kinds[f] & {3, 4, 5} and vortex is None and not step_start_data:
                if bstate is None or bstate[f] is None:
                    raise ValueError("face %d needs Dirichlet data" % f)
                v = np.ascontiguousarray(bstate[f], dtype=np.float64)
                assert v.shape == (self.m,)
                L.or_set_boundary_state(self._h, f, _dp(v))

    @classmethod
    def unstructured(cls, dim, degree, cell_points, points, face_bc, bstate=None, map_degree=1,
                     step_start_data=False):
        """Unstructured mesh: cell K is the image of the reference cell under
        the map of degree map_degree through points[cell_points[K, v]] (v the
        digits q_e in base map_degree + 1, first axis lowest); cells sharing a
        face's corner points are neighbours.  face_bc[K, f]: for a face on no
        other cell, its kind (1-5) + 8 * the box-face slot of its data in
        bstate.  step_start_data: the data are the node's own state at the
        start of the step instead (strategy (d) of Sec. 6.3)."""
        self = cls.__new__(cls)
        L = lib()
        cp = np.ascontiguousarray(cell_points, dtype=np.int64)
        pts = np.ascontiguousarray(points, dtype=np.float64)
        fb = np.ascontiguousarray(face_bc, dtype=np.int8)
        ncells = cp.shape[0]
        assert cp.shape == (ncells, (map_degree + 1) ** dim) and pts.shape[1] == dim
        assert fb.shape == (ncells, 2 * dim)
        self._keep = (cp, pts, fb)
        self._h = L.or_create_unstructured(dim, degree, ncells, cp.ctypes.data_as(C.POINTER(C.c_long)),
                                           pts.shape[0], _dp(pts), int(map_degree),
                                           fb.ctypes.data_as(C.POINTER(C.c_byte)))
        if not self._h:
            raise ValueError("invalid unstructured mesh")
        self.dim, self.degree = dim, degree
        self.cells = (ncells,)
        self.bc = (1,) * (2 * dim)
        self.ndofs = L.or_num_dofs(self._h)
        self.m = dim + 2
        for f in range(6):
            if bstate is not None and f < len(bstate) and bstate[f] is not None:
                v = np.ascontiguousarray(bstate[f], dtype=np.float64)
                L.or_set_boundary_state(self._h, f, _dp(v))
        if step_start_data:
            L.or_set_step_start_data(self._h)
        return self

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_destroy(h)
            self._h = None

    @property
    def volume(self) -> float:
        return lib().or_volume(self._h)

    def set_reference_volume(self, vol: float):
        """|Omega| in hhat_i = (m_i/|Omega|)^(1/d) (eq. ViscMin, ViscMinConst2):
        a sub-box of a larger domain passes that domain's volume."""
        lib().or_set_reference_volume(self._h, float(vol))

    def coords(self) -> np.ndarray:
        x = np.zeros((self.ndofs, self.dim))
        lib().or_node_coords(self._h, _dp(x))
        return x

    def csr(self):
        L = lib()
        nnz = L.or_nnz(self._h)
        rowptr = np.zeros(self.ndofs + 1, dtype=np.int64)
        col = np.zeros(nnz, dtype=np.int64)
        c = np.zeros((nnz, self.dim))
        mij = np.zeros(nnz)
        kind = np.zeros(nnz, dtype=np.int32)
        L.or_csr(self._h, rowptr.ctypes.data_as(C.POINTER(C.c_long)),
                 col.ctypes.data_as(C.POINTER(C.c_long)), _dp(c), _dp(mij),
                 kind.ctypes.data_as(C.POINTER(C.c_int)))
        return rowptr, col, c, mij, kind

    def lumped(self) -> np.ndarray:
        mi = np.zeros(self.ndofs)
        lib().or_lumped(self._h, _dp(mi))
        return mi

    def boundary(self):
        L = lib()
        nb = L.or_nbnd(self._h)
        bptr = np.zeros(self.ndofs + 1, dtype=np.int64)
        bface = np.zeros(max(nb, 1), dtype=np.int32)
        bc_c = np.zeros((max(nb, 1), self.dim))
        L.or_boundary(self._h, bptr.ctypes.data_as(C.POINTER(C.c_long)),
                      bface.ctypes.data_as(C.POINTER(C.c_int)), _dp(bc_c))
        return bptr, bface[:nb], bc_c[:nb]

    def literal_cij(self, i, j) -> np.ndarray:
        out = np.zeros(self.dim)
        lib().or_literal_cij(self._h, i, j, _dp(out))
        return out

    # -- scheme ------------------------------------------------------------
    def stage(self, prm: _Params, U: np.ndarray, tau: float = 0.0, diag: bool = False):
        """One forward-Euler stage Phi(U; tau); tau <= 0 picks Cr * tau_max."""
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(self.m, self.ndofs)
        out = np.zeros_like(U)
        d = _Diag()
        arrs = {}
        if diag:
            N, nnz, m = self.ndofs, lib().or_nnz(self._h), self.m
            shapes = {"N": (N,), "rho_min": (N,), "rho_max": (N,), "s_min": (N,),
                      "UL": (m, N), "dUH": (m, N), "U1": (m, N), "dij": (nnz,),
                      "lij": (nnz,), "lbd": (N,), "Aij": (nnz, m), "Abd": (N, m), "Ncond": (N,)}
            for k, shp in shapes.items():
                arrs[k] = np.zeros(shp)
                setattr(d, k, _dp(arrs[k]))
        st = lib().or_stage(self._h, C.byref(prm), _dp(U), float(tau), _dp(out), C.byref(d))
        arrs["tau_max"] = d.tau_max
        arrs["status"] = st
        return (out, arrs) if diag else out

    def tau_rows(self, prm: _Params, U: np.ndarray) -> np.ndarray:
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(self.m, self.ndofs)
        out = np.zeros(self.ndofs)
        lib().or_tau_rows(self._h, C.byref(prm), _dp(U), _dp(out))
        return out

    def set_time(self, t: float):
        """Time of the step's start, for time-dependent boundary data."""
        lib().or_set_time(self._h, float(t))

    def step(self, prm: _Params, U: np.ndarray, dt_cap: float = 0.0, dt_fixed: float = 0.0):
        """One step of the integrator prm names.  Returns (U_new, dt_taken,
        restarts, status)."""
        U = np.array(U, dtype=np.float64).reshape(self.m, self.ndofs)
        dt = C.c_double(0.0)
        nres = C.c_int(0)
        st = lib().or_step(self._h, C.byref(prm), _dp(U), float(dt_cap), float(dt_fixed),
                           C.byref(dt), C.byref(nres))
        return U, dt.value, nres.value, st

    def run_to(self, prm: _Params, U: np.ndarray, t_final: float, max_steps: int = 10**9):
        U = np.array(U, dtype=np.float64).reshape(self.m, self.ndofs)
        t, n = 0.0, 0
        while t < t_final and n < max_steps:
            cap = t_final - t
            self.set_time(t)
            U, dt, _, st = self.step(prm, U, dt_cap=cap)
            if st:
                raise RuntimeError("oracle step failed with status %d" % st)
            t = t_final if dt == cap else t + dt
            n += 1
        return U, t, n


_THREADS0 = None


def num_threads() -> int:
    """Threads the oracle's row loops run on."""
    return lib().or_num_threads()


def num_threads_available() -> int:
    """Threads the row loops ran on before any set_num_threads() call (the
    OpenMP default of this process: OMP_NUM_THREADS, else the cores)."""
    global _THREADS0
    if _THREADS0 is None:
        _THREADS0 = lib().or_num_threads()
    return _THREADS0


def set_num_threads(n: int):
    """Threads of the row loops (results do not depend on it)."""
    num_threads_available()
    lib().or_set_num_threads(int(n))


# -- physics helpers -------------------------------------------------------
def lambda_max(gamma, UL, UR, n) -> float:
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UR = np.ascontiguousarray(UR, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    return lib().or_lambda_max(gamma, len(n), _dp(UL), _dp(UR), _dp(n))


def exact_riemann(gamma, rl, ul, pl, rr, ur, pr):
    ps, us = C.c_double(), C.c_double()
    vac = lib().or_exact_riemann(gamma, rl, ul, pl, rr, ur, pr, C.byref(ps), C.byref(us))
    return ps.value, us.value, vac


def exact_lambda(gamma, rl, ul, pl, rr, ur, pr) -> float:
    return lib().or_exact_lambda(gamma, rl, ul, pl, rr, ur, pr)


def inoutflow_state(gamma, Ui, Ud, n):
    """Boundary state of the sub- and supersonic in/outflow kind for node
    state Ui, data Ud and outward unit normal n: (state, status)."""
    Ui = np.ascontiguousarray(Ui, dtype=np.float64)
    Ud = np.ascontiguousarray(Ud, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    out = np.zeros_like(Ui)
    st = lib().or_inoutflow_state(len(n), gamma, _dp(Ui), _dp(Ud), _dp(n), _dp(out))
    return out, st


def riemann_sample(gamma, left, right, xi):
    out = np.zeros(3)
    lib().or_riemann_sample(gamma, *left, *right, float(xi), _dp(out))
    return out
