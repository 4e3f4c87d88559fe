"""Seeded synthetic inputs shaped like the paper's test problems.

This module holds no arithmetic of the scheme: it only lays out initial
states (primitive data converted to conserved variables) on the dof numbering
that the library documents, so that the GPU path and the CPU oracle can be
fed bit-identical inputs.  The problems:

* ``sod``      1D shock tube on [0, 1], 200 Q1 cells, outflow (the role of the
               paper's LeBlanc tube, Sec. 6.2 (iii), with textbook Sod data).
* ``vortex``   2D isentropic vortex on [-5, 5]^2, periodic (Sec. 6.2 (i)),
               gamma = 1.4; velocity factor exp((1 - r^2)/2), the steady form.
* ``quadrant`` 2D four-quadrant Riemann data on [0, 1]^2, states drawn per
               quadrant from SplitMix64 (seed 240204514 + q).
* ``blast``    3D blast on [0, 1]^3 with slip walls: p = 100 in the cells whose
               centre lies within 0.1 of the box centre, p = 0.1 elsewhere.

Numbering: dof = cell * (k+1)^d + local; cells lexicographic with x fastest,
local Gauss-Lobatto nodes lexicographic with x fastest.  Piecewise data are
assigned per cell from the cell centre, so duplicated face nodes of
neighbouring cells keep their own cell's value.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BC_PERIODIC, BC_OUTFLOW, BC_SLIP, BC_DIRICHLET, BC_SUPERSONIC, BC_INOUTFLOW = 0, 1, 2, 3, 4, 5
GAMMA = 1.4


@dataclass
class MeshSpec:
    dim: int
    degree: int
    cells: tuple
    lo: tuple
    hi: tuple
    bc: tuple  # per box face 2*axis+side
    # per box face: the conserved Dirichlet data U^d of the Dirichlet and
    # supersonic kinds (None elsewhere, or None for no such face)
    bstate: tuple | None = None
    # (beta, x0_1, x0_2, u_1, u_2, gamma): the data of those faces from the
    # isentropic vortex at the node and the time instead
    vortex: tuple | None = None
    # general cells: the lattice's points, shape (prod(cells + 1), dim), x
    # fastest (lo and hi then only name the box the points were drawn in)
    vertices: np.ndarray | None = field(default=None, repr=False, compare=False)
    # boundary parts: a kind per boundary cell face (each non-periodic box face
    # in order, its cells over the other axes, the lowest axis fastest)
    bc_cells: np.ndarray | None = field(default=None, repr=False, compare=False)
    # degree of the cell maps of general cells: 1 multilinear, 2 quadratic
    # (vertices then holds 2 cells + 1 points per axis)
    map_degree: int = 1

    @property
    def nloc(self) -> int:
        return (self.degree + 1) ** self.dim

    @property
    def ncells(self) -> int:
        return int(np.prod(self.cells))

    @property
    def ndofs(self) -> int:
        return self.ncells * self.nloc


@dataclass
class Workload:
    name: str
    mesh: MeshSpec
    U0: np.ndarray = field(repr=False)  # (dim+2, ndofs) conserved SoA
    t_final: float | None = None
    steps: int | None = None


def gl_nodes(degree: int) -> np.ndarray:
    r = 0.5 / math.sqrt(5.0)
    return np.array({1: [0.0, 1.0], 2: [0.0, 0.5, 1.0], 3: [0.0, 0.5 - r, 0.5 + r, 1.0]}[degree])


def node_coords(ms: MeshSpec):
    """Node coordinates (ndofs, dim) and owning cell centres (ndofs, dim)."""
    d, k = ms.dim, ms.degree
    nb = k + 1
    h = [(ms.hi[e] - ms.lo[e]) / ms.cells[e] for e in range(d)]
    cell = np.arange(ms.ncells)
    loc = np.arange(ms.nloc)
    ci, li = [], []
    r = cell.copy()
    for e in range(d):
        ci.append(r % ms.cells[e])
        r //= ms.cells[e]
    r = loc.copy()
    for e in range(d):
        li.append(r % nb)
        r //= nb
    xg = gl_nodes(k)
    x = np.zeros((ms.ndofs, d))
    xc = np.zeros((ms.ndofs, d))
    for e in range(d):
        xs = ms.lo[e] + (ci[e][:, None] + xg[li[e]][None, :]) * h[e]
        cs = ms.lo[e] + (ci[e][:, None] + 0.5 + 0.0 * li[e][None, :]) * h[e]
        x[:, e] = xs.reshape(-1)
        xc[:, e] = cs.reshape(-1)
    return x, xc


def lattice(cells, lo, hi) -> np.ndarray:
    """The points of a uniform cell lattice, (prod(cells + 1), dim), x fastest."""
    axes = [np.linspace(lo[e], hi[e], cells[e] + 1) for e in range(len(cells))]
    grids = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.transpose(*reversed(range(len(cells)))).ravel() for g in grids], axis=1)


def refine_points(V, cells) -> np.ndarray:
    """The quadratic point lattice (2 n_e + 1 per axis, x fastest) of the
    multilinear cells of the lattice V: each new point is the multilinear
    interpolation of its cell's corners at the edge, face or cell midpoint, so
    the quadratic cell maps through these points equal the multilinear ones."""
    d = len(cells)
    n1 = [c + 1 for c in cells]
    n2 = [2 * c + 1 for c in cells]
    P = np.asarray(V, dtype=np.float64).reshape(tuple(reversed(n1)) + (d,))
    out = np.zeros(tuple(reversed(n2)) + (d,))
    # axis order of P and out: (z, y, x) reversed; interpolate axis by axis
    cur = P
    for ax in range(d):
        a = d - 1 - ax  # array axis of lattice axis ax
        shape = list(cur.shape)
        shape[a] = 2 * (shape[a] - 1) + 1
        nxt = np.zeros(shape)
        sl_even = [slice(None)] * len(shape)
        sl_even[a] = slice(0, None, 2)
        nxt[tuple(sl_even)] = cur
        sl_odd = [slice(None)] * len(shape)
        sl_odd[a] = slice(1, None, 2)
        lo_ = [slice(None)] * len(shape)
        hi_ = [slice(None)] * len(shape)
        lo_[a] = slice(0, -1)
        hi_[a] = slice(1, None)
        nxt[tuple(sl_odd)] = 0.5 * (cur[tuple(lo_)] + cur[tuple(hi_)])
        cur = nxt
    out[...] = cur
    return out.reshape(-1, d)


def perturbed_lattice(cells, lo, hi, amp=0.25, seed=3, periodic=False) -> np.ndarray:
    """General cells: the lattice with its interior points moved by up to amp
    cell widths per axis (uniform random, seeded), or (periodic) by the smooth
    field amp h_e sin(2 pi xi_1) .. sin(2 pi xi_d) (+ on even axes, - on odd),
    which vanishes on the box's faces, so opposite boundary layers stay
    congruent."""
    V = lattice(cells, lo, hi)
    d = len(cells)
    h = np.array([(hi[e] - lo[e]) / cells[e] for e in range(d)])
    idx = np.stack(np.unravel_index(np.arange(V.shape[0]), tuple(c + 1 for c in reversed(cells))), axis=1)[:, ::-1]
    interior = np.all((idx > 0) & (idx < np.array(cells)), axis=1)
    if periodic:
        xi = (V - np.array(lo)) / (np.array(hi) - np.array(lo))
        s = np.prod(np.sin(2 * np.pi * xi), axis=1)
        for e in range(d):
            V[:, e] += amp * h[e] * s * (1 if e % 2 == 0 else -1)
        return V
    rng = np.random.default_rng(seed)
    V[interior] += amp * h * rng.uniform(-1, 1, size=(int(interior.sum()), d))
    return V


def to_conserved(rho, vel, p, gamma=GAMMA) -> np.ndarray:
    """[rho, rho u, p/(gamma-1) + rho |u|^2 / 2] as a (d+2, n) array."""
    rho = np.asarray(rho, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64)
    d = vel.shape[0]
    U = np.empty((d + 2, rho.shape[0]))
    U[0] = rho
    for e in range(d):
        U[1 + e] = rho * vel[e]
    U[d + 1] = p / (gamma - 1.0) + 0.5 * rho * np.sum(vel * vel, axis=0)
    return U


# -- SplitMix64 (Steele, Lea & Flood 2014) -----------------------------------
_M64 = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed: int):
        self.s = seed & _M64

    def next_u64(self) -> int:
        self.s = (self.s + 0x9E3779B97F4A7C15) & _M64
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))


def quadrant_states(seed_base: int = 240204514):
    """rho in [0.1, 2], p in [0.1, 10], u uniform in the unit disk, per quadrant."""
    out = []
    for q in range(4):
        g = SplitMix64(seed_base + q)
        rho = 0.1 + 1.9 * g.uniform()
        p = 0.1 + 9.9 * g.uniform()
        rad = math.sqrt(g.uniform())
        ang = 2.0 * math.pi * g.uniform()
        out.append((rho, rad * math.cos(ang), rad * math.sin(ang), p))
    return out


# -- problems ----------------------------------------------------------------
def sod(cells: int = 200, gamma: float = GAMMA) -> Workload:
    ms = MeshSpec(1, 1, (cells,), (0.0,), (1.0,), (BC_OUTFLOW, BC_OUTFLOW))
    _, xc = node_coords(ms)
    left = xc[:, 0] < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    U = to_conserved(rho, np.zeros((1, ms.ndofs)), p, gamma)
    return Workload("sod_q1_%d" % cells, ms, U, t_final=0.2)


def vortex_exact(x: np.ndarray, t: float, beta=5.0, x0=(-1.0, -1.0), uinf=(1.0, 1.0),
                 gamma=GAMMA, lo=-5.0, hi=5.0, periodic=True) -> np.ndarray:
    """Isentropic vortex at time t, periodically wrapped on [lo, hi)^2 (or in
    free space with periodic=False)."""
    L = hi - lo
    xb = np.empty_like(x)
    for e in range(2):
        xb[:, e] = x[:, e] - x0[e] - t * uinf[e]
        if periodic:
            xb[:, e] = (xb[:, e] - lo) % L + lo
    r2 = xb[:, 0] ** 2 + xb[:, 1] ** 2
    T = 1.0 - (gamma - 1.0) * beta ** 2 / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    fac = beta / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
    vel = np.stack([uinf[0] - fac * xb[:, 1], uinf[1] + fac * xb[:, 0]])
    return to_conserved(rho, vel, p, gamma)


def vortex(cells: int = 256, gamma: float = GAMMA) -> Workload:
    ms = MeshSpec(2, 1, (cells, cells), (-5.0, -5.0), (5.0, 5.0), (BC_PERIODIC,) * 4)
    x, _ = node_coords(ms)
    return Workload("vortex_q1_%d" % cells, ms, vortex_exact(x, 0.0, gamma=gamma), t_final=2.0)


def quadrant(cells: int = 1024, degree: int = 2, seed_base: int = 240204514,
             gamma: float = GAMMA, bc: int = BC_OUTFLOW) -> Workload:
    ms = MeshSpec(2, degree, (cells, cells), (0.0, 0.0), (1.0, 1.0), (bc,) * 4)
    _, xc = node_coords(ms)
    q = (xc[:, 0] >= 0.5).astype(int) + 2 * (xc[:, 1] >= 0.5).astype(int)
    st = np.array(quadrant_states(seed_base))
    rho, ux, uy, p = (st[q, c] for c in range(4))
    U = to_conserved(rho, np.stack([ux, uy]), p, gamma)
    return Workload("quadrant_q%d_%d" % (degree, cells), ms, U, steps=500)


def blast(cells: int = 128, gamma: float = GAMMA) -> Workload:
    ms = MeshSpec(3, 1, (cells,) * 3, (0.0,) * 3, (1.0,) * 3, (BC_SLIP,) * 6)
    _, xc = node_coords(ms)
    r2 = np.sum((xc - 0.5) ** 2, axis=1)
    p = np.where(r2 <= 0.1 ** 2, 100.0, 0.1)
    U = to_conserved(np.ones(ms.ndofs), np.zeros((3, ms.ndofs)), p, gamma)
    return Workload("blast_q1_%d" % cells, ms, U, steps=200)


# Supersonic inflow problem: a uniform supersonic stream (DOWNSTREAM) fills
# the box; from t = 0 the inflow face feeds a different supersonic state
# (INFLOW).  Every wave of the Riemann problem INFLOW | DOWNSTREAM moves into
# the box (slowest: the rarefaction head at u - a = 1.32), so the exact
# solution is that Riemann fan centred on the inflow face.  (rho, u_n, p).
INFLOW = (1.0, 2.5, 1.0)
DOWNSTREAM = (0.5, 2.5, 0.6)


def inflow(cells: int = 200, dim: int = 1, axis: int = 0, degree: int = 1, cross: int = 4,
           kind: int = BC_SUPERSONIC) -> Workload:
    """Unit box, `cells` cells along the flow axis and `cross` across it
    (periodic), flow along +axis; both faces of the flow axis of boundary kind
    `kind` with the INFLOW state as data on the inflow face and DOWNSTREAM on
    the outflow face."""
    n = tuple(cells if e == axis else cross for e in range(dim))
    bc = []
    bstate = []
    for e in range(dim):
        for side in range(2):
            bc.append(kind if e == axis else BC_PERIODIC)
            if e != axis:
                bstate.append(None)
                continue
            rho, un, p = INFLOW if side == 0 else DOWNSTREAM
            vel = np.zeros((dim, 1))
            vel[axis] = un
            bstate.append(tuple(to_conserved(np.array([rho]), vel, np.array([p]))[:, 0]))
    ms = MeshSpec(dim, degree, n, (0.0,) * dim, (1.0,) * dim, tuple(bc), tuple(bstate))
    vel = np.zeros((dim, ms.ndofs))
    vel[axis] = DOWNSTREAM[1]
    U = to_conserved(np.full(ms.ndofs, DOWNSTREAM[0]), vel, np.full(ms.ndofs, DOWNSTREAM[2]))
    return Workload("inflow_%dd_q%d_%d" % (dim, degree, cells), ms, U, t_final=0.2)


def serving_trace(count: int = 256, n_min: int = 32, n_max: int = 512, seed0: int = 1000,
                  arrival_seed: int = 7, rate: float = 20.0):
    """Requests of the serving workload: (arrival time, cells per side, state
    seed base).  Arrivals are a Poisson process of the given rate (cumulative
    Exp(1/rate) gaps from SplitMix64(arrival_seed)); request r draws its size
    log-uniformly in [n_min, n_max] from SplitMix64(seed0 + r), and its four
    quadrant states from seed base 4 (seed0 + r), so that no two requests share
    a quadrant's generator.  The requests are run in a closed box (slip walls):
    with do-nothing outflow boundaries, random quadrant velocities that point
    into the box at a corner keep injecting mass there (density grows without
    bound well before t = 0.25), which is a property of that boundary data,
    not of a solver."""
    arr = SplitMix64(arrival_seed)
    t = 0.0
    out = []
    for r in range(count):
        t += -math.log(1.0 - arr.uniform()) / rate
        g = SplitMix64(seed0 + r)
        n = int(round(n_min * (n_max / n_min) ** g.uniform()))
        out.append((t, n, 4 * (seed0 + r)))
    return out


def cylinder_ogrid(ntheta: int = 512, nr: int = 128, degree: int = 1, mach: float = 3.0,
                   center=(0.6, 0.0), radius: float = 0.25, box=((0.0, 4.0), (-1.0, 1.0)),
                   stretch: float = 0.0, map_degree: int = 1):
    """The geometry of the Mach 3 flow past a cylinder (Sec. 6.4): the channel
    box[0] x box[1] minus the disk of the given centre and radius, meshed by
    an O-grid of general cells.  Axis 0 runs around the cylinder (periodic,
    ntheta cells, the first and last layers of points coincide), axis 1 from
    the cylinder (face 2) to the channel's walls (face 3), nr cells.

    The ray from the centre at angle theta_i = pi - 2 pi i / ntheta (i = 0 at
    the upstream stagnation line) meets the circle and the channel's
    boundary; points on it are spaced by (e^(stretch s) - 1)/(e^stretch - 1)
    (uniform for stretch 0).  The outer point nearest each of the channel's
    four corners is moved onto that corner, so the outer face is the
    rectangle itself.  Boundary parts of face 3: Dirichlet on x = box[0][0]
    (the inflow, data: the free stream), outflow on x = box[0][1], slip on the
    top and bottom walls; the cylinder (face 2) is a slip wall.

    map_degree 2 gives curved cells: the lattice of 2 n + 1 points per axis,
    with the cylinder's edge midpoints on the circle, the outer edge
    midpoints halfway along the straight channel walls, and the points
    between on the rays of the half angles at the half radial steps.

    Returns (vertices of shape ((m ntheta+1)(m nr+1), 2) for map degree m, bc,
    bc_cells, the free stream as conserved data): rho = gamma, p = 1 (sound
    speed 1), u = mach."""
    (x0, x1), (y0, y1) = box
    cx, cy = center
    # clockwise, so that (around, outwards) is a positively oriented frame
    th = math.pi - 2.0 * math.pi * np.arange(ntheta + 1) / ntheta
    dx, dy = np.cos(th), np.sin(th)
    # distance along each ray to the rectangle
    with np.errstate(divide="ignore", invalid="ignore"):
        tx = np.where(dx > 0, (x1 - cx) / dx, np.where(dx < 0, (x0 - cx) / dx, np.inf))
        ty = np.where(dy > 0, (y1 - cy) / dy, np.where(dy < 0, (y0 - cy) / dy, np.inf))
    t = np.minimum(tx, ty)
    outer = np.stack([cx + t * dx, cy + t * dy], axis=1)
    for corner in ((x0, y0), (x0, y1), (x1, y0), (x1, y1)):
        ang = math.atan2(corner[1] - cy, corner[0] - cx) % (2 * math.pi)
        rel = (th - ang) % (2 * math.pi)
        i = int(np.argmin(np.minimum(rel, 2 * math.pi - rel)[:ntheta]))
        outer[i] = corner
        if i == 0:
            outer[ntheta] = corner
    m = int(map_degree)
    # kinds of the outer face's cell faces, by the midpoint of each edge
    mid = 0.5 * (outer[:-1] + outer[1:])
    if m == 2:
        thh = math.pi - 2.0 * math.pi * np.arange(2 * ntheta + 1) / (2 * ntheta)
        dx, dy = np.cos(thh), np.sin(thh)
        o2 = np.zeros((2 * ntheta + 1, 2))
        o2[0::2] = outer
        o2[1::2] = mid
        outer = o2
    inner = np.stack([cx + radius * dx, cy + radius * dy], axis=1)
    s = np.arange(m * nr + 1) / (m * nr)
    g = s if stretch == 0.0 else np.expm1(stretch * s) / math.expm1(stretch)
    # point (i, j): i around (fastest), j outwards
    V = inner[None, :, :] + g[:, None, None] * (outer - inner)[None, :, :]
    V = V.reshape(-1, 2)
    eps = 1e-9 * max(x1 - x0, y1 - y0)
    kinds = np.full(ntheta, BC_SLIP, dtype=np.int8)
    kinds[np.abs(mid[:, 0] - x0) < eps] = BC_DIRICHLET
    kinds[np.abs(mid[:, 0] - x1) < eps] = BC_OUTFLOW
    bc = (BC_PERIODIC, BC_PERIODIC, BC_SLIP, BC_SLIP)
    bc_cells = np.concatenate([np.full(ntheta, BC_SLIP, dtype=np.int8), kinds])
    free = to_conserved(np.array([GAMMA]), np.array([[mach], [0.0]]), np.array([1.0]))[:, 0]
    return V, bc, bc_cells, free


def annulus_ogrid(ntheta: int, nr: int, r0: float = 0.5, r1: float = 1.0, map_degree: int = 2) -> np.ndarray:
    """Points of an O-grid of the annulus r0 < r < r1 (axis 0 around,
    clockwise, periodic; axis 1 outwards): map_degree * n + 1 points per axis
    on circles and rays, so that quadratic cells (map_degree 2) follow the
    circles through their edge midpoints and bilinear ones (1) are polygons."""
    m = map_degree
    th = -2.0 * math.pi * np.arange(m * ntheta + 1) / (m * ntheta)
    r = r0 + (r1 - r0) * np.arange(m * nr + 1) / (m * nr)
    R, T = np.meshgrid(r, th, indexing="ij")  # (radial, angular): angular fastest
    return np.stack([R * np.cos(T), R * np.sin(T)], axis=-1).reshape(-1, 2)


def _rotations(dim):
    """The orientation-preserving symmetries of the reference square or cube,
    as integer matrices acting on centred coordinates."""
    out = []
    for perm in ([0, 1], [1, 0]) if dim == 2 else ([0, 1, 2], [0, 2, 1], [1, 0, 2], [1, 2, 0], [2, 0, 1], [2, 1, 0]):
        for signs in np.ndindex(*(2,) * dim):
            R = np.zeros((dim, dim), dtype=int)
            for r in range(dim):
                R[r, perm[r]] = 1 if signs[r] == 0 else -1
            if round(np.linalg.det(R)) == 1:
                out.append(R)
    return out


def unstructured_from_lattice(cells, points, bc, map_degree=1, seed=0, shuffle=True):
    """The lattice mesh of `points` (map_degree * n_e + 1 per axis, x fastest)
    written as an unstructured mesh: the point list, each cell's (g+1)^d
    point ids in a randomly rotated local order, the cells in a random order
    (seeded).  No axis may be periodic: an unstructured mesh connects cells
    through shared points only, and a translated periodic image is another
    point.  face_bc[K, f] = kind + 8 *
    the lattice face the part lies on (that face's data).

    Returns (cell_points, points, face_bc, perm, rot): cell perm[K] of the
    unstructured mesh is lattice cell K, with its local axes turned by rot[K]
    (an index into _rotations(d))."""
    d = len(cells)
    g = map_degree
    npa = [g * c + 1 for c in cells]
    P = np.asarray(points, dtype=np.float64)
    if any(b == 0 for b in bc):
        raise ValueError("periodic axes cannot be written as an unstructured mesh")

    def pid(idx):
        k, st = 0, 1
        for e in range(d):
            k += idx[e] * st
            st *= npa[e]
        return k
    ncells = int(np.prod(cells))
    rng = np.random.default_rng(seed)
    perm = rng.permutation(ncells) if shuffle else np.arange(ncells)
    rots = _rotations(d)
    rot = rng.integers(0, len(rots), size=ncells) if shuffle else np.zeros(ncells, dtype=int)
    np_ = (g + 1) ** d
    cp = np.zeros((ncells, np_), dtype=np.int64)
    fb = np.zeros((ncells, 2 * d), dtype=np.int8)
    for K in range(ncells):
        ki, r = [], K
        for e in range(d):
            ki.append(r % cells[e])
            r //= cells[e]
        R = rots[rot[K]]
        for v in range(np_):
            q, rr = [], v
            for e in range(d):
                q.append(rr % (g + 1))
                rr //= g + 1
            # new local position q comes from old position R^T (q - c) + c
            c = g / 2.0
            old = np.rint(R.T @ (np.array(q) - c) + c).astype(int)
            cp[perm[K], v] = pid([g * ki[e] + old[e] for e in range(d)])
        # local face f of the new cell: outward normal R e_f in old axes
        for f in range(2 * d):
            nvec = np.zeros(d, dtype=int)
            nvec[f // 2] = 1 if f % 2 else -1
            o = R.T @ nvec
            e = int(np.nonzero(o)[0][0])
            fo = 2 * e + (1 if o[e] > 0 else 0)
            on_bnd = (ki[e] == 0 and fo % 2 == 0) or (ki[e] == cells[e] - 1 and fo % 2 == 1)
            if on_bnd and bc[fo] != 0:
                fb[perm[K], f] = bc[fo] + 8 * fo
    return cp, P, fb, perm, rot


def triangle_three_blocks(n, corners=((0.0, 0.0), (1.0, 0.0), (0.3, 0.9)), map_degree=1):
    """An unstructured mesh of a triangle: three quadrilateral blocks (each
    corner, the two adjacent edge midpoints and the centroid), each cut into
    n x n cells by bilinear interpolation; the centroid has three cells.
    Returns (cell_points, points, face_bc with kind 0 everywhere; the caller
    sets the boundary kinds on the faces without a neighbour)."""
    A = [np.array(c, dtype=float) for c in corners]
    G = (A[0] + A[1] + A[2]) / 3.0
    blocks = []
    for i in range(3):
        a, b, c = A[i], A[(i + 1) % 3], A[(i + 2) % 3]
        blocks.append((a, 0.5 * (a + b), G, 0.5 * (a + c)))  # counterclockwise: a, mab, G, mac
    g = map_degree
    m = g * n
    pts, index = [], {}
    def point_id(x):
        key = (round(x[0], 12), round(x[1], 12))
        if key not in index:
            index[key] = len(pts)
            pts.append(x)
        return index[key]
    cps = []
    for (p00, p10, p11, p01) in blocks:
        ids = np.zeros((m + 1, m + 1), dtype=np.int64)
        for j in range(m + 1):
            for i in range(m + 1):
                s, t = i / m, j / m
                x = (1 - s) * (1 - t) * p00 + s * (1 - t) * p10 + s * t * p11 + (1 - s) * t * p01
                ids[j, i] = point_id(x)
        for cj in range(n):
            for ci in range(n):
                cps.append([ids[g * cj + qj, g * ci + qi] for qj in range(g + 1) for qi in range(g + 1)])
    cp = np.array(cps, dtype=np.int64)
    return cp, np.array(pts), np.zeros((len(cp), 4), dtype=np.int8)


def cylinder(ntheta: int = 512, nr: int = 128, degree: int = 1, mach: float = 3.0, stretch: float = 0.0,
             t_final: float = 4.0, map_degree: int = 1) -> Workload:
    """Mach 3 flow past a cylinder on the O-grid of cylinder_ogrid(): uniform
    free stream everywhere at t = 0 (the wall of the cylinder starts the bow
    shock)."""
    V, bc, bc_cells, free = cylinder_ogrid(ntheta, nr, degree, mach, stretch=stretch, map_degree=map_degree)
    bstate = (None, None, None, tuple(free))
    ms = MeshSpec(2, degree, (ntheta, nr), (0.0, -1.0), (4.0, 1.0), bc, bstate=bstate, vertices=V,
                  bc_cells=bc_cells, map_degree=map_degree)
    U = np.repeat(free[:, None], ms.ndofs, axis=1)
    name = "cylinder_q%d_%dx%d" % (degree, ntheta, nr) + ("_curved" if map_degree == 2 else "")
    return Workload(name, ms, U, t_final=t_final)


CONFIGS = {
    "sod": sod,
    "vortex": vortex,
    "quadrant": quadrant,
    "blast": blast,
    "inflow": inflow,
    "cylinder": cylinder,
}
