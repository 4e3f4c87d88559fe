"""Pins of the oracle's Dirichlet and supersonic in/outflow boundary data
(Sec. 4.1: Dirichlet data; eq. supersonic_inoutflow).

* Supersonic inflow into a supersonic stream: every wave of the Riemann problem
  between the inflow data and the stream moves into the box, so the exact
  solution is that Riemann fan centred on the inflow face.  The scheme
  converges to it at first order (L1, discontinuous data), in 1D and along
  the y axis of a 2D mesh; with the inflow face made an outflow face instead,
  the error stays large, so the data is what drives the solution.
* Dirichlet data equal to the state the boundary nodes hold gives the same
  ghost state as outflow: identical runs while the waves are inside (bit for
  bit upstream of a supersonic stream; within the numerical foot of the
  waves, 1e-12, where the boundary state is at rest).
* Dirichlet data on the faces of the inflow problem gives the supersonic
  result bit for bit (the inflow face takes the data either way, and the
  outflow face still holds the data).
* A uniform state that equals the data of every face stays exactly uniform.
* Subsonic normal flow at a supersonic face is reported (status -4).
"""
import math

import numpy as np
import pytest

from paper_2402_04514_amd import workloads as W

G = 1.4


def make(O, ms):
    return O.Mesh(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc, bstate=ms.bstate)


def _l1_rho(M, U, rho_ex):
    mi = M.lumped()
    return np.sum(np.abs(U[0] - rho_ex) * mi) / np.sum(np.abs(rho_ex) * mi)


def _exact_rho(O, x, t):
    left = W.INFLOW
    right = W.DOWNSTREAM
    return np.array([O.riemann_sample(G, left, right, xx / t)[0] for xx in x])


@pytest.mark.parametrize("dim,axis", [(1, 0), (2, 1)])
def test_supersonic_inflow_converges_to_riemann_fan(oracle, dim, axis):
    tf = 0.2
    errs = []
    sizes = (50, 100, 200) if dim == 1 else (40, 80, 160)
    for n in sizes:
        wl = W.inflow(n, dim=dim, axis=axis, cross=2)
        M = make(oracle, wl.mesh)
        U, t, _ = M.run_to(oracle.params(), wl.U0, tf)
        assert t == pytest.approx(tf, abs=1e-15)
        x = M.coords()[:, axis]
        errs.append(_l1_rho(M, U, _exact_rho(oracle, x, tf)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 0.02, errs
    assert all(0.6 < r < 1.4 for r in rates), (errs, rates)


def test_dirichlet_inflow_equals_supersonic(oracle):
    a = W.inflow(60)
    b = W.inflow(60, kind=W.BC_DIRICHLET)
    # t = 0.1: the fastest wave's numerical foot has not reached the outflow face
    Ua, ta, na = make(oracle, a.mesh).run_to(oracle.params(), a.U0, 0.1)
    Ub, tb, nb = make(oracle, b.mesh).run_to(oracle.params(), b.U0, 0.1)
    assert (ta, na) == (tb, nb)
    assert np.array_equal(Ua, Ub)
    assert np.max(np.abs(Ua - a.U0)) > 0.1


def test_inflow_data_drives_the_solution(oracle):
    """The same problem with the inflow face as outflow keeps the stream:
    far from the exact fan."""
    wl = W.inflow(100)
    ms = wl.mesh
    out = W.MeshSpec(1, 1, ms.cells, ms.lo, ms.hi, (W.BC_OUTFLOW, W.BC_OUTFLOW))
    M = make(oracle, out)
    U, _, _ = M.run_to(oracle.params(), wl.U0, 0.2)
    assert np.max(np.abs(U - wl.U0)) == 0.0
    assert _l1_rho(M, U, _exact_rho(oracle, M.coords()[:, 0], 0.2)) > 0.3


@pytest.mark.parametrize("kind", [W.BC_DIRICHLET, W.BC_SUPERSONIC])
def test_data_equal_to_boundary_state_matches_outflow(oracle, kind):
    """Sod data (subsonic, so Dirichlet) and the inflow stream (supersonic):
    while no wave reaches a face, the boundary nodes keep the data, the ghost
    states equal outflow's U_i, and the runs agree bit for bit."""
    if kind == W.BC_DIRICHLET:
        wl = W.sod(100)
        ms0 = wl.mesh
        bstate = (tuple(wl.U0[:, 0]), tuple(wl.U0[:, -1]))
        ms = W.MeshSpec(1, 1, ms0.cells, ms0.lo, ms0.hi, (kind, kind), bstate)
        U0, tf = wl.U0, 0.2
    else:
        w0 = W.inflow(128)
        U0 = w0.U0.copy()
        U0[:, : 3 * U0.shape[1] // 4] = np.array(w0.mesh.bstate[0])[:, None]  # a step at x = 3/4
        ms, tf = w0.mesh, 0.1
    Ma = make(oracle, ms)
    Mb = make(oracle, W.MeshSpec(1, 1, ms.cells, ms.lo, ms.hi, (W.BC_OUTFLOW, W.BC_OUTFLOW)))
    Ua, ta, na = Ma.run_to(oracle.params(), U0, tf)
    Ub, tb, nb = Mb.run_to(oracle.params(), U0, tf)
    assert na == nb and ta == tb
    if kind == W.BC_SUPERSONIC:
        assert np.array_equal(Ua, Ub)
    else:
        assert np.max(np.abs(Ua - Ub)) <= 1e-12


@pytest.mark.parametrize("kind", [W.BC_DIRICHLET, W.BC_SUPERSONIC])
def test_uniform_state_equal_to_data_is_kept(oracle, kind):
    """An oblique uniform stream (supersonic along the diagonal, so every face
    is either inflow or outflow) that equals every face's data."""
    ms0 = W.MeshSpec(2, 2, (5, 4), (0.0, 0.0), (1.0, 2.0), (kind,) * 4)
    n = ms0.ndofs
    vel = np.stack([np.full(n, 2.2), np.full(n, -1.9)])
    U = W.to_conserved(np.full(n, 0.9), vel, np.full(n, 0.7))
    ms = W.MeshSpec(2, 2, ms0.cells, ms0.lo, ms0.hi, ms0.bc, (tuple(U[:, 0]),) * 4)
    M = make(oracle, ms)
    Un = U
    for _ in range(5):
        Un, dt, nres, st = M.step(oracle.params(degree=2), Un)
        assert st == 0 and nres == 0
    assert np.max(np.abs(Un - U) / np.abs(U).max(1, keepdims=True)) <= 1e-14


def test_subsonic_flow_at_supersonic_face_reported(oracle):
    wl = W.sod(20)
    ms = W.MeshSpec(1, 1, wl.mesh.cells, wl.mesh.lo, wl.mesh.hi, (W.BC_SUPERSONIC, W.BC_OUTFLOW),
                    (tuple(wl.U0[:, 0]), None))
    M = make(oracle, ms)
    out, dg = M.stage(oracle.params(), wl.U0, diag=True)
    assert dg["status"] == -4
    _, _, _, st = M.step(oracle.params(), wl.U0)
    assert st == -4


def test_dirichlet_needs_data(oracle):
    with pytest.raises(ValueError):
        oracle.Mesh(1, 1, (4,), (0.0,), (1.0,), (W.BC_DIRICHLET, W.BC_OUTFLOW))
