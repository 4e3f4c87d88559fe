"""GPU parity of the Dirichlet and supersonic in/outflow boundary kinds
(Sec. 4.1: Dirichlet data; eq. supersonic_inoutflow) against the oracle,
through the C-ABI, at the tolerances of the other parity tests (1e-11 of the
component scale per dof for a stage, 1e-10 after several steps; the scale of
a component that is zero up to rounding is 1e-3 of the largest).

Cases: the supersonic inflow problem in 1D, along y in 2D (Q2) and along x in
3D; quadrant data with Dirichlet faces (each face its own data) in 1D, 2D and
3D next to outflow, slip and periodic faces; the smallest meshes (two cells
per axis, every row a boundary row) with Dirichlet faces; an oblique supersonic stream with
a smooth perturbation and supersonic kinds on every face.  Also: equivalence
with outflow bit for bit upstream of a supersonic stream (the data's node
fields equal the node cache of the same state), the subsonic report
(GDG_E_BOUNDARY) on both the eager and the graph path, the mixed variant, and
a request served with Dirichlet data.
"""
import numpy as np
import pytest

from paper_2402_04514_amd import gdg
from paper_2402_04514_amd import workloads as W

from test_gpu_parity import _check_ev, _close, quadrant_on, smooth_on
from test_gpu_mixed import l1_rel

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-boundary] " + msg, flush=True)


def _with_data(ms, U, faces, seed=3):
    """The mesh of (ms, U) with Dirichlet data on `faces`: admissible states
    drawn from the quadrant state table, one per face."""
    st = np.array(W.quadrant_states(seed))
    bstate = []
    for f in range(2 * ms.dim):
        if f not in faces:
            bstate.append(None)
            continue
        r, u, v, p = st[f % 4]
        vel = np.zeros((ms.dim, 1))
        vel[0] = u
        if ms.dim > 1:
            vel[1] = v
        bstate.append(tuple(W.to_conserved(np.array([r]), vel, np.array([p]))[:, 0]))
    return W.MeshSpec(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc, tuple(bstate)), U


def _inflow(dim, axis, degree, cells, cross):
    wl = W.inflow(cells, dim=dim, axis=axis, degree=degree, cross=cross)
    U = wl.U0.copy()
    # a smooth density bump inside the stream, so that every stage has
    # structure away from the faces too
    x = W.node_coords(wl.mesh)[0][:, axis]
    U[:] *= (1.0 + 0.2 * np.exp(-80.0 * (x - 0.6) ** 2))[None, :]
    return wl.mesh, U


def _oblique(dim, degree, cells, kind=W.BC_SUPERSONIC):
    ms, U = smooth_on(dim, degree, cells, (kind,) * (2 * dim), seed=11)
    n = ms.ndofs
    rho = np.full(n, 1.0)
    vel = np.zeros((dim, n))
    vel[0] = 2.4
    if dim > 1:
        vel[1] = -2.1
    if dim > 2:
        vel[2] = 1.9
    base = W.to_conserved(rho, vel, np.full(n, 0.6))
    Ub = base * (1.0 + 0.05 * (U[0] - 1.0))[None, :]
    bstate = tuple(tuple(base[:, 0]) for _ in range(2 * dim))
    return W.MeshSpec(dim, degree, ms.cells, ms.lo, ms.hi, ms.bc, bstate), Ub


CASES = {
    "inflow_1d_q1": lambda: _inflow(1, 0, 1, 40, 1),
    "inflow_2d_q2_y": lambda: _inflow(2, 1, 2, 12, 3),
    "inflow_3d_q1_x": lambda: _inflow(3, 0, 1, 10, 2),
    "dirichlet_1d_q2": lambda: _with_data(*quadrant_on(1, 2, (17,), (3, 3)), faces=(0, 1)),
    "dirichlet_2d_q1_ragged": lambda: _with_data(*quadrant_on(2, 1, (11, 9), (3, 1, 2, 3)), faces=(0, 3)),
    "dirichlet_2d_q2_all": lambda: _with_data(*quadrant_on(2, 2, (7, 8), (3,) * 4, seed=9), faces=(0, 1, 2, 3)),
    "dirichlet_3d_q1_mixed": lambda: _with_data(*quadrant_on(3, 1, (5, 4, 4), (3, 1, 0, 0, 2, 3), seed=3),
                                                faces=(0, 5)),
    "two_cells_2d_dirichlet": lambda: _with_data(*smooth_on(2, 1, (2, 2), (3, 3, 3, 3)), faces=(0, 1, 2, 3)),
    "two_cells_3d_q2_dirichlet": lambda: _with_data(*smooth_on(3, 2, (2, 2, 2), (3, 1, 2, 3, 3, 2)),
                                                    faces=(0, 3, 4)),
    "supersonic_2d_oblique": lambda: _oblique(2, 1, (9, 8)),
    "supersonic_3d_q2_oblique": lambda: _oblique(3, 2, (3, 3, 2)),
}


def _close_u(a, b, U, tol=1e-11, what=""):
    """|a - b| within tol of the component scale of the state U, per dof (a
    component that is zero up to rounding, such as the cross-stream momentum,
    is measured against 1e-3 of the largest component)."""
    s = np.abs(U).max(axis=1, keepdims=True)
    s = np.maximum(s, 1e-3 * s.max())
    err = (np.abs(np.asarray(a).reshape(b.shape) - b) / s).max()
    assert err <= tol, "%s: worst relative error %.3e (tol %.1e)" % (what, err, tol)


def _pair(oracle, name, precision=gdg.GDG_FP64):
    ms, U = CASES[name]()
    M = oracle.Mesh(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc, bstate=ms.bstate)
    p = gdg.gdg_default_params(ms.degree)
    p.precision = precision
    S = gdg.Solver.from_spec(ms, p)
    S.upload(U)
    return ms, U, M, S, oracle.params(degree=ms.degree)


@pytest.mark.parametrize("name", sorted(CASES))
def test_boundary_stage_fields(oracle, name):
    _say("stage fields " + name)
    ms, U, M, S, op = _pair(oracle, name)
    out, dg = M.stage(op, U, diag=True)
    assert dg["status"] == 0
    tau_g = S.stage(0.0)
    assert tau_g == pytest.approx(op.cfl * dg["tau_max"], rel=1e-13)
    _close_u(S.field(gdg.GDG_FIELD_UL), dg["UL"], U, what="U^L")
    B = S.field(gdg.GDG_FIELD_BOUNDS)
    _close(B, np.stack([dg["rho_min"], dg["rho_max"], dg["s_min"]]), what="bounds")
    _check_ev(S.field(gdg.GDG_FIELD_EV_N)[0], dg)
    _close_u(S.field(gdg.GDG_FIELD_DUH), dg["dUH"], U, what="dU^H")
    _close_u(S.field(gdg.GDG_FIELD_U1), dg["U1"], U, what="U^(1)")
    _close_u(S.download(), out, U, what="Phi(U)")


@pytest.mark.parametrize("name", sorted(CASES))
def test_boundary_graph_run(oracle, name):
    """Ten steps through run_to (captured graphs) against ten oracle steps."""
    _say("graph run " + name)
    ms, U, M, S, op = _pair(oracle, name)
    Uo, t_o, n_o = M.run_to(op, U, 1e30, max_steps=10)
    st = S.run_to(1e30, max_steps=10)
    assert st.steps == n_o == 10
    assert st.t == pytest.approx(t_o, rel=1e-12)
    _close_u(S.download(), Uo, U, tol=1e-10, what="U after 10 steps")


def test_inflow_to_final_time_mixed(oracle):
    """The mixed variant on the inflow problem to t = 0.1: L1 within 1e-5."""
    wl = W.inflow(100)
    ms = wl.mesh
    M = oracle.Mesh(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc, bstate=ms.bstate)
    Uo, _, _ = M.run_to(oracle.params(), wl.U0, 0.1)
    p = gdg.gdg_default_params(1)
    p.precision = gdg.GDG_MIXED
    S = gdg.Solver.from_spec(ms, p)
    S.upload(wl.U0)
    st = S.run_to(0.1)
    assert st.t == 0.1
    e = l1_rel(S.download(), Uo, M.lumped())
    _say("  inflow mixed L1 %s" % np.array2string(e, precision=2))
    assert e.max() <= 1e-5


def test_supersonic_equals_outflow_upstream():
    """Upstream of a supersonic stream the data equals the boundary nodes'
    state, so the supersonic kind gives the outflow result bit for bit: the
    device-built node fields of the data equal the node cache."""
    # the step sits at x = 3/4: by t = 0.1 the scheme's upstream numerical
    # foot has changed no dof left of x = 0.47 (the oracle's run), so the
    # inflow nodes still hold the data exactly
    w0 = W.inflow(128)
    U0 = w0.U0.copy()
    U0[:, : 3 * U0.shape[1] // 4] = np.array(w0.mesh.bstate[0])[:, None]
    out = W.MeshSpec(1, 1, w0.mesh.cells, w0.mesh.lo, w0.mesh.hi, (W.BC_OUTFLOW, W.BC_OUTFLOW))
    res = []
    for ms in (w0.mesh, out):
        S = gdg.Solver.from_spec(ms)
        S.upload(U0)
        st = S.run_to(0.1)
        res.append((S.download(), st.steps))
    assert res[0][1] == res[1][1]
    assert np.array_equal(res[0][0], res[1][0])


def test_subsonic_flow_at_supersonic_face_reported():
    wl = W.sod(20)
    ms = W.MeshSpec(1, 1, wl.mesh.cells, wl.mesh.lo, wl.mesh.hi, (W.BC_SUPERSONIC, W.BC_OUTFLOW),
                    (tuple(wl.U0[:, 0]), None))
    for path in ("step", "run_to"):
        S = gdg.Solver.from_spec(ms)
        S.upload(wl.U0)
        with pytest.raises(gdg.GdgError) as ei:
            if path == "step":
                S.step()
            else:
                S.run_to(0.1)
        assert ei.value.status == gdg.GDG_E_BOUNDARY, path
        S.close()


def test_served_request_with_dirichlet_data():
    """A request with Dirichlet and supersonic faces through the server: the
    same result as the single-mesh path (1e-12; the two paths are separately
    compiled kernels)."""
    reqs = [_inflow(2, 1, 1, 24, 3), _with_data(*quadrant_on(2, 1, (9, 10), (3, 1, 2, 3)), faces=(0, 3))]
    S = gdg.Server(2, 1, gdg.GDG_FP64, budget_bytes=256 << 20, max_slots=4, steps_per_graph=4)
    tickets = [S.submit(ms, U, 0.01) for ms, U in reqs]
    for _ in range(100000):
        res, pend = S.pump()
        if res == 0 and pend == 0:
            break
    S.sync()
    for t, (ms, U) in zip(tickets, reqs):
        info = S.poll(t)
        assert info.state == gdg.GDG_REQ_DONE and info.t == 0.01
        got = S.result(t)
        A = gdg.Solver.from_spec(ms)
        A.upload(U)
        st = A.run_to(0.01)
        assert st.steps == info.steps
        ref = A.download()
        scale = np.abs(ref).max(axis=1, keepdims=True)
        scale = np.maximum(scale, 1e-3 * scale.max())
        assert (np.abs(got - ref) / scale).max() <= 1e-12
    S.close()
