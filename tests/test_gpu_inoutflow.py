"""GPU parity of the sub- and supersonic in/outflow kind (Sec. 4.1,
eq. supersonic_inoutflow and eq. characteristics) and of boundary data taken
from the isentropic vortex at the node and the stage time (Sec. 6.2, 6.3),
against the oracle through the C-ABI (1e-11 of the component scale per dof
for a stage, 1e-10 after several steps), and the boundary experiment of
Sec. 6.3 run in full on the GPU.

The experiment: the vortex (beta 5, gamma 5/3, rho_inf = p_inf = 1) moving
with u_inf = (M, M) from (-1, -1) on [-5, 5]^2 until t_F = 6/M, when its core
sits on the top right corner; Q1, the limited scheme, SSP-RK3 (the paper uses
SSPRK-54); boundary data by strategy (a) exact Dirichlet data, (b) in/outflow
faces fed the exact data, (c) in/outflow faces fed the far-field state.
Context, Table ErrorBoundaryConditions: (a) and (b) converge at about second
order at every M; (c) only where the outflow is supersonic (M = 2, 2.5), its
rates fall towards 0 at M = 1.  Strategy (d), in/outflow faces fed the node's
own state at the start of the step (GDG_DATA_STEP_START), has its parity
cases here; the experiment does not run it: read that way, (d) turns the
inflow faces into do-nothing faces, and the oracle's own runs drift far from
the vortex at every M (24^2 cells: L1 1.17 at M = 2, where the table's (d)
equals (b)).
"""
import math

import numpy as np
import pytest

from paper_2402_04514_amd import gdg
from paper_2402_04514_amd import workloads as W

from test_gpu_parity import _check_ev, _close

pytestmark = pytest.mark.gpu
G53 = 5.0 / 3.0


def _say(msg):
    print("[gpu-inoutflow] " + msg, flush=True)


def vortex_case(n, M, bc, degree=1, far=False, x0=(-1.0, -1.0)):
    ms = W.MeshSpec(2, degree, (n, n), (-5.0, -5.0), (5.0, 5.0), (bc,) * 4)
    x, _ = W.node_coords(ms)
    U0 = W.vortex_exact(x, 0.0, x0=x0, uinf=(M, M), gamma=G53, periodic=False)
    if far:
        Uf = tuple(W.to_conserved(np.array([1.0]), np.array([[M], [M]]), np.array([1.0]), G53)[:, 0])
        ms = W.MeshSpec(2, degree, ms.cells, ms.lo, ms.hi, ms.bc, bstate=(Uf,) * 4)
    else:
        ms = W.MeshSpec(2, degree, ms.cells, ms.lo, ms.hi, ms.bc, vortex=(5.0, x0[0], x0[1], M, M, G53))
    return ms, U0


def _pair(oracle, ms, U):
    M = oracle.Mesh(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc, bstate=ms.bstate, vortex=ms.vortex)
    p = gdg.gdg_default_params(ms.degree)
    p.gamma = G53
    S = gdg.Solver.from_spec(ms, p)
    S.upload(U)
    return M, S, oracle.params(gamma=G53, degree=ms.degree)


CASES = {
    # the vortex core near the top right corner, so that its subsonic part
    # leaves through in/outflow faces; M = 1 is subsonic at those faces
    "dirichlet_vortex_q1": lambda: vortex_case(12, 1.0, W.BC_DIRICHLET, x0=(3.0, 3.0)),
    "inoutflow_vortex_q1_m1": lambda: vortex_case(12, 1.0, W.BC_INOUTFLOW, x0=(3.0, 3.0)),
    "inoutflow_vortex_q1_m2": lambda: vortex_case(12, 2.0, W.BC_INOUTFLOW, x0=(3.0, 3.0)),
    "inoutflow_vortex_q2_m1": lambda: vortex_case(8, 1.0, W.BC_INOUTFLOW, degree=2, x0=(3.0, 3.0)),
    "inoutflow_vortex_q3_m1": lambda: vortex_case(6, 1.0, W.BC_INOUTFLOW, degree=3, x0=(3.0, 3.0)),
    "inoutflow_farfield_q1_m1": lambda: vortex_case(12, 1.0, W.BC_INOUTFLOW, far=True, x0=(3.0, 3.0)),
}


def _plain(n, M, bc, degree=1, x0=(3.0, 3.0)):
    """The vortex box with no data source: the data kind comes from the caller."""
    ms = W.MeshSpec(2, degree, (n, n), (-5.0, -5.0), (5.0, 5.0), (bc,) * 4)
    x, _ = W.node_coords(ms)
    return ms, W.vortex_exact(x, 0.0, x0=x0, uinf=(M, M), gamma=G53, periodic=False)


def _smooth3d():
    ms = W.MeshSpec(3, 1, (5, 4, 3), (0.0,) * 3, (1.0,) * 3, (W.BC_INOUTFLOW, W.BC_INOUTFLOW, 2, 2, 0, 0))
    x, _ = W.node_coords(ms)
    f = lambda s: np.sin(2 * np.pi * x[:, 0] + s) * np.cos(2 * np.pi * x[:, 2])
    U = W.to_conserved(1.0 + 0.2 * f(0.3), np.stack([0.4 + 0.1 * f(1.0), 0.1 * f(2.0), 0.1 * f(0.7)]),
                       1.0 + 0.2 * f(1.9), G53)
    return ms, U


def _general():
    ms, U = _plain(10, 1.0, W.BC_INOUTFLOW)
    V = W.perturbed_lattice(ms.cells, ms.lo, ms.hi, amp=0.2, seed=11)
    return W.MeshSpec(2, 1, ms.cells, ms.lo, ms.hi, ms.bc, vertices=V), None  # U at the mapped nodes below


# strategy (d): (case, integrator)
STEP_START = {
    "inoutflow_q1_m1": (lambda: _plain(12, 1.0, W.BC_INOUTFLOW), gdg.GDG_SSPRK3),
    "inoutflow_q1_m1_ssprk54": (lambda: _plain(12, 1.0, W.BC_INOUTFLOW), gdg.GDG_SSPRK54),
    "inoutflow_q2_m2": (lambda: _plain(8, 2.0, W.BC_INOUTFLOW, degree=2), gdg.GDG_SSPRK3),
    "dirichlet_q1_m1": (lambda: _plain(12, 1.0, W.BC_DIRICHLET), gdg.GDG_SSPRK3),
    "inoutflow_3d_q1": (_smooth3d, gdg.GDG_SSPRK3),
    "inoutflow_general_q1_m1": (_general, gdg.GDG_SSPRK3),
}


@pytest.mark.parametrize("name", sorted(STEP_START))
def test_step_start_data(oracle, name):
    """Strategy (d): the data of the in/outflow (or Dirichlet) faces are the
    node's own state at the start of the step.  A stage and twelve steps
    against the oracle's."""
    _say("step-start data " + name)
    make, integ = STEP_START[name]
    ms, U = make()
    M = oracle.Mesh(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc, vertices=ms.vertices, step_start_data=True)
    if U is None:
        U = W.vortex_exact(M.coords(), 0.0, x0=(3.0, 3.0), uinf=(1.0, 1.0), gamma=G53, periodic=False)
    p = gdg.gdg_default_params(ms.degree)
    p.gamma = G53
    p.integrator = integ
    S = gdg.Solver.from_spec(ms, p, step_start_data=True)
    S.upload(U)
    op = oracle.params(gamma=G53, degree=ms.degree, integrator=integ)
    out, dg = M.stage(op, U, diag=True)
    assert dg["status"] == 0
    assert S.stage(0.0) == pytest.approx(op.cfl * dg["tau_max"], rel=1e-13)
    _close(S.field(gdg.GDG_FIELD_UL), dg["UL"], what="U^L")
    _close(S.download(), out, what="Phi(U)")
    S.upload(U)
    Uo, t_o, n_o = M.run_to(op, U, 1e30, max_steps=12)
    st = S.run_to(1e30, max_steps=12)
    assert st.steps == n_o == 12 and st.t == pytest.approx(t_o, rel=1e-12)
    assert st.bound_violations == 0
    _close(S.download(), Uo, tol=1e-10, what="U after 12 steps")


@pytest.mark.parametrize("name", sorted(CASES))
def test_stage_fields_and_steps(oracle, name):
    _say("stage fields and steps " + name)
    ms, U = CASES[name]()
    M, S, op = _pair(oracle, ms, U)
    M.set_time(0.0)
    out, dg = M.stage(op, U, diag=True)
    assert dg["status"] == 0
    tau_g = S.stage(0.0)
    assert tau_g == pytest.approx(op.cfl * dg["tau_max"], rel=1e-13)
    _close(S.field(gdg.GDG_FIELD_UL), dg["UL"], what="U^L")
    B = S.field(gdg.GDG_FIELD_BOUNDS)
    _close(B, np.stack([dg["rho_min"], dg["rho_max"], dg["s_min"]]), what="bounds")
    _check_ev(S.field(gdg.GDG_FIELD_EV_N)[0], dg)
    _close(S.field(gdg.GDG_FIELD_DUH), dg["dUH"], what="dU^H")
    _close(S.field(gdg.GDG_FIELD_U1), dg["U1"], what="U^(1)")
    _close(S.download(), out, what="Phi(U)")
    # whole steps: the stages take the data at t, t + tau, t + tau / 2
    S.upload(U)
    Uo, t_o, n_o = M.run_to(op, U, 1e30, max_steps=12)
    st = S.run_to(1e30, max_steps=12)
    assert st.steps == n_o == 12 and st.t == pytest.approx(t_o, rel=1e-12)
    assert st.bound_violations == 0
    _close(S.download(), Uo, tol=1e-10, what="U after 12 steps")


def test_no_characteristic_state_is_reported():
    """Data whose incoming characteristic leaves no positive sound speed
    (a strong expansion against the node's state): the step fails with
    GDG_E_BOUNDARY instead of inventing a state."""
    ms = W.MeshSpec(1, 1, (8,), (0.0,), (1.0,), (W.BC_INOUTFLOW,) * 2,
                    bstate=(tuple(W.to_conserved(np.array([1.0]), np.array([[-30.0]]), np.array([1.0]))[:, 0]),
                            tuple(W.to_conserved(np.array([1.0]), np.array([[30.0]]), np.array([1.0]))[:, 0])))
    U = W.to_conserved(np.ones(16), np.zeros((1, 16)), np.ones(16))
    S = gdg.Solver.from_spec(ms)
    S.upload(U)
    with pytest.raises(gdg.GdgError) as ei:
        S.step()
    assert ei.value.status == gdg.GDG_E_BOUNDARY


def _l1(U, Uex, mi):
    e = np.sum(np.abs(U[0] - Uex[0]) * mi) / np.sum(np.abs(Uex[0]) * mi)
    dm = np.sqrt(np.sum((U[1:3] - Uex[1:3]) ** 2, 0))
    e += np.sum(dm * mi) / np.sum(np.sqrt(np.sum(Uex[1:3] ** 2, 0)) * mi)
    e += np.sum(np.abs(U[3] - Uex[3]) * mi) / np.sum(np.abs(Uex[3]) * mi)
    return e


def test_boundary_experiment_of_sec_6_3(oracle):
    sizes = (24, 48, 96, 192)  # 2304 ... 147456 dofs, as the first four rows of the paper's table
    table = {}
    for strat, bc, far in (("a", W.BC_DIRICHLET, False), ("b", W.BC_INOUTFLOW, False), ("c", W.BC_INOUTFLOW, True)):
        for Mach in (1.0, 1.5, 2.0, 2.5):
            tf = 6.0 / Mach
            errs = []
            for n in sizes:
                ms, U0 = vortex_case(n, Mach, bc, far=far)
                p = gdg.gdg_default_params(1)
                p.gamma = G53
                S = gdg.Solver.from_spec(ms, p)
                S.upload(U0)
                st = S.run_to(tf)
                U = S.download()
                assert st.t == tf and st.bound_violations == 0
                mi = np.tile(oracle.Mesh(2, 1, (1, 1), (0, 0), (1, 1), (1,) * 4).lumped(), ms.ncells)
                Uex = W.vortex_exact(W.node_coords(ms)[0], tf, x0=(-1.0, -1.0), uinf=(Mach, Mach), gamma=G53,
                                     periodic=False)
                errs.append(_l1(U, Uex, mi))
                S.close()
            rates = [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
            table[strat, Mach] = (errs, rates)
            _say("strategy (%s) M = %.1f: L1 %s rates %s" % (strat, Mach, ["%.3e" % e for e in errs],
                                                               ["%.2f" % r for r in rates]))
    for Mach in (1.0, 1.5, 2.0, 2.5):
        for strat in ("a", "b"):
            assert table[strat, Mach][1][-1] > 1.5, (strat, Mach, table[strat, Mach])
    for Mach in (2.0, 2.5):
        assert table["c", Mach][1][-1] > 1.5, (Mach, table["c", Mach])
    # far-field data where the outflow is subsonic: the error stalls
    assert table["c", 1.0][1][-1] < 1.0, table["c", 1.0]
    assert table["c", 1.0][0][-1] > 5.0 * table["b", 1.0][0][-1]


# Table ErrorIsentropicConvex of the paper (L1, limited scheme, SSPRK-54):
# the first four refinement levels (2304 ... 147456 dofs)
PAPER_L1 = {1: (0.0225513, 0.00728095, 0.00206252, 0.000548656),
            2: (0.00978699, 0.00114886, 0.000156191, 2.0117e-05),
            3: (0.00335439, 0.000256794, 1.70566e-05, 1.14504e-06)}

# (degree, parameter overrides, levels, largest ratio to the table's error,
# smallest rate over the last two levels (their mean for Q2))
TABLE_CASES = {
    "q1": (1, {}, 4, 1.5, 1.75),
    "q2": (2, {}, 4, 1.6, 2.7),
    # the Q3 bounds relaxed with p_r = 1 instead of 1.5
    "q3_pr1": (3, {"p_r": 1.0}, 4, 1.5, 3.5),
    "q3_unlimited": (3, {"scheme": gdg.GDG_HIGH_ORDER}, 4, 1.5, 3.5),
    # the paper's constants: the entropy bound cuts fluxes at every level
    "q3_paper_constants": (3, {}, 3, None, 1.2),
    # the paper's integrator, SSPRK(5,4)
    "q1_ssprk54": (1, {"integrator": gdg.GDG_SSPRK54}, 4, 1.5, 1.75),
    "q2_ssprk54": (2, {"integrator": gdg.GDG_SSPRK54}, 4, 1.6, 2.7),
    "q3_pr1_ssprk54": (3, {"p_r": 1.0, "integrator": gdg.GDG_SSPRK54}, 4, 1.5, 3.5),
    "q3_unlimited_ssprk54": (3, {"scheme": gdg.GDG_HIGH_ORDER, "integrator": gdg.GDG_SSPRK54}, 4, 1.5, 3.5),
    "q3_paper_constants_ssprk54": (3, {"integrator": gdg.GDG_SSPRK54}, 3, None, 1.2),
}


@pytest.mark.parametrize("name", sorted(TABLE_CASES))
def test_vortex_with_exact_boundary_data(oracle, name):
    """The vortex test (i) of Sec. 6.2: gamma = 5/3, [-5, 5]^2, Dirichlet
    data from the exact solution at the node and the stage time, t_F = 2,
    n_k 2^r cells per edge with n_k = 24, 16, 12 for k = 1, 2, 3, against
    Table ErrorIsentropicConvex (there SSPRK-54; here both SSP-RK3 and
    SSPRK(5,4), at Cr = 0.5).

    Measured: Q1 at 0.84-0.85 of the table's errors with its rates (1.63,
    1.81, 1.91); Q2 at 1.02-1.39 of them, rates 2.64, 3.31, 2.54.  For Q3
    with c_r = 4, p_r = 1.5 the rescaled-entropy bound of eq. local_bounds
    binds on the directional states of Lemma ConsInvariants (relaxed by
    c_r hhat_i^p_r, hhat_i = (m_i/|Omega|)^(1/d), about 1e-4 at the Gauss-
    Lobatto corner nodes of the finest level): errors 4.4e-3, 9.2e-4,
    2.8e-4, 9.7e-5, rates 2.3, 1.7, 1.5, where the table has 3.7-3.9.  With
    p_r = 1 (or without limiting) the errors are 0.77-1.10 of the table's
    and the rates 3.65, 4.37, 3.96.

    SSPRK(5,4) gives the same errors to four digits for Q1, Q3 with p_r = 1
    and unlimited Q3 (the spatial error dominates at Cr = 0.5), Q2 errors
    lower by up to 6% (1.01-1.39 of the table's, rates 2.64, 3.36, 2.58), and
    Q3 with the paper's constants 4.3e-3, 8.4e-4, 2.5e-4: the rate loss comes
    from the entropy bound, not from the time integration."""
    k, over, levels, factor, rate_floor = TABLE_CASES[name]
    nk = {1: 24, 2: 16, 3: 12}[k]
    mi1 = oracle.Mesh(2, k, (1, 1), (0, 0), (1, 1), (1,) * 4).lumped()
    errs = []
    for r in range(levels):
        n = nk * 2 ** r
        ms = W.MeshSpec(2, k, (n, n), (-5.0, -5.0), (5.0, 5.0), (W.BC_DIRICHLET,) * 4,
                        vortex=(5.0, -1.0, -1.0, 1.0, 1.0, G53))
        x, _ = W.node_coords(ms)
        U0 = W.vortex_exact(x, 0.0, gamma=G53, periodic=False)
        p = gdg.gdg_default_params(k)
        p.gamma = G53
        for a, b in over.items():
            setattr(p, a, b)
        S = gdg.Solver.from_spec(ms, p)
        S.upload(U0)
        st = S.run_to(2.0)
        U = S.download()
        S.close()
        assert st.t == 2.0 and st.bound_violations == 0
        mi = np.tile(mi1 * (10.0 / n) ** 2, ms.ncells)
        errs.append(_l1(U, W.vortex_exact(x, 2.0, gamma=G53, periodic=False), mi))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(levels - 1)]
    ratio = [errs[i] / PAPER_L1[k][i] for i in range(levels)]
    _say("%s: L1 %s rates %s, ratio to the table %s" % (
        name, ["%.3e" % e for e in errs], ["%.2f" % r for r in rates], ["%.2f" % q for q in ratio]))
    if factor is not None:
        assert max(ratio) < factor and min(ratio) > 1.0 / factor, (errs, ratio)
    tail = rates[-2:]
    if k == 2:
        assert sum(tail) / 2 > rate_floor, (errs, rates)
    else:
        assert min(tail) > rate_floor, (errs, rates)
