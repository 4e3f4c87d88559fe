"""GPU mixed-precision variant (GDG_MIXED) against the FP64 CPU oracle.

The variant stores c_ij in FP32 and accumulates the flux sums of the low-
and high-order updates and the entropy-residual sums in FP32; the state,
d_ij, bar states, bounds and the line search stay in FP64.  Its results therefore differ from the FP64 scheme by FP32 rounding of
those sums, about 1e-7 of the flux scale per stage, and the stated bound is an
L1 (mass-weighted, per component) error of at most 1e-5 relative to the FP64
oracle, after whole runs.  Invariant-set properties hold exactly: every stage
output is checked for rho > 0, eps > 0 on the device.
"""
import numpy as np
import pytest

from paper_2402_04514_amd import gdg
from paper_2402_04514_amd import workloads as W

from test_gpu_parity import CASES, quadrant_on

pytestmark = pytest.mark.gpu
L1_TOL = 1e-5


def _say(msg):
    print("[gpu-mixed] " + msg, flush=True)


def _mixed_params(degree):
    p = gdg.gdg_default_params(degree)
    p.precision = gdg.GDG_MIXED
    return p


def _setup(oracle, ms, U):
    M = oracle.Mesh(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc)
    p = _mixed_params(ms.degree)
    S = gdg.Solver.from_spec(ms, p)
    S.upload(U)
    op = oracle.params(degree=ms.degree)
    return M, S, op


def l1_rel(Ug, Uo, mi):
    """Per component: sum_i m_i |Ug - Uo| / sum_i m_i |Uo| (a component whose
    norm is below 1e-3 of the largest is measured against the largest)."""
    num = (np.abs(Ug - Uo) * mi).sum(1)
    den = (np.abs(Uo) * mi).sum(1)
    den = np.maximum(den, 1e-3 * den.max())
    return num / den


def _admissible(U, dim):
    eps = U[dim + 1] - 0.5 * np.sum(U[1:dim + 1] ** 2, 0) / U[0]
    return bool(np.all(U[0] > 0) and np.all(eps > 0))


@pytest.mark.parametrize("name", ["sod_q1_40", "q1_2d_outflow_ragged", "q2_2d_slip", "q1_3d_mixed",
                                  "vortex_q1_32", "q3_2d_slip_ragged"])
def test_mixed_stage_fields(oracle, name):
    """One stage: U^L, dU^H and the stage output within 1e-5 of the scale per
    dof; tau and the bounds (FP64 parts) within FP32 effects on the state-free
    coefficients: tau uses |c_ij| rounded to FP32, so 1e-6."""
    _say("stage " + name)
    ms, U = CASES[name]()
    M, S, op = _setup(oracle, ms, U)
    out, dg = M.stage(op, U, diag=True)
    tau_g = S.stage(0.0)
    assert tau_g == pytest.approx(op.cfl * dg["tau_max"], rel=1e-6)
    # per-component scale; a component that is zero throughout (momentum at
    # rest) is measured against the largest one
    scale = np.abs(U).max(axis=1, keepdims=True)
    scale = np.maximum(scale, 1e-3 * scale.max())
    for field, ref, what in ((gdg.GDG_FIELD_UL, dg["UL"], "U^L"), (gdg.GDG_FIELD_DUH, dg["dUH"], "dU^H")):
        err = np.abs(S.field(field) - ref) / scale
        assert err.max() <= 1e-5, (what, err.max())
    g = S.download()
    assert _admissible(g, ms.dim)
    assert (np.abs(g - out) / scale).max() <= 1e-5


@pytest.mark.parametrize("name,t_final", [("sod_c1", 0.2), ("vortex_q1_48", 0.5), ("quadrant_q2_24", 0.02),
                                          ("blast_q1_10", 0.004)])
def test_mixed_run_l1_vs_oracle(oracle, name, t_final):
    """Whole runs to t_final: L1 error of the mixed variant against the FP64
    oracle at most 1e-5 relative per component; the state stays in A."""
    _say("run " + name)
    if name == "sod_c1":
        wl = W.sod(200)
        ms, U = wl.mesh, wl.U0
    elif name == "vortex_q1_48":
        wl = W.vortex(48)
        ms, U = wl.mesh, wl.U0
    elif name == "quadrant_q2_24":
        ms, U = quadrant_on(2, 2, (24, 24), (1,) * 4)
    else:
        wl = W.blast(10)
        ms, U = wl.mesh, wl.U0
    M, S, op = _setup(oracle, ms, U)
    Uo, t_o, n_o = M.run_to(op, U, t_final)
    st = S.run_to(t_final)
    assert st.t == t_final and t_o == pytest.approx(t_final, rel=1e-14)
    assert abs(st.steps - n_o) <= 1
    Ug = S.download()
    assert _admissible(Ug, ms.dim)
    e = l1_rel(Ug, Uo, M.lumped())
    _say("  %s: %d steps, L1 rel per component %s" % (name, st.steps, np.array2string(e, precision=2)))
    assert e.max() <= L1_TOL, e


def test_mixed_conservation_periodic(oracle):
    """FP32 c_ij keep c_ji = -c_ij exactly but their row sums only to FP32
    rounding, so mass and energy are conserved to about 1e-7 per step."""
    ms, U = quadrant_on(2, 1, (16, 16), (0,) * 4, seed=23)
    M, S, op = _setup(oracle, ms, U)
    mi = M.lumped()
    tot0 = (U * mi).sum(1)
    for _ in range(20):
        S.step()
    out = S.download()
    assert _admissible(out, 2)
    tot1 = (out * mi).sum(1)
    assert np.all(np.abs(tot1 - tot0) <= 1e-6 * (np.abs(U) * mi).sum(1))


def test_mixed_constant_state_exact():
    """Equal states give exactly zero FP32 flux differences too."""
    ms = W.MeshSpec(2, 2, (6, 5), (0, 0), (1, 1), (1, 1, 2, 2))
    V = W.to_conserved(np.full(ms.ndofs, 1.2), np.stack([np.full(ms.ndofs, 0.3), np.zeros(ms.ndofs)]),
                       np.full(ms.ndofs, 0.8))
    S = gdg.Solver.from_spec(ms, _mixed_params(2))
    S.upload(V)
    for _ in range(3):
        S.step()
    assert np.max(np.abs(S.download() - V)) <= 1e-15 * np.abs(V).max()


def test_mixed_graph_run_matches_eager():
    """The captured-graph loop runs the same mixed kernels as eager steps."""
    ms, U = quadrant_on(2, 2, (10, 9), (1, 1, 2, 2), seed=31)
    A = gdg.Solver.from_spec(ms, _mixed_params(2))
    B = gdg.Solver.from_spec(ms, _mixed_params(2))
    A.upload(U)
    B.upload(U)
    for _ in range(11):
        A.step()
    B.run_to(1e9, max_steps=11)
    assert np.array_equal(A.download(), B.download())


@pytest.mark.parametrize("name", ["quadrant_2d_q2", "blast_3d_q1"])
def test_low_order_update_against_unrelaxed_bounds(oracle, name):
    """In FP64, U^L is a convex combination of bar states (eq. ConvexRef), so
    it lies inside the unrelaxed local bounds up to rounding.  The mixed
    variant forms U^L from FP32-accumulated flux sums while the bar states and
    bounds are FP64, so U^L can leave the unrelaxed bounds by the FP32
    rounding of those sums; the limiter then starts from inside the relaxed
    bounds only if that excursion stays below the relaxation margin
    r_i = c_r hhat_i^{p_r} (eq. ViscMinConst2).  Measured after 6 steps: the
    largest excursion as a fraction of the margin (density below or above,
    rescaled entropy below; negative when every U^L is inside), FP64 next to
    mixed."""
    if name == "quadrant_2d_q2":
        ms, U = quadrant_on(2, 2, (24, 20), (1, 1, 1, 1))
    else:
        wl = W.blast(cells=12)
        ms, U = wl.mesh, wl.U0
    M = oracle.Mesh(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc)
    mi = M.lumped()
    p0 = gdg.gdg_default_params(ms.degree)
    r = p0.c_r * (mi / M.volume) ** (p0.p_r / ms.dim)
    frac = {}
    for prec in (gdg.GDG_FP64, gdg.GDG_MIXED):
        p = gdg.gdg_default_params(ms.degree)
        p.precision = prec
        S = gdg.Solver.from_spec(ms, p)
        S.upload(U)
        S.run_to(1e30, max_steps=6)
        S.stage(0.0)
        UL = S.field(gdg.GDG_FIELD_UL)
        rmin_r, rmax_r, smin_r = S.field(gdg.GDG_FIELD_BOUNDS)
        S.close()
        rmin, rmax, smin = rmin_r / (1.0 - r), rmax_r / (1.0 + r), smin_r / (1.0 - r)
        d = ms.dim
        rho = UL[0]
        s_l = (UL[d + 1] - 0.5 * np.sum(UL[1:d + 1] ** 2, 0) / rho) * rho ** (-p0.gamma)
        exc = np.maximum.reduce([(rmin - rho) / (r * rmin), (rho - rmax) / (r * rmax), (smin - s_l) / (r * smin)])
        frac[prec] = float(exc.max())
    # negative: every U^L inside the unrelaxed bounds, by that many margins at the closest node
    _say("%s: largest U^L excursion beyond the unrelaxed bounds, in units of the relaxation margin: "
         "FP64 %.3e, mixed %.3e" % (name, frac[gdg.GDG_FP64], frac[gdg.GDG_MIXED]))
    assert frac[gdg.GDG_FP64] <= 1e-9
    assert frac[gdg.GDG_MIXED] <= 0.1
