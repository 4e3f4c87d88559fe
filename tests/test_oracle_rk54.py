"""Pins of the oracle's SSPRK(5,4) (the fourth-order strong stability
preserving Runge-Kutta method of Spiteri and Ruuth that Sec. 6.2 uses for the
isentropic vortex), against the mathematics of the method rather than its
table:

* the Butcher form recovered from the Shu-Osher coefficients meets the eight
  conditions of order four (to the 15 printed digits), and not those of
  order five;
* every coefficient is non-negative, the alpha rows sum to one, and the SSP
  coefficient min alpha/beta is the method's 1.508;
* fixed-step errors on a smooth 1D flow fall at fourth order (SSP-RK3 beside
  it at third order), against a run at a sixteenth of the step;
* the CFL step is Cr tau_max(U^n) divided by the largest Euler sub-step
  factor beta/alpha (reading R45), and a step of a constant state is exact.
"""
import math

import numpy as np
import pytest

from paper_2402_04514_amd import workloads as W


def _butcher(alpha, beta):
    """Stage i = sum_k alpha_ik u(k) + tau beta_ik L(u(k)) unrolled into
    u(i) = u0 + tau sum_j A_ij L(u(j))."""
    A = np.zeros((6, 5))
    for i in range(1, 6):
        for k in range(i):
            A[i] += alpha[i, k] * A[k]
            A[i, k] += beta[i, k]
    return A[:5], A[5]


def test_order_conditions(oracle):
    a, b = oracle.ssprk54_table()
    A, w = _butcher(a, b)
    c = A.sum(axis=1)
    conds = [(w.sum(), 1.0), (w @ c, 1 / 2), (w @ c ** 2, 1 / 3), (w @ (A @ c), 1 / 6),
             (w @ c ** 3, 1 / 4), (w @ (c * (A @ c)), 1 / 8), (w @ (A @ c ** 2), 1 / 12),
             (w @ (A @ (A @ c)), 1 / 24)]
    for got, want in conds:
        assert abs(got - want) < 5e-15, (got, want)
    # not fifth order: the bushy tree's condition fails by far more than rounding
    assert abs(w @ c ** 4 - 1 / 5) > 1e-4
    # explicit: A strictly lower triangular
    assert np.all(np.triu(A) == 0.0)


def test_ssp_coefficient(oracle):
    a, b = oracle.ssprk54_table()
    assert np.all(a >= 0) and np.all(b >= 0)
    assert np.abs(a[1:].sum(axis=1) - 1.0).max() < 2e-15
    pos = b > 0
    assert np.all(a[pos] > 0)
    assert (a[pos] / b[pos]).min() == pytest.approx(1.508, abs=1e-3)


@pytest.mark.parametrize("integrator,order,steps", [(1, 4.0, (20, 40, 80)), (0, 3.0, (40, 80, 160))])
def test_fixed_step_convergence(oracle, integrator, order, steps):
    """A monotone density profile carried at constant velocity and pressure
    between outflow ends: the low-order scheme keeps u and p and the branch
    of every max in lambda and d_ij, so its right-hand side is smooth in time
    and the integrator's own order shows (a flow where neighbouring sound
    speeds cross makes d_ij kink in time and caps any method near second
    order)."""
    M = oracle.Mesh(1, 2, (24,), (0.0,), (1.0,), (1, 1))
    x = M.coords()[:, 0]
    U0 = W.to_conserved(1.2 - 0.4 * x + 0.05 * np.sin(2 * np.pi * x), np.stack([0.5 + 0 * x]), 1.0 + 0 * x)
    op = oracle.params(degree=2, scheme=oracle.LOW_ORDER, integrator=integrator)
    _, dg = M.stage(op, U0, diag=True)
    T = 24 * dg["tau_max"]

    def run(n):
        U = U0.copy()
        for _ in range(n):
            U, _, nres, st = M.step(op, U, dt_fixed=T / n)
            assert st == 0 and nres == 0
        return U

    ref = run(640)
    errs = [np.abs(run(n) - ref).max() for n in steps]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - order) < 0.35 for r in rates), (errs, rates)


def test_cfl_step_and_constant_state(oracle):
    M = oracle.Mesh(2, 2, (5, 4), (0.0, 0.0), (1.0, 1.0), (0, 0, 2, 2))
    x = M.coords()
    U = W.to_conserved(1.0 + 0.2 * np.sin(2 * np.pi * x[:, 0]), np.stack([0.2 + 0 * x[:, 0], 0 * x[:, 0]]),
                       1.0 + 0.1 * np.cos(2 * np.pi * x[:, 0]))
    op = oracle.params(degree=2, cfl=0.5, integrator=oracle.SSPRK54)
    a, b = oracle.ssprk54_table()
    r = max(b[k + 1, k] / a[k + 1, k] for k in range(5))
    _, dg = M.stage(op, U, diag=True)
    _, dt, nres, st = M.step(op, U)
    assert st == 0
    assert nres == 0 and dt == pytest.approx(0.5 * dg["tau_max"] / r, rel=1e-14)
    Uc = W.to_conserved(np.full(len(x), 1.3), np.stack([np.full(len(x), 0.4), np.full(len(x), -0.2)]),
                        np.full(len(x), 2.0))
    Mp = oracle.Mesh(2, 2, (5, 4), (0.0, 0.0), (1.0, 1.0), (0, 0, 0, 0))
    Un, _, _, st = Mp.step(op, Uc)
    assert st == 0
    assert np.abs(Un - Uc).max() < 1e-14 * np.abs(Uc).max()


def test_step_equals_the_butcher_form_with_stage_times(oracle):
    """The low-order stage is affine in tau (Phi_tau(u) = u + tau L(u, t)),
    so one SSPRK(5,4) step must equal u0 + tau sum_j b_j L(u(j), t0 + c_j tau)
    with u(i) = u0 + tau sum_j A_ij L(u(j), t0 + c_j tau), A and b from the
    pinned table: the vortex's exact, time-dependent Dirichlet data on all
    four sides of a 2D Q1 mesh, so a stage taken at a wrong time fails."""
    G53 = 5.0 / 3.0
    M = oracle.Mesh(2, 1, (8, 8), (-5.0, -5.0), (5.0, 5.0), (3,) * 4, vortex=(5.0, -1.0, -1.0, 1.0, 1.0, G53))
    U0 = W.vortex_exact(M.coords(), 0.0, gamma=G53, periodic=False)
    op = oracle.params(gamma=G53, degree=1, scheme=oracle.LOW_ORDER, integrator=oracle.SSPRK54)
    a, b = oracle.ssprk54_table()
    A, w = _butcher(a, b)
    c = A.sum(axis=1)
    t0, tau = 0.3, 0.05

    def L(u, t):
        M.set_time(t)
        return (M.stage(op, u, tau=tau) - u) / tau

    Ls = []
    for i in range(5):
        u = U0 + tau * sum(A[i, j] * Ls[j] for j in range(i)) if i else U0.copy()
        Ls.append(L(u, t0 + c[i] * tau))
    want = U0 + tau * sum(w[j] * Ls[j] for j in range(5))
    M.set_time(t0)
    got, dt, nres, st = M.step(op, U0, dt_fixed=tau)
    assert st == 0 and nres == 0 and dt == tau
    scale = np.abs(U0).max(axis=1, keepdims=True)
    assert (np.abs(got - want) / scale).max() < 1e-13
    # the data's time matters: the same step from t0 + tau differs
    M.set_time(t0 + tau)
    other, _, _, _ = M.step(op, U0, dt_fixed=tau)
    assert (np.abs(other - want) / scale).max() > 1e-8
