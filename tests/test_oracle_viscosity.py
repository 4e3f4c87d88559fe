"""Pins of the oracle's high-order viscosity (Sec. 5.1-5.2) against the
paper's own definitions and constants, read back from what the limiter sees.

Across a face the consistent mass matrix couples nothing (m_ij = 0 between
cells), so eq. HighLowOrderIdentity reduces to A_ij = tau (d^H_ij - d^L_ij)
(U_j - U_i) there: the viscosity that the oracle used for a face pair can be
read off its antidiffusive flux, and it must be the one of
eq. HighOrderViscosity with eq. ViscMin and the printed constants,
  d^H = max(c_k hhat_ij^{p_k} d^L [x_i = x_j only], d^L min(c_ev max(|N_i|, |N_j|), 1)),
  c_k = 1, p_k = 0 (odd k) or 1/2 (even k), c_ev = 1, 0.5, 0.25 (k = 1, 2, 3),
  hhat_ij = ((m_i + m_j) / (2 |Omega|))^(1/d).
The boundary part A_i^d of a row with one boundary face checks reading R7,
d^{d,H} = max(c_k hhat_i^{p_k} d^{d,L}, d^{d,L} min(c_ev |N_i|, 1)), with
d^{d,L} = |c_i^d| lambda^+ of the wave-speed bound (pinned on its own in
test_oracle_physics).  The only case where A_i^d is not zero is even degree
at a boundary whose data differ from U_i: here slip walls.

The Q2 convergence pin checks the even-degree scheme as a whole: third order
on the smooth vortex (context: the paper's Q2 rates of 2.9-3.1 in Table
ErrorIsentropicConvex, at gamma = 5/3 with exact boundary data and another
integrator)."""
import math

import numpy as np
import pytest

from paper_2402_04514_amd import workloads as W

from test_oracle_scheme import _l1, make, quadrant_on

G = 1.4
PAPER_CEV = {1: 1.0, 2: 0.5, 3: 0.25}     # Sec. 5.2
PAPER_PK = {1: 0.0, 2: 0.5, 3: 0.0}       # eq. ViscMin: 1/2 for even degree, 0 for odd
PAPER_CK = 1.0                            # eq. ViscMin
KIND_CELL, KIND_FACE_COLLOC, KIND_FACE = 0, 1, 2


def smooth_on(dim, k, cells, bc, seed=7):
    """Smooth data with a small jump at every face: each cell scales density
    and pressure by its own factor within 1 +- 1%, so collocated face nodes
    hold different states (as a DG solution does) while the entropy residual
    stays small."""
    ms = W.MeshSpec(dim, k, (cells,) * dim, (0.0,) * dim, (1.0,) * dim, bc)
    x, _ = W.node_coords(ms)
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, size=(4, dim))
    f = lambda r: np.sum(np.sin(2 * np.pi * x + ph[r]), axis=1) / dim
    jump = np.repeat(1.0 + 0.01 * rng.uniform(-1, 1, size=ms.ncells), ms.nloc)
    vel = np.stack([0.4 * f(1 + (e % 2)) for e in range(dim)])
    return ms, W.to_conserved((1.0 + 0.4 * f(0)) * jump, vel, (1.0 + 0.5 * f(3)) * jump)


CASES = {
    "q1_smooth": lambda: smooth_on(2, 1, 6, (0,) * 4),
    "q2_smooth": lambda: smooth_on(2, 2, 6, (0,) * 4),
    "q2_quadrant": lambda: quadrant_on(2, 2, 6, (1,) * 4),
    "q2_smooth_3d": lambda: smooth_on(3, 2, 3, (0,) * 6),
    "q3_smooth": lambda: smooth_on(2, 3, 4, (0,) * 4),
    "q3_quadrant": lambda: quadrant_on(2, 3, 4, (1,) * 4),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_face_pair_viscosity_is_the_papers(oracle, name):
    ms, U = CASES[name]()
    k, d = ms.degree, ms.dim
    M = make(oracle, ms)
    prm = oracle.params(degree=k)
    _, dg = M.stage(prm, U, diag=True)
    tau = prm.cfl * dg["tau_max"]
    rp, col, c, mij, kind = M.csr()
    mi = M.lumped()
    vol = M.volume
    N = dg["N"]
    cev = PAPER_CEV[k]
    checked, by_min, by_ev = 0, 0, 0
    worst = 0.0
    for i in range(M.ndofs):
        for q in range(rp[i], rp[i + 1]):
            j = int(col[q])
            if kind[q] == KIND_CELL:
                continue
            dU = U[:, j] - U[:, i]
            cq = int(np.argmax(np.abs(dU)))
            if abs(dU[cq]) < 1e-3 * np.abs(U[cq]).max():
                continue
            dL = dg["dij"][q]
            dH = dL + dg["Aij"][q, cq] / (tau * dU[cq])
            dev = dL * min(cev * max(abs(N[i]), abs(N[j])), 1.0)
            dmin = 0.0
            if kind[q] == KIND_FACE_COLLOC:
                hh = (0.5 * (mi[i] + mi[j]) / vol) ** (1.0 / d)
                dmin = PAPER_CK * hh ** PAPER_PK[k] * dL
            expect = max(dmin, dev)
            worst = max(worst, abs(dH - expect) / dL)
            # the other components carry the same factor
            for cc in range(d + 2):
                assert abs(dg["Aij"][q, cc] - tau * (expect - dL) * dU[cc]) <= 1e-9 * tau * dL * np.abs(dU).max()
            checked += 1
            by_min += dmin > dev
            by_ev += dev > dmin
    assert checked > 20
    assert worst <= 1e-9, worst
    if k % 2 == 0 and "smooth" in name:
        assert by_min > 0       # the minimal viscosity of eq. ViscMin is exercised
    assert by_ev > 0 or k == 2 and "smooth" in name


@pytest.mark.parametrize("seed", [240204514, 5])
def test_boundary_viscosity_even_degree(oracle, seed):
    """Q2 in a slip box: A_i^d of rows with one boundary face against
    tau (d^{d,H} - d^{d,L}) (U^d - U_i) with reading R7's d^{d,H}."""
    ms, U = quadrant_on(2, 2, 6, (2,) * 4, seed=seed)
    M = make(oracle, ms)
    prm = oracle.params(degree=2)
    _, dg = M.stage(prm, U, diag=True)
    tau = prm.cfl * dg["tau_max"]
    bptr, bface, bc_c = M.boundary()
    mi = M.lumped()
    vol = M.volume
    N = dg["N"]
    n_checked, n_nonzero = 0, 0
    for i in range(M.ndofs):
        if bptr[i + 1] - bptr[i] != 1:
            continue
        b = bptr[i]
        cb = bc_c[b]
        nn = np.linalg.norm(cb)
        n = cb / nn
        Ui = U[:, i]
        Ug = Ui.copy()
        Ug[1:3] = Ui[1:3] - 2.0 * np.dot(Ui[1:3], n) * n     # eq. slip_boundary
        dL = nn * oracle.lambda_max(G, Ui, Ug, n)
        hh = (mi[i] / vol) ** 0.5
        dH = max(PAPER_CK * hh ** PAPER_PK[2] * dL, dL * min(PAPER_CEV[2] * abs(N[i]), 1.0))
        expect = tau * (dH - dL) * (Ug - Ui)
        got = dg["Abd"][i]
        assert np.all(np.abs(got - expect) <= 1e-11 * tau * dL * (np.abs(Ui).max() + 1e-300)), (i, got, expect)
        n_checked += 1
        n_nonzero += np.any(got != 0.0)
    assert n_checked > 10 and n_nonzero > 5


def _vortex_q2(n):
    ms = W.MeshSpec(2, 2, (n, n), (-5.0, -5.0), (5.0, 5.0), (0,) * 4)
    x, _ = W.node_coords(ms)
    return ms, W.vortex_exact(x, 0.0)


def test_vortex_convergence_q2(oracle):
    """Convex-limited Q2 on the smooth vortex: third order between 16^2 and
    32^2 cells at t = 0.5 (measured 2.6 then 3.1: the coarsest level is
    pre-asymptotic, as Remark rem:asymptotic_regime warns)."""
    tf = 0.5
    errs = []
    for n in (8, 16, 32):
        ms, U0 = _vortex_q2(n)
        M = make(oracle, ms)
        U, t, _ = M.run_to(oracle.params(degree=2), U0, tf)
        errs.append(_l1(M, U, W.vortex_exact(M.coords(), tf)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert rates[0] > 2.3, (errs, rates)
    assert 2.85 < rates[1] < 3.6, (errs, rates)


def _vortex_k(n, k):
    ms = W.MeshSpec(2, k, (n, n), (-5.0, -5.0), (5.0, 5.0), (0,) * 4)
    x, _ = W.node_coords(ms)
    return ms, W.vortex_exact(x, 0.0)


def test_vortex_convergence_q3(oracle):
    """Q3 (c_ev = 0.25, p_k = 0) on the smooth vortex to t = 0.5 at 8^2 and
    16^2 cells: the unlimited high-order scheme converges at fourth order
    (measured 3.6 on this pre-asymptotic pair; context: the paper's Q3 rates of
    3.7-3.9 with SSPRK-54), the convex-limited one at third order or better
    (measured 3.1: at Cr = 0.5 with SSP-RK3 the limiter still cuts some fluxes
    of the smooth solution on coarse meshes; at Cr = 0.125 its error equals
    the unlimited one), and well below the first-order scheme's error."""
    tf = 0.5
    err = {}
    for scheme in (oracle.HIGH_ORDER, oracle.LIMITED):
        for n in (8, 16):
            ms, U0 = _vortex_k(n, 3)
            M = make(oracle, ms)
            U, _, _ = M.run_to(oracle.params(degree=3, scheme=scheme), U0, tf)
            err[scheme, n] = _l1(M, U, W.vortex_exact(M.coords(), tf))
    r_high = math.log2(err[oracle.HIGH_ORDER, 8] / err[oracle.HIGH_ORDER, 16])
    r_lim = math.log2(err[oracle.LIMITED, 8] / err[oracle.LIMITED, 16])
    assert 3.3 < r_high < 4.6, err
    assert 2.8 < r_lim < 4.6, err
    assert err[oracle.LIMITED, 16] < 2.0 * err[oracle.HIGH_ORDER, 16], err
