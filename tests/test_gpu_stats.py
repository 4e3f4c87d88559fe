"""GPU statistics of gdg_get_stats (gdg_stats): the measures of the current
state reduced on the device, against numpy on the downloaded state, and the
counters of the limiter and the quiet-cell path.

* min rho is a minimum of stored values: exact.
* min eps = min (E - |m|^2 / (2 rho)): the device may contract the squares
  into fused multiply-adds, so it is compared to 4 ulps of the value.
* sum_i m_i U_i: the device sums in a fixed tree order, numpy pairwise; both
  are within a few ulps per addition of the exact sum, compared at 1e-13 of the
  sum of magnitudes.  The totals are Lemma TotBalLemma's conserved quantities:
  on a periodic mesh they stay at their initial values to rounding.
* bound_violations: Lemma ConsInvariants puts every limiter output in its
  relaxed bounds, so the count is zero on every case, shocks included.
* limited_pairs: pairs of limiter pass 1 with l_ij < 1, against the oracle's
  l_ij of the same stage (pairs with a zero flux excluded on both sides: the
  device records l = 1 for them without a search).
* quiet_rows: a uniform state makes every row quiet in every stage.
"""
import numpy as np
import pytest

from paper_2402_04514_amd import gdg
from paper_2402_04514_amd import workloads as W

from test_gpu_parity import CASES, blob_on, quadrant_on

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-stats] " + msg, flush=True)


def _numpy_stats(U, dim, mi):
    eps = U[dim + 1] - 0.5 * np.sum(U[1:dim + 1] ** 2, 0) / U[0]
    return U[0].min(), eps.min(), (U * mi).sum(1), (np.abs(U) * mi).sum(1)


@pytest.mark.parametrize("name", ["q1_2d_periodic", "q2_2d_slip", "q1_3d_mixed", "q2_3d_tiled", "sod_q1_40"])
def test_state_measures_match_numpy(oracle, name):
    _say("state measures " + name)
    ms, U = CASES[name]()
    M = oracle.Mesh(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc)
    mi = M.lumped()
    S = gdg.Solver.from_spec(ms)
    S.upload(U)
    st0 = S.stats()
    r0, e0, tot0, mag0 = _numpy_stats(U, ms.dim, mi)
    assert st0.min_rho == r0
    assert abs(st0.min_eps - e0) <= 4 * np.spacing(abs(e0))
    assert np.all(np.abs(np.array(st0.total[:ms.dim + 2]) - tot0) <= 1e-13 * mag0)
    st = S.run_to(1e30, max_steps=6)
    V = S.download()
    r1, e1, tot1, mag1 = _numpy_stats(V, ms.dim, mi)
    assert st.min_rho == r1 and st.min_rho > 0
    assert abs(st.min_eps - e1) <= 4 * np.spacing(abs(e1)) and st.min_eps > 0
    assert np.all(np.abs(np.array(st.total[:ms.dim + 2]) - tot1) <= 1e-13 * mag1)
    assert st.bound_violations == 0
    if all(b == gdg.GDG_BC_PERIODIC for b in ms.bc):
        # Lemma TotBalLemma: every component is conserved on a periodic mesh
        assert np.all(np.abs(np.array(st.total[:ms.dim + 2]) - tot0) <= 1e-13 * mag0)
    # the same state gives the same bits
    again = S.stats()
    assert again.min_rho == st.min_rho and again.min_eps == st.min_eps
    assert list(again.total) == list(st.total)


def test_slip_box_keeps_mass_and_energy(oracle):
    """In a box of slip walls the boundary flux of mass and energy vanishes
    (u.n = 0 for the reflected state's average), so sum m_i rho_i and
    sum m_i E_i stay at their initial values."""
    ms, U = quadrant_on(2, 1, (14, 12), (2,) * 4, seed=11)
    S = gdg.Solver.from_spec(ms)
    S.upload(U)
    st0 = S.stats()
    st = S.run_to(1e30, max_steps=20)
    for c in (0, ms.dim + 1):
        assert abs(st.total[c] - st0.total[c]) <= 1e-13 * abs(st0.total[c])
    assert st.bound_violations == 0 and st.min_rho > 0 and st.min_eps > 0


@pytest.mark.parametrize("name", ["q1_2d_outflow_ragged", "q2_2d_outflow", "q1_3d_slip"])
def test_limited_pairs_match_oracle(oracle, name):
    _say("limited pairs " + name)
    ms, U = CASES[name]()
    M = oracle.Mesh(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc)
    S = gdg.Solver.from_spec(ms)
    S.upload(U)
    _, dg = M.stage(oracle.params(degree=ms.degree), U, diag=True)
    rp, col = M.csr()[:2]
    nonzero = np.any(dg["Aij"] != 0.0, axis=1)
    cut = int(np.sum((dg["lij"] < 1.0) & nonzero))
    S.stage(0.0)
    st = S.stats()
    assert cut > 0
    # l_ij = 1 exactly on both sides where the bounds hold at the full flux;
    # a pair at the edge may round the other way on one side
    assert abs(st.limited_pairs - cut) <= max(2, 0.002 * cut), (st.limited_pairs, cut)
    assert st.bound_violations == 0


def test_quiet_rows_counted():
    ms = W.MeshSpec(2, 2, (6, 5), (0, 0), (1, 1), (1, 1, 2, 2))
    U = W.to_conserved(np.full(ms.ndofs, 1.2), np.stack([np.full(ms.ndofs, 0.3), np.zeros(ms.ndofs)]),
                       np.full(ms.ndofs, 0.8))
    S = gdg.Solver.from_spec(ms)
    S.upload(U)
    S.run_to(1e30, max_steps=2)
    st = S.stats()
    # outflow rows see U_i itself as boundary state; the slip faces reflect
    # a zero normal momentum (u_y = 0): every row of every stage is quiet
    assert st.quiet_rows == 2 * 3 * ms.ndofs
    assert st.limited_pairs == 0 and st.bound_violations == 0
    ms, U = blob_on(2, 1, (20, 18), (1, 1, 2, 2))
    S = gdg.Solver.from_spec(ms)
    S.upload(U)
    S.stage(0.0)
    st = S.stats()
    assert 0 < st.quiet_rows < ms.ndofs
