"""GPU request server: continuous batching of independent simulations.

A served request takes the same per-request steps as gdg_run_to on a context
of its own (its own CFL steps, capped last step, restarts), inside persistent
batched launches shared with whatever else is resident.  The results must
therefore be bit-identical alone and in a mix with requests that arrive while
it runs.  Against the single-mesh path they agree to rounding: the batched
kernels are compiled separately, so the compiler may contract other
multiply-adds into FMAs (measured after 20 steps: about 1e-14 of the
component scale in FP64 and 4e-9 in the mixed variant, whose FP32 sums round
at 6e-8; the bounds here are 1e-12 and 1e-7, with the same number of
steps).  On
the FP64 class they also match the oracle at the final time (1e-10, as for
the oracle runs of several steps).
"""
import time

import numpy as np
import pytest

from paper_2402_04514_amd import gdg
from paper_2402_04514_amd import workloads as W

from test_gpu_parity import quadrant_on

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-serving] " + msg, flush=True)


def _requests(dim, degree, n, seed0=40):
    """n small requests of uneven sizes with seeded four-quadrant data."""
    out = []
    sizes = [(6, 5), (13, 11), (9, 16), (21, 7), (8, 8), (17, 19), (5, 12), (11, 10)]
    bcs = [(1, 1, 1, 1), (2, 2, 2, 2), (1, 1, 2, 2), (0, 0, 0, 0)]
    for r in range(n):
        cells = sizes[r % len(sizes)] if dim == 2 else (sizes[r % len(sizes)][0] + 3,)
        bc = bcs[r % len(bcs)] if dim == 2 else (1, 1)
        ms, U = quadrant_on(dim, degree, cells, bc, seed=seed0 + r)
        out.append((ms, U, 0.004 + 0.002 * (r % 3)))
    return out


def _run_server(reqs, precision, max_slots=8, budget=None, arrivals=None, spg=4, solo_dofs=0,
                after_submit=None):
    """Submits reqs (at pump index arrivals[r], default all at once), pumps
    until all finish; returns results, infos and the peak resident count.
    after_submit: called once all requests are submitted."""
    dim, degree = reqs[0][0].dim, reqs[0][0].degree
    if budget is None:
        budget = 256 << 20
    S = gdg.Server(dim, degree, precision, budget_bytes=budget, max_slots=max_slots, steps_per_graph=spg,
                   solo_dofs=solo_dofs)
    arrivals = arrivals or [0] * len(reqs)
    tickets = [None] * len(reqs)
    peak, k = 0, 0
    t0 = time.perf_counter()
    while True:
        for r, (ms, U, tf) in enumerate(reqs):
            if tickets[r] is None and arrivals[r] <= k:
                tickets[r] = S.submit(ms, U, tf)
                if after_submit is not None and all(t is not None for t in tickets):
                    after_submit()
        res, pend = S.pump()
        peak = max(peak, res)
        k += 1
        if all(t is not None for t in tickets) and res == 0 and pend == 0:
            break
        # a pump returns at once while a launch is in flight: bound the time
        assert time.perf_counter() - t0 < 300
    S.sync()
    infos = [S.poll(t) for t in tickets]
    outs = [S.result(t) for t in tickets]
    S.close()
    return outs, infos, peak


def _alone_run_to(ms, U, tf, precision):
    p = gdg.gdg_default_params(ms.degree)
    p.precision = precision
    S = gdg.Solver.from_spec(ms, p)
    S.upload(U)
    st = S.run_to(tf)
    return S.download(), st


@pytest.mark.parametrize("precision", [gdg.GDG_FP64, gdg.GDG_MIXED])
def test_mix_equals_alone_and_single_path(precision):
    """Six requests of uneven sizes, three arriving after the others are on
    the GPU: each result equals, bit for bit, the same request served alone
    and gdg_run_to on a context of its own."""
    _say("mix vs alone, precision %d" % precision)
    reqs = _requests(2, 1, 6)
    outs, infos, peak = _run_server(reqs, precision, max_slots=4, arrivals=[0, 0, 0, 2, 3, 5])
    assert peak <= 4
    for r, (ms, U, tf) in enumerate(reqs):
        assert infos[r].state == gdg.GDG_REQ_DONE and infos[r].t == tf, (r, infos[r].state, infos[r].t)
        alone, _, _ = _run_server([(ms, U, tf)], precision, max_slots=1)
        ref, st = _alone_run_to(ms, U, tf, precision)
        assert np.array_equal(outs[r], alone[0]), ("mix differs from alone", r)
        assert infos[r].steps == st.steps
        scale = np.abs(ref).max(axis=1, keepdims=True)
        scale = np.maximum(scale, 1e-3 * scale.max())
        err = (np.abs(outs[r] - ref) / scale).max()
        tol = 1e-12 if precision == gdg.GDG_FP64 else 1e-7
        assert err <= tol, ("served vs single-mesh path", r, err)


@pytest.mark.parametrize("precision", [gdg.GDG_FP64, gdg.GDG_MIXED])
def test_solo_requests_equal_the_single_mesh_path(precision):
    """With solo_dofs set, the requests of at least that many dofs replay
    their own single-mesh graph inside the server's launches: bit-identical
    to gdg_run_to on a context of their own, while the smaller ones, batched
    beside them, stay bit-identical to being served alone."""
    _say("solo requests, precision %d" % precision)
    reqs = _requests(2, 1, 8, seed0=120)
    solo_dofs = 4 * 13 * 11  # the 13 x 11, 9 x 16, 21 x 7 and 17 x 19 requests
    outs, infos, _ = _run_server(reqs, precision, max_slots=5, arrivals=[0, 0, 1, 1, 2, 4, 4, 6],
                                 solo_dofs=solo_dofs)
    nsolo = 0
    for r, (ms, U, tf) in enumerate(reqs):
        assert infos[r].state == gdg.GDG_REQ_DONE and infos[r].t == tf, (r, infos[r].state, infos[r].t)
        if ms.ndofs >= solo_dofs:
            nsolo += 1
            ref, st = _alone_run_to(ms, U, tf, precision)
            assert np.array_equal(outs[r], ref), ("solo request differs from gdg_run_to", r)
            assert infos[r].steps == st.steps
        else:
            alone, _, _ = _run_server([(ms, U, tf)], precision, max_slots=1)
            assert np.array_equal(outs[r], alone[0]), ("batched request differs from alone", r)
    assert 0 < nsolo < len(reqs)


def test_fp64_served_matches_oracle(oracle):
    """FP64 class, Q2: served results against the oracle's run to the same time."""
    reqs = _requests(2, 2, 3, seed0=70)
    outs, infos, _ = _run_server(reqs, gdg.GDG_FP64, max_slots=3)
    for r, (ms, U, tf) in enumerate(reqs):
        M = oracle.Mesh(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc)
        Uo, t_o, n_o = M.run_to(oracle.params(degree=2), U, tf)
        assert infos[r].steps == n_o
        scale = np.abs(Uo).max(axis=1, keepdims=True)
        scale = np.maximum(scale, 1e-3 * scale.max())
        assert (np.abs(outs[r] - Uo) / scale).max() <= 1e-10, r


def test_admission_by_memory_budget():
    """A pool with room for about two of the requests at a time: the server
    admits while memory is free, in arrival order, and finishes them all with
    the results of unconstrained serving."""
    reqs = _requests(2, 1, 5, seed0=90)
    p = gdg.gdg_default_params(1)
    p.precision = gdg.GDG_MIXED
    sizes = [gdg.gdg_workspace_bytes(gdg.mesh_desc(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc), p)
             for ms, _, _ in reqs]
    over = gdg.gdg_server_overhead_bytes(gdg.server_desc(2, 1, gdg.GDG_MIXED))
    budget = over + sorted(sizes)[-1] + sorted(sizes)[-2] + 4096
    outs, infos, peak = _run_server(reqs, gdg.GDG_MIXED, max_slots=8, budget=budget)
    free_outs, _, _ = _run_server(reqs, gdg.GDG_MIXED, max_slots=8)
    assert peak <= 3
    for r in range(len(reqs)):
        assert infos[r].state == gdg.GDG_REQ_DONE
        assert np.array_equal(outs[r], free_outs[r])
    # arrival order: a request is never admitted before an earlier one
    adm = [i.admit_s for i in infos]
    assert all(adm[r] <= adm[r + 1] for r in range(len(adm) - 1))


def test_one_dimensional_class_and_errors():
    """A 1D server; a request larger than the pool is refused with
    GDG_E_BUDGET, one of another class with GDG_E_INVALID."""
    reqs = _requests(1, 1, 3, seed0=11)
    outs, infos, _ = _run_server(reqs, gdg.GDG_FP64, max_slots=2)
    for r, (ms, U, tf) in enumerate(reqs):
        ref, _ = _alone_run_to(ms, U, tf, gdg.GDG_FP64)
        assert np.abs(outs[r] - ref).max() <= 1e-12 * np.abs(ref).max()
    S = gdg.Server(2, 1, gdg.GDG_FP64, budget_bytes=1 << 20, max_slots=2)
    ms, U = quadrant_on(2, 1, (64, 64), (1,) * 4)
    with pytest.raises(gdg.GdgError) as ei:
        S.submit(ms, U, 0.01)
    assert ei.value.status == gdg.GDG_E_BUDGET
    ms, U = quadrant_on(2, 2, (4, 4), (1,) * 4)
    with pytest.raises(gdg.GdgError) as ei:
        S.submit(ms, U, 0.01)
    assert ei.value.status == gdg.GDG_E_INVALID
    S.close()


def test_served_requests_with_cfl_restarts():
    """Cr = 0.95: served requests go through the server's restart path; each
    result equals its run through gdg_run_to (same steps and restarts)."""
    reqs = _requests(2, 1, 3, seed0=120)
    S = gdg.Server(2, 1, gdg.GDG_FP64, budget_bytes=256 << 20, max_slots=4, steps_per_graph=4)
    tickets = []
    for ms, U, tf in reqs:
        p = gdg.gdg_default_params(1)
        p.cfl = 0.95
        tickets.append(S.submit(ms, U, tf, params=p))
    while True:
        res, pend = S.pump()
        if res == 0 and pend == 0:
            break
    S.sync()
    total_restarts = 0
    for (ms, U, tf), tk in zip(reqs, tickets):
        info = S.poll(tk)
        assert info.state == gdg.GDG_REQ_DONE, info.state
        out = S.result(tk)
        p = gdg.gdg_default_params(1)
        p.cfl = 0.95
        A = gdg.Solver.from_spec(ms, p)
        A.upload(U)
        st = A.run_to(tf)
        assert info.steps == st.steps and info.restarts == st.restarts
        total_restarts += st.restarts
        ref = A.download()
        assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()
    S.close()
    assert total_restarts > 0


def test_admission_overlaps_the_launch_in_flight():
    """A request submitted while a long batched launch runs is admitted (set
    up and uploaded on the admission stream) before that launch is processed,
    joins the next launch, and its result is still the same as served alone."""
    big_ms, big_U = quadrant_on(2, 1, (256, 256), (2,) * 4, seed=3)
    small_ms, small_U = quadrant_on(2, 1, (24, 20), (2,) * 4, seed=4)
    S = gdg.Server(2, 1, gdg.GDG_FP64, budget_bytes=1 << 30, max_slots=4, steps_per_graph=64)
    tb = S.submit(big_ms, big_U, 0.002)
    res, _ = S.pump()                       # admits the big request and launches 64 of its steps
    assert res == 1
    ts = S.submit(small_ms, small_U, 0.002)
    res, pend = S.pump()                    # the launch is still running: admission only
    info_big, info_small = S.poll(tb), S.poll(ts)
    _say("while in flight: resident %d, big steps %d, small state %d" % (res, info_big.steps, info_small.state))
    assert res == 2 and pend == 0
    assert info_small.state == gdg.GDG_REQ_RUNNING and info_small.admit_s > 0
    assert info_big.steps == 0              # the launch in flight has not been processed
    while True:
        res, pend = S.pump()
        if res == 0 and pend == 0:
            break
    S.sync()
    out_big, out_small = S.result(tb), S.result(ts)
    S.close()
    alone_big, _, _ = _run_server([(big_ms, big_U, 0.002)], gdg.GDG_FP64, max_slots=1)
    alone_small, _, _ = _run_server([(small_ms, small_U, 0.002)], gdg.GDG_FP64, max_slots=1)
    assert np.array_equal(out_big, alone_big[0]) and np.array_equal(out_small, alone_small[0])
