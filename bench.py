#!/usr/bin/env python3
"""Throughput of the graph-based DG hot path on one MI355X.

A step is one SSP-RK3 step of the convex-limited scheme (three forward-Euler
stages, each: sweep 1, sweep 2 with the cell solve, two limiter passes) over
the whole mesh, through the C-ABI of libgdg (gdg_run_to: the device-driven
loop of captured step graphs).  The metric is dof-stage updates per second:
dofs x 3 stages x steps / seconds, with the state resident in HBM before the
timed region starts.

The default workload is the largest single-GPU configuration: the 3D Q1 blast
on 128^3 cells (16.8M dofs), FP64, its full 200 steps from the initial state
(warmup steps run first on the same context, which is then reset to the
initial state, so the timed steps are exactly the configured run).

Prints one JSON line.  Besides the contract fields it carries
  roofline      the stage's algorithmic bytes per dof-stage (the whole-stage
                byte model: stencil once, state in and out, each grid-wide
                intermediate written and read once) times the dof-stages of
                the timed region, over the region's duration from HIP events
                on the library's stream, against the 8 TB/s HBM peak;
                `traffic` = FETCH_SIZE + WRITE_SIZE bytes per stage from the
                committed counter profile of the same kernel source; the
                dominant kernel's own figures under `dominant_kernel`;
  windows       throughput and the fraction of quiet rows per quarter of the
                run (the quiet-cell path skips the limiter's pairs where the
                whole stencil holds one state, which depends on the data);
  checks        min rho, min eps, conserved totals and bound violations of
                the final state (gdg_get_stats);
  mixed         the mixed-precision variant on the same workload and steps,
                and its L1 difference from FP64 at equal time levels, beside
                the growth of a 1e-13 input perturbation under FP64 alone;
  serving       p50 / p99 time to solution and aggregate throughput of the
                batched request server on a Poisson trace of 2D problems,
                against FIFO one-at-a-time FP64;
  cpu_baseline  the CPU oracle timed on this host's cores on a bounded
                sample, all cores and one core.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "dof-stage updates/s FP64 vs mixed at stated L1 error; p50/p99 solve latency"
CELLS_OVERRIDE = 0  # --cells: the same problem on another mesh (not a benchmark line)
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (factory kwargs, description, default steps, warmup)
    "blast": ({}, "3D Euler DG Q1, 128^3 cells on [0,1]^3 (16,777,216 dofs), blast p=100 in r<0.1, "
                  "slip walls, FP64, convex-limited, SSP-RK3 at Cr=0.5, 200 steps from t=0", 200, 3),
    "quadrant": ({}, "2D Euler DG Q2, 1024x1024 cells on [0,1]^2 (9,437,184 dofs), seeded "
                     "four-quadrant Riemann data, outflow, FP64, convex-limited, SSP-RK3, 500 steps from t=0",
                 500, 3),
    "vortex": ({}, "2D Euler DG Q1, 256x256 periodic cells on [-5,5]^2 (262,144 dofs), "
                   "isentropic vortex beta=5, gamma=1.4, FP64, convex-limited, SSP-RK3 at Cr=0.5", 400, 20),
    "sod": ({}, "1D Euler DG Q1, 200 cells on [0,1] (400 dofs), Sod shock tube, outflow, FP64", 700, 20),
    "inflow": ({"cells": 1024, "dim": 2, "axis": 0, "degree": 2, "cross": 1024},
               "2D Euler DG Q2, 1024x1024 cells on [0,1]^2 (9,437,184 dofs), supersonic inflow (Dirichlet data "
               "rho,u,p = 1,2.5,1) into a supersonic stream (0.5,2.5,0.6), supersonic in/outflow faces in x, "
               "periodic in y, FP64, convex-limited, SSP-RK3", 100, 3),
    "cylinder": ({"ntheta": 2048, "nr": 1152},
                 "2D Euler DG Q1, Mach 3 flow past a cylinder of radius 0.25 at (0.6, 0) in the channel "
                 "[0,4]x[-1,1], O-grid of 2048x1152 general (bilinearly mapped) cells (9,437,184 dofs), Dirichlet "
                 "inflow, slip channel walls and cylinder, outflow (boundary parts), FP64, convex-limited, "
                 "SSP-RK3, 100 steps from the uniform free stream at t=0", 100, 3),
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("gdg_kernels.hip", "gdg_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2402_04514_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def stencil_width(dim: int, degree: int) -> int:
    """Mean stencil width s of interior rows, diagonal included: the
    (k+1)^d in-cell dofs, plus (k+1)^(d-1) face partners for each of the faces
    a node lies on (2d/(k+1) faces on average)."""
    nb = degree + 1
    return nb ** dim + 2.0 * dim * nb ** (dim - 2.0)


def b_alg(dim: int, degree: int, mixed: bool = False) -> float:
    """Algorithmic bytes per dof-stage of the whole stage: the stencil read
    once (int32 column + c_ij in 8 or 4 bytes per axis per entry), m_i and the
    cell mass block, the state read and written plus U^n re-read by the SSP
    combination (2/3 on average), and each grid-wide intermediate written and
    read once (N_i with the ring-1 partials, U^L, the bounds, dU^H, U^(1));
    d_ij, A_ij and l_ij recomputed, not stored."""
    s = stencil_width(dim, degree)
    m = dim + 2
    wc = 4 if mixed else 8
    return s * (4 + wc * dim) + 8 * (1 + (degree + 1) ** dim) + 8 * m * (2 + 2.0 / 3.0) + \
        2 * (32 + 8 * m + 24 + 8 * m + 8 * m)


def algorithmic_bytes(kernel: str, dim: int, slots: float, ghosts: float = 0.0) -> float:
    """Per-kernel byte model of this implementation (per row, each array it
    touches counted once: stencil entries, per-slot d^L and l, per-dof fields;
    a neighbour's values once per sweep).  It counts the stored d^L, l and
    flux sums, which the whole-stage model above recomputes instead."""
    M = dim + 2
    st = slots * (4 + 1 + 8 * dim)    # column, meta, c_ij
    idx = slots * (4 + 1)             # column, meta
    if kernel == "prim":
        return 8 * M + 8 * (dim + 5)
    if kernel == "sweep1":   # U, node cache in; d^L, N, ring-1 partials, flux sums out
        return st + 8 * (M + dim + 5) + 8 * slots + 8 + 24 + 8 * M
    if kernel == "sweep2":   # U, u, p, N, q, d^L, flux sums in; U^L, bounds, dU^H out
        return idx + 8 * dim * ghosts + 8 * slots + 8 * (M + dim + 1) + 8 + 24 + 8 * M + 8 * M + 24 + 8 * M
    lim = idx + 8 * slots + 8 * M * 3 + 24 + 8 + 4 + 8 * M + 8 * slots
    if kernel == "limit1":
        return lim + 8 * M
    if kernel == "limit2":
        return lim + 8 * M + 8 * M
    raise KeyError(kernel)


def stencil_slots(ms) -> tuple[float, float]:
    """Average stored slots per row (graph entries + boundary parts) and
    average boundary parts per row."""
    d, k = ms.dim, ms.degree
    nb = k + 1
    tot = 0.0
    ghost = 0.0
    for e in range(d):
        n = ms.cells[e]
        periodic = ms.bc[2 * e] == 0
        face_nodes_frac = 2.0 / nb
        interior = 1.0 if periodic else (n - 1) / n
        tot += face_nodes_frac * (interior * nb ** (d - 1) + (1 - interior) * 1)
        ghost += face_nodes_frac * (1 - interior)
    return nb ** d + tot, ghost


def _params(gdg, degree, precision):
    p = gdg.gdg_default_params(degree)
    p.precision = precision
    return p


def _workload(name):
    from paper_2402_04514_amd import workloads as W
    kw, desc, _, _ = WORKLOADS[name]
    if CELLS_OVERRIDE:
        kw = dict(kw, cells=CELLS_OVERRIDE)
        desc = desc + " [cells per side overridden: %d]" % CELLS_OVERRIDE
    return W.CONFIGS[name](**kw), desc


def run_gpu(name, steps, warmup, precision=0, windows=4, profile_steps=10):
    """Warmup steps (graph capture), reset to the initial state, then the
    timed steps from t = 0 in `windows` chunks (one host sync between chunks;
    the graph loop syncs once per 8 steps anyway), bracketed by HIP events on
    the library's stream; then a short host-driven region with per-launch HIP
    events for the per-kernel figures."""
    import numpy as np
    import torch

    from paper_2402_04514_amd import gdg

    wl, desc = _workload(name)
    S = gdg.Solver.from_spec(wl.mesh, _params(gdg, wl.mesh.degree, precision), device="cuda:0")
    S.upload(wl.U0)
    if warmup:
        S.run_to(1e30, max_steps=warmup)   # also captures the step graph
    S.upload(wl.U0)                        # the timed run starts from the initial state
    st0 = S.stats()
    torch.cuda.synchronize()
    stream = S.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    bounds = [round(steps * w / windows) for w in range(windows + 1)]
    win = []
    prev_q, prev_t = 0, 0.0
    t0 = time.perf_counter()
    e0.record(stream)
    for w in range(windows):
        n = bounds[w + 1] - bounds[w]
        if n <= 0:
            continue
        a = time.perf_counter()
        st = S.run_to(1e30, max_steps=n)
        b = time.perf_counter()
        win.append({"steps": [bounds[w] + 1, bounds[w + 1]], "dof_stage_per_s": S.ndofs * 3 * n / (b - a),
                    "quiet_row_fraction": (st.quiet_rows - prev_q) / (S.ndofs * 3.0 * n),
                    "t": [prev_t, st.t]})
        prev_q, prev_t = st.quiet_rows, st.t
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    secs_ev = e0.elapsed_time(e1) / 1e3
    final = S.stats()
    out = S.download()
    dim = wl.mesh.dim
    eps = out[dim + 1] - 0.5 * np.sum(out[1:dim + 1] ** 2, 0) / out[0]
    admissible = bool(np.all(out[0] > 0) and np.all(eps > 0))
    checks = {"admissible": admissible, "min_rho": final.min_rho, "min_eps": final.min_eps,
              "bound_violations": final.bound_violations, "limited_pairs": final.limited_pairs,
              "quiet_row_fraction": final.quiet_rows / (S.ndofs * 3.0 * steps),
              "totals_initial": list(st0.total)[:dim + 2], "totals_final": list(final.total)[:dim + 2],
              "restarts": final.restarts, "simulated_time": final.t}
    # per-kernel figures: host-driven steps with HIP events around every launch
    gdg.gdg_profile(S.ctx, True)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    S.run_to(1e30, max_steps=profile_steps)
    torch.cuda.synchronize()
    p1 = time.perf_counter()
    prof = gdg.gdg_profile_read(S.ctx)
    gdg.gdg_profile(S.ctx, False)
    S.close()
    return {"wl": wl, "desc": desc, "ndofs": S.ndofs, "secs": secs_ev, "secs_host": t1 - t0, "windows": win,
            "checks": checks, "prof": prof, "prof_region": (profile_steps, (p1 - p0) / profile_steps * 1e3)}


def mixed_vs_fp64(name, steps):
    """Mixed-precision against FP64 on the GPU at equal time levels: the FP64
    path takes `steps` CFL steps (host-driven, recording tau), the mixed path
    replays the same taus.  Reported per component and in the paper's
    consolidated norm (relative density + relative momentum, Euclidean per
    node, + relative energy error, all L1 with the lumped masses, which are
    equal per local node on a uniform mesh).  Beside it, the same measure for
    the FP64 path fed the input with a 1e-13 relative density perturbation:
    how far rounding-level differences grow on this workload by themselves."""
    import numpy as np

    from paper_2402_04514_amd import gdg

    wl, _ = _workload(name)
    dim = wl.mesh.dim

    def solver(prec, U):
        S = gdg.Solver.from_spec(wl.mesh, _params(gdg, wl.mesh.degree, prec), device="cuda:0")
        S.upload(U)
        return S

    def norms(a, b):
        num = np.abs(a - b).sum(1)
        den = np.abs(b).sum(1)
        comp = num / np.maximum(den, 1e-300)
        mom = np.sqrt(((a[1:dim + 1] - b[1:dim + 1]) ** 2).sum(0)).sum() / max(
            np.sqrt((b[1:dim + 1] ** 2).sum(0)).sum(), 1e-300)
        return [float(x) for x in comp], float(comp[0] + mom + comp[dim + 1])

    S = solver(gdg.GDG_FP64, wl.U0)
    dts = []
    for k in range(steps):
        dts.append(S.step())
        if k % 50 == 49:
            log("mixed vs fp64: fp64 step %d" % (k + 1))
    ref = S.download()
    S.close()
    M = solver(gdg.GDG_MIXED, wl.U0)
    for k, dt in enumerate(dts):
        M.step(dt_fixed=dt)
        if k % 50 == 49:
            log("mixed vs fp64: mixed step %d" % (k + 1))
    mix = M.download()
    mst = M.stats()
    M.close()
    rng = np.random.default_rng(2402)
    Up = wl.U0.copy()
    Up[0] *= 1.0 + 1e-13 * rng.standard_normal(Up.shape[1])
    P = solver(gdg.GDG_FP64, Up)
    for k, dt in enumerate(dts):
        P.step(dt_fixed=dt)
        if k % 50 == 49:
            log("mixed vs fp64: perturbed fp64 step %d" % (k + 1))
    per = P.download()
    P.close()
    comp, cons = norms(mix, ref)
    pcomp, pcons = norms(per, ref)
    return {"steps": steps, "t": float(sum(dts)), "l1_rel_per_component": comp, "l1_consolidated": cons,
            "mixed_bound_violations": mst.bound_violations, "mixed_min_rho": mst.min_rho,
            "mixed_min_eps": mst.min_eps,
            "fp64_perturbed_1e-13": {"l1_rel_per_component": pcomp, "l1_consolidated": pcons}}


def serving(count, n_max, t_final, budget_gib, max_slots, spg, solo_dofs=0):
    """The serving workload on a trace of `count` requests (2D Q1 four-quadrant
    Riemann problems of n x n cells, n log-uniform in [32, n_max], slip walls,
    run to t_final; Poisson arrivals at 20 per second), served in real time by
    the batched server (mixed precision), and the same trace served FIFO one at
    a time on the FP64 single-mesh path (each request's service time measured
    back to back; queueing replayed on the arrival clock)."""
    import numpy as np
    import torch

    from paper_2402_04514_amd import gdg
    from paper_2402_04514_amd import workloads as W

    trace = W.serving_trace(count, n_max=n_max)
    reqs = [(a, W.quadrant(cells=n, degree=1, seed_base=sb, bc=W.BC_SLIP)) for a, n, sb in trace]
    # -- batched, continuous admission, real time
    S = gdg.Server(2, 1, gdg.GDG_MIXED, budget_bytes=int(budget_gib * (1 << 30)), max_slots=max_slots,
                   steps_per_graph=spg, solo_dofs=solo_dofs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = [None] * count
    done = [None] * count
    nsub = 0
    last_note = 0.0
    while True:
        now = time.perf_counter() - t0
        if now - last_note > 5.0:
            last_note = now
            log("serving %.1f s: %d submitted, %d finished" % (now, nsub, sum(d is not None for d in done)))
        while nsub < count and reqs[nsub][0] <= now:
            wl = reqs[nsub][1]
            tickets[nsub] = S.submit(wl.mesh, wl.U0, t_final)
            nsub += 1
        res, pend = S.pump()
        for r in range(nsub):
            if done[r] is None:
                info = S.poll(tickets[r])
                if info.state >= gdg.GDG_REQ_DONE:
                    done[r] = info
        if nsub == count and all(d is not None for d in done):
            break
        if res == 0 and pend == 0 and nsub < count:
            time.sleep(max(0.0, reqs[nsub][0] - (time.perf_counter() - t0)))
    makespan = time.perf_counter() - t0
    failed = sum(1 for d in done if d.state != gdg.GDG_REQ_DONE)
    # server clock starts at creation, just before t0: its done times are
    # on the same clock as the arrivals up to that gap
    tts = np.array([d.done_s - a for d, (a, _) in zip(done, reqs)])
    steps = np.array([d.steps for d in done])
    work = float(sum(d.ndofs * 3 * d.steps for d in done))
    served = {"requests": count, "failed": failed, "makespan_s": makespan,
              "p50_s": float(np.percentile(tts, 50)), "p99_s": float(np.percentile(tts, 99)),
              "dof_stage_per_s": work / makespan, "steps_total": int(steps.sum()),
              "precision": "mixed", "max_slots": max_slots, "steps_per_graph": spg, "solo_dofs": solo_dofs,
              "solo_requests": sum(1 for _, wl in reqs if solo_dofs > 0 and wl.mesh.ndofs >= solo_dofs),
              "budget_gib": budget_gib}
    S.close()
    # -- one at a time, FP64, FIFO
    service, work1 = [], 0.0
    for k, (a, wl) in enumerate(reqs):
        if k % 8 == 0:
            log("serving one at a time: request %d of %d" % (k, count))
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        Sv = gdg.Solver.from_spec(wl.mesh, device="cuda:0")
        Sv.upload(wl.U0)
        st = Sv.run_to(t_final)
        work1 += wl.mesh.ndofs * 3 * st.steps
        Sv.download()
        Sv.close()
        torch.cuda.synchronize()
        service.append(time.perf_counter() - s0)
    end, tts1 = 0.0, []
    for (a, _), sv in zip(reqs, service):
        start = max(a, end)
        end = start + sv
        tts1.append(end - a)
    tts1 = np.array(tts1)
    single = {"p50_s": float(np.percentile(tts1, 50)), "p99_s": float(np.percentile(tts1, 99)),
              "makespan_s": end, "dof_stage_per_s": work1 / end, "precision": "fp64",
              "busy_s": float(sum(service))}
    sizes = [n for _, n, _ in trace]
    return {"trace": "%d requests, 2D Q1 n x n cells with n log-uniform in [32, %d] (drawn: %d..%d), four-quadrant "
                     "Riemann data, slip walls, t_final %.3g, Poisson arrivals at 20/s" % (
                         count, n_max, min(sizes), max(sizes), t_final),
            "batched": served, "one_at_a_time_fp64": single}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name, budget_s):
    """The oracle, as it stands, on a bounded sample of the same workload: all
    host cores (OpenMP over rows), then one core."""
    import oracle

    oracle.build()
    base = WORKLOADS[name][0]
    from paper_2402_04514_amd import workloads as W
    full = W.CONFIGS[name](**base)
    wl = full
    note = ""
    if full.mesh.ndofs > 300_000:  # one oracle step would exceed the budget: same problem, coarser
        f = {2: 8, 3: 4}.get(full.mesh.dim, 1)
        if "ntheta" in base:  # the cylinder's O-grid: both axes
            kw = dict(base, ntheta=base["ntheta"] // f, nr=base["nr"] // f)
        else:
            kw = dict(base, cells=full.mesh.cells[0] // f)
        if "cross" in kw:
            kw["cross"] = kw["cross"] // f
        wl = W.CONFIGS[name](**kw)
        note = "; the same problem on %s cells (1/%d per axis) to bound the CPU time" % (
            "x".join(str(c) for c in wl.mesh.cells), f)
    ms = wl.mesh
    M = oracle.Mesh(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc, bstate=ms.bstate, vortex=ms.vortex,
                    vertices=ms.vertices, bc_cells=ms.bc_cells, map_degree=ms.map_degree)
    prm = oracle.params(degree=ms.degree)

    def timed(threads, budget):
        oracle.set_num_threads(threads)
        U = wl.U0
        n, t0 = 0, time.perf_counter()
        while True:
            U, dt, _, st = M.step(prm, U)
            n += 1
            el = time.perf_counter() - t0
            if el > budget or n >= 1000:
                break
        return ms.ndofs * 3 * n / el, n, el

    allc = oracle.num_threads_available()
    log("cpu baseline: oracle on %d threads" % allc)
    rate, n, el = timed(allc, budget_s)
    log("cpu baseline: oracle on one thread")
    rate1, n1, el1 = timed(1, budget_s)
    oracle.set_num_threads(allc)
    return {"value": rate, "unit": "dof-stage updates/s", "cores": allc, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "single_core": {"value": rate1, "cores": 1, "steps": n1, "seconds": el1},
            "sample": "%d SSP-RK3 steps (%.1f s) of %s, %d dofs, oracle at gcc -O2 with OpenMP over "
                      "rows%s; then %d steps (%.1f s) on one thread" % (n, el, wl.name, ms.ndofs, note, n1, el1)}


def load_traffic(workload, kernels):
    """Measured HBM bytes per launch of each kernel from the committed counter
    profile, if it was taken on the current kernel source."""
    tf = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(tf):
        return None
    rec = json.load(open(tf))
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {})
    if not all(n in k for n in STAGE_KERNELS):
        return None
    # the primitives kernel runs once per run (after an upload or a reset),
    # not per stage: the stage traffic is that of the four stage kernels
    return {n: k[n] for n in kernels if n in STAGE_KERNELS}


STAGE_KERNELS = ("sweep1", "sweep2", "limit1", "limit2")


def _kernel_class(name):
    """'void gdg::k_limit<3, 1>(gdg::KArgs, ...)' -> 'limit'; None for kernels
    that are not one of the stage's."""
    import re
    m = re.search(r"gdg::k_(sweep1|sweep2|limit|prim)[<(]", name)
    return m.group(1) if m else None


def _region(rows, profile_steps):
    """The dispatches of the host-driven profile region at the end of the run:
    the last 3P launches of each sweep and the last 6P limiter launches, whose
    order within a stage gives the pass.  rows: (dispatch id, kernel name,
    value) in any order.  Returns {kernel: [values]}."""
    by = {"sweep1": [], "sweep2": [], "limit": []}
    for _, name, v in sorted(rows, key=lambda r: r[0]):
        c = _kernel_class(name)
        if c in by:
            by[c].append(v)
    n = 3 * profile_steps
    out = {"sweep1": by["sweep1"][-n:], "sweep2": by["sweep2"][-n:]}
    lim = by["limit"][-2 * n:]
    out["limit1"], out["limit2"] = lim[0::2], lim[1::2]
    if any(len(out[k]) != n for k in out):
        raise SystemExit("profile region incomplete: %s" % {k: len(v) for k, v in out.items()})
    return out


def _read_csv(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _find(dirname, suffix):
    for root, _, files in os.walk(dirname):
        for f in sorted(files):
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise SystemExit("no *%s under %s" % (suffix, dirname))


def summarize_counters(workload, fetch_dir, write_dir, profile_steps, copy_gib, commands):
    """profiles/traffic_<workload>.json (read by the bench line) and .md from
    two rocprofv3 --pmc runs of this script, FETCH_SIZE and WRITE_SIZE (KiB
    per dispatch), each scaled by what the same counter reads for the plain
    device copy of copy_gib GiB that the runs made (--calib-copy-gib)."""
    import statistics
    res = {}
    calib = {"copy_bytes": copy_gib * (1 << 30)}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _read_csv(_find(d, "counter_collection.csv")) if r["Counter_Name"] == counter]
        vals = [(int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"]) * 1024.0) for r in rows]
        copies = sorted(v for _, n, v in vals if "copyBuffer" in n)[-3:]
        if len(copies) < 3:
            raise SystemExit("no calibration copy in %s" % d)
        measured = statistics.median(copies)
        key = "fetch" if counter == "FETCH_SIZE" else "write"
        calib[key + "_measured"] = measured
        calib[key + "_scale"] = calib["copy_bytes"] / measured
        for k, v in _region(vals, profile_steps).items():
            res.setdefault(k, {})[key + "_bytes"] = statistics.mean(v) * calib[key + "_scale"]
            res[k]["dispatches"] = len(v)
    for k in res:
        res[k]["bytes_per_launch"] = res[k]["fetch_bytes"] + res[k]["write_bytes"]
    wl, desc = _workload(workload)
    slots, ghosts = stencil_slots(wl.mesh)
    N = wl.mesh.ndofs
    rec = {"workload": workload, "description": desc, "kernel_source_hash": kernel_source_hash(),
           "region": "the %d host-driven steps after the run's timed steps (%d stages)" % (profile_steps,
                                                                                       3 * profile_steps),
           "calibration": calib, "commands": commands, "kernels": res}
    base = os.path.join(ROOT, "profiles", "traffic_%s" % workload)
    with open(base + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    lines = ["# HBM traffic per launch: %s" % desc, "",
             "FETCH_SIZE and WRITE_SIZE from two `rocprofv3 --pmc` runs, averaged over the launches of "
             "the profile region (%s), kernel source %s." % (rec["region"], rec["kernel_source_hash"]),
             "Calibration: a plain %.0f GiB device copy in the same process reads FETCH_SIZE = %.3f GiB and "
             "WRITE_SIZE = %.3f GiB, so fetches are scaled by %.4f and writes by %.4f." % (
                 copy_gib, calib["fetch_measured"] / (1 << 30), calib["write_measured"] / (1 << 30),
                 calib["fetch_scale"], calib["write_scale"]), "",
             "| kernel | fetch GB | write GB | total GB | per-kernel model GB | measured / model |",
             "|---|---|---|---|---|---|"]
    for k in STAGE_KERNELS:
        mdl = algorithmic_bytes(k, wl.mesh.dim, slots, ghosts) * N
        r = res[k]
        lines.append("| %s | %.3f | %.3f | %.3f | %.3f | %.2f |" % (
            k, r["fetch_bytes"] / 1e9, r["write_bytes"] / 1e9, r["bytes_per_launch"] / 1e9, mdl / 1e9,
            r["bytes_per_launch"] / mdl))
    tot = sum(res[k]["bytes_per_launch"] for k in STAGE_KERNELS)
    lines += ["", "Stage total %.3f GB against the whole-stage model's %.3f GB (%.1f bytes per dof-stage)." % (
        tot / 1e9, b_alg(wl.mesh.dim, wl.mesh.degree) * N / 1e9, b_alg(wl.mesh.dim, wl.mesh.degree)), "",
              "Commands (from the repository root on the GPU box):", ""]
    lines += ["    " + c for c in commands]
    with open(base + ".md", "w") as f:
        f.write("\n".join(lines) + "\n")
    print(json.dumps({k: res[k]["bytes_per_launch"] for k in STAGE_KERNELS}))


def summarize_pmc(workload, dirs, profile_steps, commands):
    """profiles/counters_<workload>.md: the mean of every counter of the given
    rocprofv3 --pmc output folders over the launches of the profile region,
    per stage kernel, with the derived occupancy, VALU-busy and L2 hit
    figures."""
    import statistics
    vals = {}
    for d in dirs:
        rows = _read_csv(_find(d, "counter_collection.csv"))
        for cn in sorted(set(r["Counter_Name"] for r in rows)):
            sel = [(int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])) for r in rows
                   if r["Counter_Name"] == cn]
            for k, v in _region(sel, profile_steps).items():
                vals.setdefault(k, {})[cn] = statistics.mean(v)
    _, desc = _workload(workload)
    names = sorted(set(c for k in vals for c in vals[k]))
    out = ["# Counters per launch: %s" % desc, "",
           "Means over the launches of the profile region (the %d host-driven steps after the run's timed steps, "
           "%d launches of each kernel); one rocprofv3 --pmc pass per command below." % (profile_steps,
                                                                                    3 * profile_steps), "",
           "| counter | " + " | ".join(STAGE_KERNELS) + " |", "|---|" + "---|" * len(STAGE_KERNELS)]
    for cn in names:
        out.append("| %s | " % cn + " | ".join("%.4g" % vals[k].get(cn, float("nan")) for k in STAGE_KERNELS) + " |")

    def derived(label, f):
        cells = []
        for k in STAGE_KERNELS:
            try:
                cells.append("%.3f" % f(vals[k]))
            except (KeyError, ZeroDivisionError):
                cells.append("-")
        out.append("| %s | " % label + " | ".join(cells) + " |")

    out += ["", "Derived.  SQ_BUSY_CYCLES sums the busy cycles of the 32 shader engines and SQ_WAVE_CYCLES the "
                "resident time of every wave in units of four cycles, so the mean number of waves resident per "
                "SIMD (1024 SIMDs) is 4 SQ_WAVE_CYCLES / (SQ_BUSY_CYCLES / 32 x 1024); its agreement with the "
                "compiler's occupancy limit of each kernel checks that reading.", "",
            "| figure | " + " | ".join(STAGE_KERNELS) + " |", "|---|" + "---|" * len(STAGE_KERNELS)]
    derived("mean waves resident per SIMD", lambda v: v["SQ_WAVE_CYCLES"] / (8.0 * v["SQ_BUSY_CYCLES"]))
    derived("VALU-active share of wave time (SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES)",
            lambda v: v["SQ_ACTIVE_INST_VALU"] / v["SQ_WAVE_CYCLES"])
    derived("waiting share of wave time (SQ_WAIT_ANY / SQ_WAVE_CYCLES)", lambda v: v["SQ_WAIT_ANY"] / v["SQ_WAVE_CYCLES"])
    derived("VALU instructions per wave (SQ_INSTS_VALU / SQ_WAVES)", lambda v: v["SQ_INSTS_VALU"] / v["SQ_WAVES"])
    derived("L2 hit rate (TCC_HIT_sum / TCC_REQ_sum)", lambda v: v["TCC_HIT_sum"] / v["TCC_REQ_sum"])
    out += ["", "Commands (from the repository root on the GPU box):", ""] + ["    " + c for c in commands]
    with open(os.path.join(ROOT, "profiles", "counters_%s.md" % workload), "w") as f:
        f.write("\n".join(out) + "\n")


def summarize_trace(workload, trace_dir, bench_json, profile_steps, command):
    """profiles/kernels_<workload>.md from a rocprofv3 --kernel-trace --stats
    run of this script: the profiler's per-kernel statistics over the whole
    run, the launches of the profile region split by limiter pass (the
    launches the bench line's per-kernel HIP events time), and the bench line
    of the same run."""
    import statistics
    stats = _read_csv(_find(trace_dir, "kernel_stats.csv"))
    trace = _read_csv(_find(trace_dir, "kernel_trace.csv"))
    line = [json.loads(x) for x in open(bench_json).read().splitlines() if x.startswith('{"metric"')][-1]
    wl, desc = _workload(workload)
    rows = [(int(r["Dispatch_Id"]), r["Kernel_Name"],
             (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3) for r in trace]
    reg = _region(rows, profile_steps)
    res = {}
    for r in trace:
        c = _kernel_class(r["Kernel_Name"])
        if c and c not in res:
            res[c] = r
    out = ["# Kernel trace: %s" % desc, "", "Command (from the repository root on the GPU box):", "",
           "    " + command, "", "rocprofv3 kernel statistics over the whole run (microseconds):", "",
           "| kernel | calls | total us | average us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:12]:
        out.append("| %s | %s | %.1f | %.3f | %.3f | %.3f | %.2f |" % (
            r["Name"].replace("|", "/"), r["Calls"], float(r["TotalDurationNs"]) / 1e3,
            float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            float(r["Percentage"])))
    out += ["", "Launches of the host-driven profile region (%d steps after the timed run), the ones the bench "
                "line's `kernels_ms_per_launch` times with HIP events:" % profile_steps, "",
            "| kernel | launches | trace average us | bench HIP-event average us | VGPR_Count | Accum_VGPR_Count "
            "| SGPR_Count | LDS B |",
            "|---|---|---|---|---|---|---|---|"]
    for k in STAGE_KERNELS:
        r = res.get("limit" if k.startswith("limit") else k, {})
        ev = line.get("kernels_ms_per_launch", {}).get(k)
        out.append("| %s | %d | %.1f | %s | %s | %s | %s | %s |" % (
            k, len(reg[k]), statistics.mean(reg[k]), "%.1f" % (ev * 1e3) if ev else "-",
            r.get("VGPR_Count", "?"), r.get("Accum_VGPR_Count", "?"), r.get("SGPR_Count", "?"),
            r.get("LDS_Block_Size", "?")))
    out += ["", "The trace's VGPR_Count is half the VGPR count that the compiler's resource remark gives for the "
                "same kernel (k_limit<3,1>: 120 against 239); occupancy follows the compiler's figure, as the "
                "counter profile's measured waves per SIMD confirm."]
    rf = line["roofline"]
    out += ["", "Bench line of the same run: %.4e %s, %.3f ms/step, whole-stage roofline %.1f GB/s of %.0f "
                "(frac %.4f), dominant kernel %s at %.3f ms/launch." % (
                    line["value"], line["unit"], line["ms_per_step"], rf["achieved"], rf["peak"], rf["frac"],
                    rf["dominant_kernel"]["kernel"], rf["dominant_kernel"]["avg_launch_ms"])]
    with open(os.path.join(ROOT, "profiles", "kernels_%s.md" % workload), "w") as f:
        f.write("\n".join(out) + "\n")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="blast", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision line")
    ap.add_argument("--mixed-compare-steps", type=int, default=None,
                    help="steps of the mixed-vs-FP64 comparison (default: the workload's steps)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--serving-requests", type=int, default=48)
    ap.add_argument("--serving-nmax", type=int, default=512)
    ap.add_argument("--serving-tfinal", type=float, default=0.02)
    ap.add_argument("--serving-budget-gib", type=float, default=4.0)
    ap.add_argument("--serving-slots", type=int, default=64)
    ap.add_argument("--serving-solo-dofs", type=int, default=65536,
                    help="requests of at least this many dofs run their own single-mesh graph in the server")
    ap.add_argument("--serving-steps-per-graph", type=int, default=8,
                    help="device-driven steps per server launch (host pump once per launch)")
    ap.add_argument("--cells", type=int, default=0,
                    help="run the workload on another number of cells per side (scaling study only)")
    ap.add_argument("--profile-steps", type=int, default=10,
                    help="host-driven steps with per-launch HIP events after the timed region")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="also run a plain device copy of this size (counter calibration)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU work: write profiles/traffic_<workload>.json and .md from the output folders "
                         "of two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this script")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_DIR", "BENCH_JSON"),
                    help="no GPU work: write profiles/kernels_<workload>.md from a rocprofv3 --kernel-trace "
                         "--stats run of this script and the JSON line it printed")
    ap.add_argument("--summarize-pmc", nargs="+", metavar="PMC_DIR",
                    help="no GPU work: write profiles/counters_<workload>.md from rocprofv3 --pmc output folders")
    ap.add_argument("--command", action="append", default=[],
                    help="the profiling command(s) to record in the summary")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(args.workload, *args.summarize_counters, args.profile_steps,
                           args.calib_copy_gib or 1.0, args.command)
        return
    if args.summarize_pmc:
        summarize_pmc(args.workload, args.summarize_pmc, args.profile_steps, args.command)
        return
    if args.summarize_trace:
        summarize_trace(args.workload, *args.summarize_trace, args.profile_steps,
                        args.command[0] if args.command else "")
        return
    global CELLS_OVERRIDE
    CELLS_OVERRIDE = args.cells
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library runs the hot path on a single MI355X; "
              "sharding across GPUs is a design note, not built", file=sys.stderr)
        sys.exit(2)
    _, desc, dsteps, dwarm = WORKLOADS[args.workload]
    steps = args.steps if args.steps is not None else dsteps
    warmup = args.warmup if args.warmup is not None else dwarm

    log("fp64 %s: %d warmup steps, then %d timed steps from the initial state" % (args.workload, warmup, steps))
    r = run_gpu(args.workload, steps, warmup, profile_steps=args.profile_steps)
    wl, ndofs, secs = r["wl"], r["ndofs"], r["secs"]
    value = ndofs * 3 * steps / secs
    log("fp64: %.4e dof-stage/s (%.3f ms/step)" % (value, secs / steps * 1e3))
    dim, deg = wl.mesh.dim, wl.mesh.degree
    balg = b_alg(dim, deg)
    stage_s = secs / (3 * steps)
    achieved = balg * ndofs / stage_s / 1e9
    prof = r["prof"]
    prof_steps, prof_ms_step = r["prof_region"]
    kernels = [k for k in prof if prof[k][1] > 0]
    dom = max(kernels, key=lambda k: prof[k][0])
    slots, ghosts = stencil_slots(wl.mesh)
    dom_avg = prof[dom][0] / prof[dom][1] / 1e3
    dom_bytes = algorithmic_bytes(dom, dim, slots, ghosts) * ndofs
    traffic_k = load_traffic(args.workload, kernels)
    traffic_stage = None
    if traffic_k:
        # launches per stage: each profiled kernel's launches over the region's stages
        per_stage = {k: prof[k][1] / (3.0 * prof_steps) for k in traffic_k}
        traffic_stage = sum(traffic_k[k]["bytes_per_launch"] * per_stage[k] for k in traffic_k)
    if args.calib_copy_gib > 0:
        import torch
        n = int(args.calib_copy_gib * (1 << 30)) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "dof-stage updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": secs / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "description": desc, "dofs": ndofs, "precision": "fp64",
                   "timed": "steps 1..%d of the run from the initial state (warmup steps ran before on the same "
                            "context, which was then reset)" % steps},
        "roofline": {"bound": "hbm", "kernel": "stage (sweep 1, sweep 2, limiter passes 1 and 2)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_stage,
                     "traffic_gbs": traffic_stage / stage_s / 1e9 if traffic_stage else None,
                     "traffic_frac": traffic_stage / stage_s / 1e9 / HBM_PEAK_GBS if traffic_stage else None,
                     "algorithmic_bytes_per_dof_stage": balg,
                     "algorithmic_bytes_per_stage": balg * ndofs,
                     "avg_stage_ms": stage_s * 1e3,
                     "timing": "HIP events on the library stream around the timed region (%d steps, %d stages); "
                               "host clock %.3f s" % (steps, 3 * steps, r["secs_host"]),
                     "dominant_kernel": {
                         "kernel": dom, "avg_launch_ms": dom_avg * 1e3,
                         "model_bytes_per_launch": dom_bytes,
                         "model_gbs": dom_bytes / dom_avg / 1e9,
                         "traffic_bytes_per_launch": traffic_k[dom]["bytes_per_launch"]
                         if traffic_k and dom in traffic_k else None,
                         "traffic_gbs": traffic_k[dom]["bytes_per_launch"] / dom_avg / 1e9
                         if traffic_k and dom in traffic_k else None,
                         "timing": "HIP events around every launch on the library stream, %d host-driven steps "
                                   "after the timed region (%.3f ms/step)" % (prof_steps, prof_ms_step)}},
        "kernels_ms_per_launch": {k: (v[0] / v[1] if v[1] else None) for k, v in prof.items()},
        "windows": r["windows"],
        "checks": r["checks"],
    }
    if not args.no_mixed:
        from paper_2402_04514_amd import gdg
        log("mixed %s: %d timed steps" % (args.workload, steps))
        rm = run_gpu(args.workload, steps, warmup, gdg.GDG_MIXED, profile_steps=args.profile_steps)
        csteps = args.mixed_compare_steps if args.mixed_compare_steps is not None else steps
        log("mixed vs fp64 at equal time levels over %d steps" % csteps)
        cmp = mixed_vs_fp64(args.workload, csteps)
        mval = ndofs * 3 * steps / rm["secs"]
        line["mixed"] = {"value": mval, "unit": "dof-stage updates/s", "vs_fp64": mval / value,
                         "ms_per_step": rm["secs"] / steps * 1e3,
                         "roofline_frac": b_alg(dim, deg, True) * ndofs / (rm["secs"] / (3 * steps)) / 1e9 /
                         HBM_PEAK_GBS,
                         "algorithmic_bytes_per_dof_stage": b_alg(dim, deg, True),
                         "precision": "c_ij, flux and entropy-viscosity sums FP32; state, d_ij, bounds, "
                                      "line search FP64",
                         "checks": rm["checks"], "windows": rm["windows"],
                         "kernels_ms_per_launch": {k: (v[0] / v[1] if v[1] else None)
                                                   for k, v in rm["prof"].items()},
                         "vs_fp64_gpu": cmp}
    if not args.no_serving:
        log("serving")
        line["serving"] = serving(args.serving_requests, args.serving_nmax, args.serving_tfinal,
                                  args.serving_budget_gib, args.serving_slots, args.serving_steps_per_graph,
                                  args.serving_solo_dofs)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
