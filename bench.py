#!/usr/bin/env python3
"""Throughput of the graph-based DG hot path on one MI355X.

A step is one SSP-RK3 step of the convex-limited scheme (three forward-Euler
stages, each: primitives, sweep 1, sweep 2 with the cell solve, two limiter
passes) over the whole mesh, through the C-ABI of libgdg (gdg_run_to: the
device-driven loop of captured step graphs).  The metric is
dof-stage updates per second: dofs x 3 stages x steps / seconds, with the
state resident in HBM before the timed region starts.

Prints one JSON line.  Besides the contract fields it carries
  roofline      the dominant kernel's algorithmic bytes per launch over its
                average duration (HIP events on the library's stream, over a
                region of host-driven steps right after the timed one),
                against the 8 TB/s HBM peak; `traffic` from the committed
                FETCH_SIZE / WRITE_SIZE profile of the same kernel source;
  mixed         the mixed-precision variant on the same workload, and its L1
                difference from FP64 at equal time levels, beside the growth
                of a 1e-13 input perturbation under FP64 alone;
  serving       p50 / p99 time to solution and aggregate throughput of the
                batched request server on a Poisson trace of small 2D
                problems, against FIFO one-at-a-time FP64;
  cpu_baseline  the CPU oracle timed on this host's cores on a bounded sample.
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
    "vortex": ({}, "2D Euler DG Q1, 256x256 periodic cells on [-5,5]^2 (262,144 dofs), "
                   "isentropic vortex beta=5, gamma=1.4, FP64, convex-limited, SSP-RK3 at Cr=0.5", 400, 20),
    "quadrant": ({}, "2D Euler DG Q2, 1024x1024 cells on [0,1]^2 (9,437,184 dofs), seeded "
                     "four-quadrant Riemann data, outflow, FP64, convex-limited, SSP-RK3", 20, 3),
    "blast": ({}, "3D Euler DG Q1, 128^3 cells on [0,1]^3 (16,777,216 dofs), blast p=100 in r<0.1, "
                  "slip walls, FP64, convex-limited, SSP-RK3", 10, 2),
    "sod": ({}, "1D Euler DG Q1, 200 cells on [0,1] (400 dofs), Sod shock tube, outflow, FP64", 700, 20),
    "inflow": ({"cells": 1024, "dim": 2, "axis": 0, "degree": 2, "cross": 1024},
               "2D Euler DG Q2, 1024x1024 cells on [0,1]^2 (9,437,184 dofs), supersonic inflow (Dirichlet data "
               "rho,u,p = 1,2.5,1) into a supersonic stream (0.5,2.5,0.6), supersonic in/outflow faces in x, "
               "periodic in y, FP64, convex-limited, SSP-RK3", 20, 3),
}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("gdg_kernels.hip", "gdg_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2402_04514_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(kernel: str, dim: int, slots: float, ghosts: float = 0.0) -> float:
    """Bytes per row (dof) a kernel must move with each array touched once:
    stencil entries (int32 column, meta byte, dim doubles of c_ij), per-slot
    fields (d^L, l: doubles), per-dof fields.  Gathers of neighbour values
    count once (each value is needed once per sweep); re-reads through the
    caches are not algorithmic.  `ghosts` is the mean number of boundary parts
    per row, the only slots whose c_ij sweep 2 reads."""
    M = dim + 2
    st = slots * (4 + 1 + 8 * dim)    # column, meta, c_ij
    idx = slots * (4 + 1)             # column, meta
    if kernel == "prim":
        return 8 * M + 8 * (dim + 5)
    if kernel == "sweep1":   # U, node cache in; d^L, N, ring-1 partials, flux sums out
        return st + 8 * (M + dim + 5) + 8 * slots + 8 + 24 + 8 * M
    if kernel == "sweep2":   # U, u, p, N, q, d^L, flux sums in; U^L, bounds, dU^H out
        return idx + 8 * dim * ghosts + 8 * slots + 8 * (M + dim + 1) + 8 + 24 + 8 * M + 8 * M + 24 + 8 * M
    # U, base, dU^H, B, N, row length of i and of the neighbours (once); l out
    lim = idx + 8 * slots + 8 * M * 3 + 24 + 8 + 4 + 8 * M + 8 * slots
    if kernel == "limit1":
        return lim + 8 * M            # U^(1) out
    if kernel == "limit2":
        return lim + 8 * M + 8 * M    # l^(1) read (in 8*slots above), U^n in, stage output out
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
        # per axis: the nodes on a face touch nb^(d-1) neighbour nodes, or one ghost part
        face_nodes_frac = 2.0 / nb
        interior = 1.0 if periodic else (n - 1) / n
        tot += face_nodes_frac * (interior * nb ** (d - 1) + (1 - interior) * 1)
        ghost += face_nodes_frac * (1 - interior)
    return nb ** d + tot, ghost


def _params(gdg, degree, precision):
    p = gdg.gdg_default_params(degree)
    p.precision = precision
    return p


def run_gpu(name, steps, warmup, host_driven=False, precision=0):
    import numpy as np
    import torch

    from paper_2402_04514_amd import gdg
    from paper_2402_04514_amd import workloads as W

    kw, desc, _, _ = WORKLOADS[name]
    if CELLS_OVERRIDE:
        kw = dict(kw, cells=CELLS_OVERRIDE)
        desc = desc + " [cells per side overridden: %d]" % CELLS_OVERRIDE
    wl = W.CONFIGS[name](**kw)
    S = gdg.Solver.from_spec(wl.mesh, _params(gdg, wl.mesh.degree, precision), device="cuda:0")
    S.upload(wl.U0)
    if host_driven:   # every step host-driven, no graph (for counter collection)
        gdg.gdg_profile(S.ctx, True)
    if warmup:
        S.run_to(1e30, max_steps=warmup)   # also captures the step graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.run_to(1e30, max_steps=steps)         # device-driven: captured graphs of steps
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # kernel timing: HIP events around every launch on the library's stream,
    # over a second timed region of the same run (host-driven steps: events
    # recorded inside graphs carry no timestamps)
    prof_steps = max(1, min(steps, 50))
    gdg.gdg_profile(S.ctx, True)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    S.run_to(1e30, max_steps=prof_steps)
    torch.cuda.synchronize()
    p1 = time.perf_counter()
    prof = gdg.gdg_profile_read(S.ctx)
    gdg.gdg_profile(S.ctx, False)
    prof["_region"] = (prof_steps, (p1 - p0) / prof_steps * 1e3)
    out = S.download()
    dim = wl.mesh.dim
    eps = out[dim + 1] - 0.5 * np.sum(out[1:dim + 1] ** 2, 0) / out[0]
    admissible = bool(np.all(out[0] > 0) and np.all(eps > 0))
    return wl, desc, S.ndofs, t1 - t0, prof, admissible, S.stats()


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
    from paper_2402_04514_amd import workloads as W

    kw = WORKLOADS[name][0]
    wl = W.CONFIGS[name](**kw)
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
    dts = [S.step() for _ in range(steps)]
    ref = S.download()
    S.close()
    M = solver(gdg.GDG_MIXED, wl.U0)
    for dt in dts:
        M.step(dt_fixed=dt)
    mix = M.download()
    M.close()
    rng = np.random.default_rng(2402)
    Up = wl.U0.copy()
    Up[0] *= 1.0 + 1e-13 * rng.standard_normal(Up.shape[1])
    P = solver(gdg.GDG_FP64, Up)
    for dt in dts:
        P.step(dt_fixed=dt)
    per = P.download()
    P.close()
    comp, cons = norms(mix, ref)
    pcomp, pcons = norms(per, ref)
    return {"steps": steps, "t": float(sum(dts)), "l1_rel_per_component": comp, "l1_consolidated": cons,
            "fp64_perturbed_1e-13": {"l1_rel_per_component": pcomp, "l1_consolidated": pcons}}


def serving(count, n_max, t_final, budget_gib, max_slots, spg):
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
                   steps_per_graph=spg)
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
            print("[serving] %.1f s: %d submitted, %d finished" % (now, nsub, sum(d is not None for d in done)),
                  file=sys.stderr, flush=True)
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
              "precision": "mixed", "max_slots": max_slots, "steps_per_graph": spg,
              "budget_gib": budget_gib}
    S.close()
    # -- one at a time, FP64, FIFO
    service, work1 = [], 0.0
    for k, (a, wl) in enumerate(reqs):
        if k % 8 == 0:
            print("[serving] one at a time: request %d of %d" % (k, count), file=sys.stderr, flush=True)
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
    return {"trace": "%d requests, 2D Q1 n x n cells with n log-uniform in [32, %d], four-quadrant Riemann data, "
                     "slip walls, t_final %.3g, Poisson arrivals at 20/s" % (count, n_max, t_final),
            "batched": served, "one_at_a_time_fp64": single}


def cpu_baseline(name, budget_s):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    import oracle
    from paper_2402_04514_amd import workloads as W

    oracle.build()
    base = WORKLOADS[name][0]
    full = W.CONFIGS[name](**base)
    wl = full
    note = ""
    if full.mesh.ndofs > 300_000:  # one oracle step would exceed the budget: same problem, coarser
        f = {2: 8, 3: 4}.get(full.mesh.dim, 1)
        kw = dict(base, cells=full.mesh.cells[0] // f)
        if "cross" in kw:
            kw["cross"] = kw["cross"] // f
        wl = W.CONFIGS[name](**kw)
        note = "; the same problem on %s cells (1/%d per axis) to bound the CPU time" % (
            "x".join(str(c) for c in wl.mesh.cells), f)
    ms = wl.mesh
    M = oracle.Mesh(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc, bstate=ms.bstate)
    prm = oracle.params(degree=ms.degree)
    U = wl.U0
    n, t0 = 0, time.perf_counter()
    while True:
        U, dt, _, st = M.step(prm, U)
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s or n >= 1000:
            break
    rate = ms.ndofs * 3 * n / el
    return {"value": rate, "unit": "dof-stage updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d SSP-RK3 steps (%.1f s) of %s, %d dofs, oracle at gcc -O2 with OpenMP over "
                      "rows%s" % (n, el, wl.name, ms.ndofs, note)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="vortex", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision line")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--serving-requests", type=int, default=32)
    ap.add_argument("--serving-nmax", type=int, default=128)
    ap.add_argument("--serving-tfinal", type=float, default=0.25)
    ap.add_argument("--serving-budget-gib", type=float, default=4.0)
    ap.add_argument("--serving-slots", type=int, default=64)
    ap.add_argument("--serving-steps-per-graph", type=int, default=8,
                    help="device-driven steps per server launch (host pump once per launch)")
    ap.add_argument("--cells", type=int, default=0,
                    help="run the workload on another number of cells per side (scaling study only)")
    ap.add_argument("--host-driven", action="store_true",
                    help="run every step host-driven (no captured graphs), e.g. under counter collection")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="also run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()
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

    wl, desc, ndofs, secs, prof, admissible, stats = run_gpu(args.workload, steps, warmup, args.host_driven)
    value = ndofs * 3 * steps / secs
    slots, ghosts = stencil_slots(wl.mesh)
    prof_steps, prof_ms_step = prof.pop("_region")
    dom = max(prof, key=lambda k: prof[k][0])
    ms_tot, launches = prof[dom]
    avg_s = ms_tot / launches / 1e3
    bytes_launch = algorithmic_bytes(dom, wl.mesh.dim, slots, ghosts) * ndofs
    achieved = bytes_launch / avg_s / 1e9
    traffic, valu = None, None
    tf = os.path.join(ROOT, "profiles", "traffic_%s.json" % args.workload)
    if os.path.exists(tf):
        rec = json.load(open(tf))
        if rec.get("kernel_source_hash") == kernel_source_hash() and dom in rec.get("kernels", {}):
            traffic = rec["kernels"][dom]["bytes_per_launch"]
            valu = rec["kernels"][dom].get("valu_instructions")
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
        "config": {"workload": wl.name, "description": desc, "dofs": ndofs,
                   "precision": "fp64", "admissible_after": admissible,
                   "simulated_time": stats.t},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_gbs": traffic / avg_s / 1e9 if traffic else None,
                     "traffic_frac": traffic / avg_s / 1e9 / HBM_PEAK_GBS if traffic else None,
                     # FP64 VALU: wave64 instructions x 4 cycles (16 lanes per SIMD per
                     # cycle) over the cycles of 1024 SIMDs at 2.4 GHz
                     "valu_busy_est": (valu * 4.0 / (avg_s * 2.4e9 * 1024)) if valu else None,
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "avg_launch_ms": avg_s * 1e3,
                     "timing": "HIP events on the library stream around each launch, %d host-driven "
                               "steps right after the timed region (%.3f ms/step)" % (prof_steps, prof_ms_step)},
        "kernels_ms_per_launch": {k: (v[0] / v[1] if v[1] else None) for k, v in prof.items()},
    }
    if not args.no_mixed:
        from paper_2402_04514_amd import gdg
        _, _, _, msecs, mprof, madm, _ = run_gpu(args.workload, steps, warmup, args.host_driven, gdg.GDG_MIXED)
        cmp = mixed_vs_fp64(args.workload, min(steps, 50))
        line["mixed"] = {"value": ndofs * 3 * steps / msecs, "unit": "dof-stage updates/s",
                         "ms_per_step": msecs / steps * 1e3, "admissible_after": madm,
                         "precision": "c_ij, flux and entropy-viscosity sums FP32; state, d_ij, bounds, "
                                      "line search FP64",
                         "kernels_ms_per_launch": {k: (v[0] / v[1] if v[1] else None)
                                                   for k, v in mprof.items() if not k.startswith("_")},
                         "vs_fp64_gpu": cmp}
    if not args.no_serving:
        line["serving"] = serving(args.serving_requests, args.serving_nmax, args.serving_tfinal,
                                  args.serving_budget_gib, args.serving_slots, args.serving_steps_per_graph)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
