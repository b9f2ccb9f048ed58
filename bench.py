"""Benchmark: discrete-velocity BGK primal + adjoint sweeps on one MI355X.

Workload (default): NACA0012 C-grid 256x128 (32768 cells), 48x48
Newton-Cotes velocity grid on [-6, 6] (2304 velocities), Kn 0.1, Ma 0.8,
diffuse wall T_w = 1, 16 Hicks-Henne shape parameters; FP64.

One step = one fixed-budget solve through the whole hot path: far-field
initialisation, S primal Jacobi sweeps (moments, Maxwellian, upwind fluxes,
wall flux, residual partials), drag, adjoint initialisation, S adjoint
sweeps (adjoint moments, wall multiplier), wall sensitivity, node transform
and the chain to the shape parameters.  Inputs (mesh, velocity tables) are
resident in HBM before timing starts.

Metric: cell-velocity updates per second, primal + adjoint
(= cells * velocities * 2S / step time).  Printed as one JSON line with the
roofline of the dominant kernel (adjoint sweep), the mixed-precision path
on the same workload, and the oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, vendor figure
# the sweep and second-order kernels, their layout constants and the host-built sweep order
KERNEL_SRCS = [os.path.join(ROOT, "paper_2501_00923_amd", "csrc", f)
               for f in ("dvm_kernels.hip", "dvm_so.hip", "dvm_device.h", "dvm_internal.h", "dvm_host.cpp")]
# scaled FETCH_SIZE + WRITE_SIZE per launch of the sweeps, from the counter
# runs of each workload (bench.py --workload c2 | c3)
TRAFFIC_FILES = {"c2": os.path.join(ROOT, "profiles", "sweeps_naca0012_c256x128_v48_traffic.json"),
                 "c3": os.path.join(ROOT, "profiles", "sweeps_naca0012_c256x128_v64sinh_traffic.json")}


def kernel_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(key: str) -> dict:
    """The counted traffic of a workload, or {} when the counters were taken
    on other kernel code."""
    path = TRAFFIC_FILES[key]
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        tr = json.load(fh)
    return tr if tr.get("kernel_sha") == kernel_hash() else {}


def bytes_per_update(kind: str, mixed: bool) -> int:
    """Algorithmic HBM bytes per (cell, velocity) per sweep: own row read +
    written once (2 values), plus the frozen primal row for the adjoint."""
    e = 4 if mixed else 8
    return (4 if kind == "primal" else 6) * e


def so_bytes_per_update(kind: str, mixed: bool, corr_per_sweep: float) -> dict:
    """Bytes per (cell, velocity) of the second-order path as built, per
    sweep: the sweep's own row traffic plus the held correction it reads,
    and the correction kernels' traffic times the corrections per sweep
    (one at the first sweep after init, then one every K sweeps; primal:
    slopes read f, write G (4 values); correction reads G, writes c.
    Adjoint: B reads phi and psi, writes B (4); E reads B, writes E)."""
    e = 4 if mixed else 8
    if kind == "primal":
        sweep, corr = 6 * e, (2 + 4) * e + (4 + 2) * e
    else:
        sweep, corr = 8 * e, (2 + 2 + 4) * e + (4 + 2) * e
    return {"sweep": sweep, "correction": corr, "per_sweep": sweep + corr * corr_per_sweep}


def run_gpu(wl, precision, sweeps, steps, warmup, order=1, correction_every=40):
    import numpy as np
    import torch

    from paper_2501_00923_amd import dvm

    s = dvm.Solver.from_workload(wl, precision=precision, order=order, correction_every=correction_every)
    jac = wl.grid.wall_jac
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    tp, ta = [], []
    out = {}

    def step(record):
        s.primal_init()
        ev[0].record()
        s.primal_sweeps(sweeps)
        ev[1].record()
        J, Cd = s.objective()
        s.adjoint_init()
        ev[2].record()
        s.adjoint_sweeps(sweeps)
        ev[3].record()
        dJ = s.param_sensitivity(jac) if order == 1 else None
        if record:
            torch.cuda.synchronize()
            tp.append(ev[0].elapsed_time(ev[1]) / sweeps)
            ta.append(ev[2].elapsed_time(ev[3]) / sweeps)
        out["J"], out["Cd"], out["dJ"] = J, Cd, dJ

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pairs = s.nc * s.nv
    ms_step = (t1 - t0) * 1e3 / steps
    out.update(pairs=pairs, ms_per_step=ms_step,
               updates_per_s=pairs * 2 * sweeps / (ms_step * 1e-3),
               primal_sweep_ms=float(np.mean(tp)), adjoint_sweep_ms=float(np.mean(ta)))
    del s
    torch.cuda.empty_cache()
    return out


def c1_leg(repeats=5):
    """The circle O-grid 64x32 with 16x16 midpoint velocities on [-5, 5] (Kn 1,
    Ma 0.5), FP64: one whole solve -- primal to a relative residual of 1e-8
    (checked every 50 sweeps), drag, adjoint to 1e-8, the 8 Fourier-mode
    sensitivities -- timed on the host clock with the device synchronised
    on both sides; the solver's buffer is allocated once, outside the timed
    region.  One untimed solve first, then `repeats` timed ones."""
    import torch

    from paper_2501_00923_amd import dvm
    from paper_2501_00923_amd import inputs as I

    wl = I.c1_circle()
    s = dvm.Solver.from_workload(wl, precision=dvm.FP64)
    times = []
    for rep in range(repeats + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.primal_init()
        itp, rp = s.primal_iterate(20000, tol=1e-8, check_every=50)
        J, Cd = s.objective()
        s.adjoint_init()
        ita, ra = s.adjoint_iterate(20000, tol=1e-8, check_every=50)
        g = s.param_sensitivity(wl.grid.wall_jac)
        torch.cuda.synchronize()
        if rep > 0:
            times.append(time.perf_counter() - t0)
    times.sort()
    med = times[len(times) // 2]
    pairs = wl.grid.ni * wl.grid.nj * wl.vgrid.n1 * wl.vgrid.n2
    return {"workload": wl.name, "precision": "fp64", "tol": 1e-8, "primal_sweeps": itp, "adjoint_sweeps": ita,
            "primal_resid": rp, "adjoint_resid": ra, "Cd": Cd, "dJ_dparams": [float(x) for x in g],
            "solve_ms_median": med * 1e3, "solve_ms_min": times[0] * 1e3, "repeats": repeats,
            "updates_per_s": pairs * (itp + ita) / med}


def batch_roofline(n_members, seed, sweeps=20, warmup=3):
    """Achieved HBM rate of the batched sweep kernels on a serving mix: the
    first `n_members` requests of the seeded serving stream (circle / NACA,
    meshes 64x32 .. 256x128, 16^2 .. 64^2 velocities), FP32 state.  Three
    batches are timed with HIP events on their stream: every member in its
    primal phase (k_batch_primal alone), the members that ask for the
    adjoint in their adjoint phase (k_batch_adjoint alone), and the serving
    mix (those in the adjoint phase, the others primal: both kernels per
    sweep).  Algorithmic bytes per sweep: 16 B per primal and 24 B per
    adjoint (cell, velocity) pair of the members."""
    import torch

    from paper_2501_00923_amd import dvm
    from paper_2501_00923_amd import inputs as I

    reqs = I.poisson_stream(n_members, 1.0, seed=seed)

    def members(adjoint_of):
        out = []
        for r in reqs:
            if adjoint_of == "only" and not r.want_adjoint:
                continue
            s = dvm.Solver.from_workload(r.workload, precision=dvm.MIXED, want_adjoint=r.want_adjoint)
            s.primal_init()
            if r.want_adjoint and adjoint_of in ("only", "mix"):
                s.adjoint_init()
            out.append(s)
        return out

    def timed(sol):
        b = dvm.Batch(sol)
        b.run(warmup)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        b.run(sweeps)
        e1.record()
        torch.cuda.synchronize()
        b.close()
        ms = e0.elapsed_time(e1) / sweeps
        nbytes = sum(s.nc * s.nv * (24 if s.phase == 1 else 16) for s in sol)
        pairs = sum(s.nc * s.nv for s in sol)
        return {"members": len(sol), "pairs": pairs, "ms_per_sweep": ms, "algorithmic_bytes_per_sweep": nbytes,
                "achieved": nbytes / (ms * 1e-3) / 1e9, "frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "updates_per_s": pairs / (ms * 1e-3)}

    out = {}
    for key, kind, kern in (("primal", "none", "k_batch_primal<float, false>"),
                            ("adjoint", "only", "k_batch_adjoint<float, false>"),
                            ("mix", "mix", "both")):
        sol = members(kind)
        out[key] = timed(sol)
        out[key]["kernel"] = kern
        print(f"[bench] batch {key}: {out[key]['members']} members, {out[key]['ms_per_sweep']:.3f} ms/sweep, "
              f"{out[key]['achieved']:.0f} GB/s ({out[key]['frac']:.3f} of peak)", file=sys.stderr, flush=True)
        del sol
        torch.cuda.empty_cache()
    out["unit"] = "GB/s"
    out["peak"] = HBM_PEAK_GBS
    out["workload"] = f"first {n_members} requests of the serving stream (seed {seed}), FP32 state"
    return out


def serving_leg(n_requests, seed, cap, tol, budget_gb, check_every, accel_below_kn=None, accel=(5, 75)):
    """Solve server on a seeded request stream (circle / NACA shapes, meshes
    {64x32, 128x64, 256x128}, velocity grids {16^2, 32^2, 64^2} on [-6, 6],
    Kn log-uniform in [1e-3, 10], Ma in [0.3, 2], half wanting the adjoint).
    1) closed loop (all requests at t = 0), continuous batching, mixed
       precision -> capacity (solves/s);
    2) Poisson arrivals at 0.8 x capacity: continuous batching, mixed;
    3) the same arrivals, one solve at a time, FP64.
    Returns solves/s, p50/p99 latency of 2) and 3) and the drag agreement
    between them."""
    import numpy as np

    from paper_2501_00923_amd import dvm
    from paper_2501_00923_amd import inputs as I
    from paper_2501_00923_amd import serving as S

    cfg = S.ServeConfig(memory_budget=int(budget_gb * 2 ** 30), sweeps_per_check=check_every, tol=tol,
                        adjoint_tol=tol, max_iter=cap)
    reqs = I.poisson_stream(n_requests, 1.0, seed=seed)
    t0 = time.perf_counter()

    def backend(prec):
        return S.GpuBackend(prec, accelerate_below_kn=accel_below_kn, accelerate=accel)
    def progress(label):
        def f(res, n):
            if n % 64 == 0:
                print(f"[bench] serving {label}: {n}/{n_requests} finished ({time.perf_counter() - t0:.0f} s)",
                      file=sys.stderr, flush=True)
        return f
    cap_run = S.serve(reqs, backend(dvm.MIXED), cfg, realtime=False, on_finish=progress("capacity"))
    capacity = cap_run["solves_per_s"]
    print(f"[bench] serving capacity {capacity:.2f} solves/s ({time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    rate = 0.8 * capacity
    stream = I.poisson_stream(n_requests, rate, seed=seed)
    mix = S.serve(stream, backend(dvm.MIXED), cfg, realtime=True, on_finish=progress("batched mixed"))
    c = mix["converged"]
    print(f"[bench] batched mixed: {c['count']} converged, {c['solves_per_s']:.2f} solves/s p50 {c['p50_ms']:.0f} ms "
          f"p99 {c['p99_ms']:.0f} ms; {mix['notconv']} capped", file=sys.stderr, flush=True)
    one = S.serve_one_at_a_time(stream, backend(dvm.FP64), cfg, realtime=True, on_finish=progress("one at a time"))
    c = one["converged"]
    print(f"[bench] one-at-a-time fp64: {c['count']} converged, {c['solves_per_s']:.2f} solves/s p50 "
          f"{c['p50_ms']:.0f} ms p99 {c['p99_ms']:.0f} ms; {one['notconv']} capped", file=sys.stderr, flush=True)
    # drag agreement only where both modes reached the tolerance: a capped
    # solve's drag is not the converged drag in either mode
    rel = []
    for a, b in zip(mix["results"], one["results"]):
        if a.status == "ok" and b.status == "ok" and b.J != 0:
            rel.append(abs(a.J - b.J) / abs(b.J))
    rel = np.array(rel)

    def summary(o):
        return {"converged": o["converged"], "capped": o["capped"], "capped_by_kn": o["capped_by_kn"],
                "all_finished": {"solves_per_s": o["solves_per_s"], "p50_ms": o["p50_ms"], "p99_ms": o["p99_ms"],
                                 "mean_ms": o["mean_ms"], "count": o["completed"]},
                "failed": o["failed"], "wall_s": o["wall_s"], "peak_resident": o["peak_resident"],
                "peak_GB": o["peak_bytes"] / 1e9,
                "failed_requests": [{"rid": r.rid, "workload": next(q.workload.name for q in stream if q.rid == r.rid),
                                     "error": r.error} for r in o["results"] if r.status == "failed"]}
    cm, co = mix["converged"], one["converged"]
    return {"requests": n_requests, "seed": seed, "arrival_rate_per_s": rate, "capacity_solves_per_s": capacity,
            "tol": tol, "iteration_cap": cap, "sweeps_per_check": check_every, "memory_budget_GB": budget_gb,
            "accelerate_below_kn": accel_below_kn, "accelerate_every_inner": list(accel),
            "batched_mixed": summary(mix), "one_at_a_time_fp64": summary(one),
            "drag_rel_diff_mixed_vs_fp64_converged_in_both": {
                "count": int(len(rel)), "median": float(np.median(rel)) if len(rel) else None,
                "max": float(rel.max()) if len(rel) else None},
            "converged_speedup_solves_per_s": cm["solves_per_s"] / co["solves_per_s"] if co["solves_per_s"] else None,
            "converged_p99_ratio_fp64_over_mixed": co["p99_ms"] / cm["p99_ms"] if cm["p99_ms"] else None,
            "all_finished_speedup_solves_per_s": mix["solves_per_s"] / one["solves_per_s"],
            "all_finished_p99_ratio_fp64_over_mixed": one["p99_ms"] / mix["p99_ms"]}


def precision_sweep(sweeps, kns, oracle_check_sweeps=2, order=1):
    """Mixed precision (FP32 f/phi, FP64 moments and integrals) against the
    FP64 path on the NACA0012 256x128 C-grid with the 64x64 sinh velocity
    grid, Ma 0.5, for each Kn: the same number of primal and adjoint sweeps
    from the free stream on both; errors of J, C_d, the 16 bump
    sensitivities and the cell moments.  The FP64 path is itself checked
    against the oracle at full size after a few sweeps (first Kn).  order 2:
    the second-order scheme (Venkatakrishnan limiter, correction every 40
    sweeps) on both paths."""
    import numpy as np

    from paper_2501_00923_amd import dvm
    from paper_2501_00923_amd import inputs as I

    rows = []
    for i, Kn in enumerate(kns):
        wl = I.c3_naca_sinh(Kn)
        res = {}
        for prec, name in ((dvm.FP64, "fp64"), (dvm.MIXED, "mixed")):
            s = dvm.Solver.from_workload(wl, precision=prec, order=order)
            s.primal_init()
            _, rp = s.primal_iterate(sweeps)
            J, Cd = s.objective()
            W = s.moments()
            s.adjoint_init()
            _, ra = s.adjoint_iterate(sweeps)
            g = s.param_sensitivity(wl.grid.wall_jac)
            res[name] = dict(J=J, Cd=Cd, W=W, g=g, rp=rp, ra=ra)
            del s
        a, b = res["mixed"], res["fp64"]
        row = {"Kn": Kn, "order": order, "sweeps": sweeps, "J_fp64": b["J"], "Cd_fp64": b["Cd"],
               "primal_resid_fp64": b["rp"], "primal_resid_mixed": a["rp"],
               "adjoint_resid_fp64": b["ra"], "adjoint_resid_mixed": a["ra"],
               "J_rel_err": abs(a["J"] - b["J"]) / abs(b["J"]),
               "Cd_rel_err": abs(a["Cd"] - b["Cd"]) / abs(b["Cd"]),
               "dJda_rel_err": float(np.max(np.abs(a["g"] - b["g"])) / np.max(np.abs(b["g"]))),
               "W_rel_err": float(np.max(np.abs(a["W"] - b["W"])) / np.max(np.abs(b["W"])))}
        if i == 0 and oracle_check_sweeps > 0:
            import oracle
            nthreads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
            o = oracle.Problem.from_workload(wl, nthreads=nthreads)
            if order == 2:
                o.set_scheme(2, True, 40)
            o.primal_init()
            o.primal_iterate(oracle_check_sweeps)
            s = dvm.Solver.from_workload(wl, precision=dvm.FP64, order=order)
            s.primal_init()
            s.primal_iterate(oracle_check_sweeps)
            row["fp64_vs_oracle_J_rel"] = abs(s.objective()[0] - o.objective()) / abs(o.objective())
            row["fp64_vs_oracle_W_rel"] = float(np.max(np.abs(s.moments() - o.W)) / np.max(np.abs(o.W)))
            row["oracle_check_sweeps"] = oracle_check_sweeps
            del s, o
        print(f"[precision] Kn {Kn:g}: J err {row['J_rel_err']:.2e}  dJ/da err {row['dJda_rel_err']:.2e}  "
              f"W err {row['W_rel_err']:.2e}", file=sys.stderr, flush=True)
        rows.append(row)
    return rows


def fd_check(h, tol, params=None, order=1, limiter=True):
    """The differentiation workload (seed-drawn NACA thickness and camber,
    192x96 C-grid, 48x48 Newton-Cotes grid, Kn 0.5, Ma 2, 24 B-spline
    offsets): dJ/dalpha from the adjoint through the autograd wrapper
    (primal f snapshotted every 50 sweeps), in the paper's wall-only form and
    in the exact discrete form, against central differences J(alpha +- h e_p)
    of re-converged primal solves.  order 2: the second-order scheme
    (correction every 40 sweeps; with the Venkatakrishnan limiter the exact
    form holds the limiter factors fixed, without it it is exact)."""
    import numpy as np
    import torch

    from paper_2501_00923_amd import autograd as AG
    from paper_2501_00923_amd import dvm

    opts = AG.SolveOptions(max_iter=60000, tol=tol, adjoint_max_iter=60000, adjoint_tol=tol, check_every=100)
    case, a0 = AG.naca_bspline_case(seed=0, options=opts, checkpoint_every=50, keep_checkpoints=1)
    case.order = order
    case.limiter = dvm.LIMITER_VENKAT if limiter else dvm.LIMITER_NONE
    rec = AG.ForwardRecord()
    alpha = torch.tensor(a0, requires_grad=True)
    t0 = time.perf_counter()
    J = AG.drag(alpha, case, rec)
    J.backward()
    t_grad = time.perf_counter() - t0
    g = alpha.grad.numpy().copy()
    case.exact = True
    alpha_e = torch.tensor(a0, requires_grad=True)
    AG.drag(alpha_e, case).backward()
    ge = alpha_e.grad.numpy().copy()
    case.exact = False
    print(f"[fd] J {J.item():.12e}, primal {rec.iters} sweeps (resid {rec.resid:.1e}), adjoint "
          f"{rec.adjoint_iters} sweeps (resid {rec.adjoint_resid:.1e}), {t_grad:.1f} s", file=sys.stderr, flush=True)
    case.checkpoint_every = 0
    params = list(range(len(a0))) if params is None else params
    rows = []
    t0 = time.perf_counter()
    for p in params:
        e = np.zeros_like(a0)
        e[p] = h
        rp, rm = AG.ForwardRecord(), AG.ForwardRecord()
        Jp = AG.drag(torch.tensor(a0 + e), case, rp).item()
        Jm = AG.drag(torch.tensor(a0 - e), case, rm).item()
        fd = (Jp - Jm) / (2 * h)
        rows.append({"param": p, "adjoint": float(g[p]), "adjoint_exact": float(ge[p]),
                     "fd": fd,
                     "sweeps": [rp.iters, rm.iters]})
        print(f"[fd] p {p:2d}: adjoint (wall-only) {g[p]: .6e}  adjoint (exact) {ge[p]: .10e}  fd {fd: .10e}",
              file=sys.stderr, flush=True)
    gv = np.array([r["adjoint"] for r in rows])
    ev = np.array([r["adjoint_exact"] for r in rows], dtype=float)
    fv = np.array([r["fd"] for r in rows])
    scale = float(np.max(np.abs(fv)))
    return {"workload": "naca_bspline_c192x96_v48nc_kn0.5_ma2 (seed 0)", "order": order,
            "limiter": "venkatakrishnan" if (order == 2 and limiter) else None, "h": h, "tol": tol,
            "J": J.item(),
            "primal_sweeps": rec.iters, "adjoint_sweeps": rec.adjoint_iters,
            "checkpoints_kept": len(rec.checkpoints), "last_checkpoint_sweep": rec.checkpoint_iters[-1],
            "grad_seconds": t_grad, "fd_seconds": time.perf_counter() - t0,
            "wall_only": {"max_abs_diff_over_max_fd": float(np.max(np.abs(gv - fv)) / scale),
                          "median_rel_diff": float(np.median(np.abs(gv - fv) / np.maximum(np.abs(fv), 1e-3 * scale))),
                          "cosine": float(gv @ fv / (np.linalg.norm(gv) * np.linalg.norm(fv)))},
            "exact": {
                "max_abs_diff_over_max_fd": float(np.max(np.abs(ev - fv)) / scale),
                "median_rel_diff": float(np.median(np.abs(ev - fv) / np.maximum(np.abs(fv), 1e-3 * scale)))},
            "rows": rows}


def optimize_leg(n_wake, n_half, nj, nv, Kn, Ma, max_steps, gradient, tol, radius, sigma, order=1,
                 max_sweeps=200000, mixed=False, adjoint_tol=None):
    """The optimisation loop of Sec. 3.4 on a NACA0012 C-grid ((2 n_wake +
    2 n_half) x nj cells), nv x nv Newton-Cotes velocities on [-6, 6]:
    CST fit (N_B = 6), Wendland-C0 RBF motion, warm-started primal and
    adjoint solves to `tol`, SLSQP under eq. (cst_constraint) and Q <= 0,
    stopping by eq. (criterion_opt).  Reports J and Q per step, the time of
    each stage and the host-inclusive time of one mesh motion and one
    transpose."""
    import numpy as np

    from paper_2501_00923_amd import inputs as I
    from paper_2501_00923_amd.optimize import ShapeOptimizer

    g = I.naca_cgrid(n_wake, n_half, nj, t=0.12)
    wl = I.Workload(f"naca0012_c{g.ni}x{nj}_v{nv}nc_kn{Kn:g}_ma{Ma:g}", g,
                    I.VGridSpec(I.VG_NEWTON_COTES, nv, nv, 6.0), I.FlowSpec(Kn, Ma, 1.0), 0)
    from paper_2501_00923_amd import dvm
    opt = ShapeOptimizer(wl, radius=radius, sigma=sigma, gradient=gradient, solve_tol=tol, order=order,
                         adjoint_tol=adjoint_tol,
                         precision=dvm.MIXED if mixed else dvm.FP64, max_sweeps=max_sweeps, progress=lambda m: print(f"[optimize] {m}", file=sys.stderr, flush=True))
    print(f"[optimize] {wl.name}: CST fit rms {opt.fit_rms:.2e}, V_min {opt.v_min:.6f}", file=sys.stderr, flush=True)
    r = opt.run(max_steps=max_steps)
    hist = r["history"]
    for k, e in enumerate(hist):
        print(f"[optimize] step {k}: Cd {e.Cd:.8f}  Q/V_min {e.Q / r['v_min']:+.2e}  N1 {e.alpha[0]:.4f} "
              f"N2 {e.alpha[1]:.4f}", file=sys.stderr, flush=True)
    evs = list(opt._cache.values())
    stages = {k: float(sum(e.times.get(k, 0.0) for e in evs)) for k in ("deform", "setup", "primal", "adjoint", "sens")}
    sweeps = {"primal": int(sum(e.primal[0] for e in evs)), "adjoint": int(sum(e.adjoint[0] for e in evs))}
    pairs = g.ni * g.nj * nv * nv
    # host-inclusive mesh motion and transpose on this grid
    wall = opt.wall0.copy()
    gvec = np.ones((g.nj + 1, g.ni + 1, 2))
    for _ in range(3):
        opt.deform.apply(wall)
        opt.deform.chain(gvec)
    t0 = time.perf_counter()
    for _ in range(20):
        opt.deform.apply(wall)
    t_apply = (time.perf_counter() - t0) / 20
    t0 = time.perf_counter()
    for _ in range(20):
        opt.deform.chain(gvec)
    t_chain = (time.perf_counter() - t0) / 20
    return {"workload": wl.name, "order": order, "precision": "mixed" if mixed else "fp64", "gradient": gradient,
            "solve_tol": tol, "adjoint_tol": opt.adjoint_tol, "max_sweeps": max_sweeps,
            "radius": radius,
            "sigma": sigma, "n_params": len(opt.alpha0), "free_params": int(len(opt.free)),
            "fit_rms": opt.fit_rms, "v_min": r["v_min"], "steps": len(hist) - 1, "stop": r["message"],
            "evaluations": r["evaluations"], "gradients": int(sum(e.dJ is not None for e in evs)),
            "Cd": [e.Cd for e in hist], "Q_over_vmin": [e.Q / r["v_min"] for e in hist],
            "drag_change": hist[-1].Cd / hist[0].Cd - 1.0, "alpha_final": [float(x) for x in hist[-1].alpha],
            "seconds": r["seconds"], "stage_seconds": stages, "sweeps": sweeps,
            "unconverged_solves": r["unconverged_solves"],
            "solve_updates_per_s": (sweeps["primal"] + sweeps["adjoint"]) * pairs
            / max(stages["primal"] + stages["adjoint"], 1e-9),
            "mesh_nodes": (g.ni + 1) * (g.nj + 1), "wall_nodes": opt.deform.nw,
            "deform_apply_ms": t_apply * 1e3, "deform_chain_ms": t_chain * 1e3}


def cst_fd_check(n_wake, n_half, nj, nv, Kn, Ma, h, tol, radius, order=1, limiter=True, max_sweeps=200000):
    """Sensitivity of the drag to the CST design variables (the check of
    Sec. 4.1, here on a NACA0012 C-grid in free stream): at the fitted
    initial design, dJ/dalpha from the adjoint in the paper's wall-node form
    (eq. sens_nod) and in the exact discrete form (mesh sensitivity chained
    through the RBF motion), against central differences J(alpha +- h e_p)
    of re-converged primal solves, over the free variables."""
    import numpy as np

    from paper_2501_00923_amd import inputs as I
    from paper_2501_00923_amd.optimize import ShapeOptimizer

    g = I.naca_cgrid(n_wake, n_half, nj, t=0.12)
    wl = I.Workload(f"naca0012_c{g.ni}x{nj}_v{nv}nc_kn{Kn:g}_ma{Ma:g}", g,
                    I.VGridSpec(I.VG_NEWTON_COTES, nv, nv, 6.0), I.FlowSpec(Kn, Ma, 1.0), 0)
    from paper_2501_00923_amd import dvm
    opt = ShapeOptimizer(wl, radius=radius, gradient="exact", solve_tol=tol, check_every=100, order=order,
                         limiter=dvm.LIMITER_VENKAT if limiter else dvm.LIMITER_NONE, max_sweeps=max_sweeps)
    a0 = opt.alpha0
    t0 = time.perf_counter()
    ev = opt.evaluate(a0)
    ge = ev.dJ.copy()
    gp = ev.deta.T @ ev.solver.wall_sensitivity()["dJ_dnodes"][:, 1]
    t_grad = time.perf_counter() - t0
    print(f"[cst-fd] {wl.name}: J {ev.J:.12e}, primal {ev.primal[0]} sweeps, adjoint {ev.adjoint[0]} sweeps, "
          f"{t_grad:.1f} s", file=sys.stderr, flush=True)
    names = ["N1", "N2"] + [f"A_u{b}" for b in range(opt.nb + 1)] + [f"A_l{b}" for b in range(opt.nb + 1)]
    rows = []
    t0 = time.perf_counter()
    for p in opt.free:
        e = np.zeros_like(a0)
        e[p] = h
        Jp = opt.evaluate(a0 + e, gradient=False).J
        Jm = opt.evaluate(a0 - e, gradient=False).J
        fd = (Jp - Jm) / (2 * h)
        rows.append({"param": names[p], "adjoint_paper": float(gp[p]), "adjoint_exact": float(ge[p]), "fd": fd})
        print(f"[cst-fd] {names[p]:5s}: paper {gp[p]: .6e}  exact {ge[p]: .10e}  fd {fd: .10e}",
              file=sys.stderr, flush=True)
    fv = np.array([r["fd"] for r in rows])
    scale = float(np.max(np.abs(fv)))

    def stats(v):
        return {"max_abs_diff_over_max_fd": float(np.max(np.abs(v - fv)) / scale),
                "median_rel_diff": float(np.median(np.abs(v - fv) / np.maximum(np.abs(fv), 1e-3 * scale))),
                "cosine": float(v @ fv / (np.linalg.norm(v) * np.linalg.norm(fv)))}

    return {"workload": wl.name, "order": order, "limiter": bool(order == 2 and limiter), "h": h, "tol": tol,
            "radius": radius, "J": ev.J, "grad_seconds": t_grad,
            "fd_seconds": time.perf_counter() - t0,
            "paper": stats(np.array([r["adjoint_paper"] for r in rows])),
            "exact": stats(np.array([r["adjoint_exact"] for r in rows])), "rows": rows}


def accel_check(kns, every, inner, cap, tol, plain_cap, precision_name="fp64"):
    """The 256x128 NACA0012 C-grid with 64x64 sinh velocities (Ma 0.5),
    conservative equilibrium: primal then adjoint solves to `tol` with the
    macroscopic prediction (every `every` sweeps, `inner` red-black steps),
    and the plain iteration with at most `plain_cap` sweeps per phase, for
    each Kn: sweeps, residual reached, seconds, drag and its agreement."""
    import numpy as np

    from paper_2501_00923_amd import dvm
    from paper_2501_00923_amd import inputs as I

    prec = dvm.FP64 if precision_name == "fp64" else dvm.MIXED
    rows = []
    for Kn in kns:
        wl = I.c3_naca_sinh(Kn)
        row = {"Kn": Kn, "workload": wl.name}
        for label, acc, mx in (("accelerated", (every, inner), cap), ("plain", None, plain_cap)):
            s = dvm.Solver.from_workload(wl, precision=prec, equilibrium=dvm.EQ_CONSERVATIVE, accelerate=acc)
            s.primal_init()
            t0 = time.perf_counter()
            itp, rp = s.primal_iterate(mx, tol=tol, check_every=25, raise_notconv=False)
            tp = time.perf_counter() - t0
            J, Cd = s.objective()
            s.adjoint_init()
            t0 = time.perf_counter()
            ita, ra = s.adjoint_iterate(mx, tol=tol, check_every=25, raise_notconv=False)
            ta = time.perf_counter() - t0
            g = s.param_sensitivity(wl.grid.wall_jac)
            row[label] = {"primal_sweeps": itp, "primal_resid": rp, "primal_s": tp, "adjoint_sweeps": ita,
                          "adjoint_resid": ra, "adjoint_s": ta, "J": J, "Cd": Cd, "dJda": g.tolist()}
            print(f"[accel] Kn {Kn:g} {label}: primal {itp} sweeps r {rp:.1e} ({tp:.1f} s), adjoint {ita} sweeps "
                  f"r {ra:.1e} ({ta:.1f} s), C_d {Cd:.8f}", file=sys.stderr, flush=True)
            del s
        a, b = row["accelerated"], row["plain"]
        row["J_rel_diff"] = abs(a["J"] - b["J"]) / abs(b["J"])
        row["dJda_rel_diff"] = float(np.max(np.abs(np.array(a["dJda"]) - np.array(b["dJda"]))) /
                                     np.max(np.abs(np.array(b["dJda"]))))
        rows.append(row)
    return {"every": every, "inner": inner, "tol": tol, "cap": cap, "plain_cap": plain_cap,
            "precision": precision_name, "rows": rows}


def stream_reference(nbytes_total):
    """Plain HIP streams (csrc/dvm_stream.hip) with the read/write mixes of
    the sweeps, moving `nbytes_total` bytes per launch: 1 read + 1 write
    (c = a: the primal), 2 reads + 1 write (c = a + b: the adjoint), and a
    pure write and a pure read stream; 16-byte loads per lane and
    non-temporal stores as in the sweeps.  GB/s of bytes moved, HIP events
    over 20 launches after 3 warm-ups, best over grid-stride launches of
    2048 to 16384 workgroups of 256 threads and a one-pass launch, with and
    without non-temporal stores."""
    import ctypes as C

    import torch

    from paper_2501_00923_amd import build as B

    lib = C.CDLL(B.STREAM_LIB)
    lib.dvm_stream_time.restype = C.c_int
    lib.dvm_stream_time.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_int,
                                    C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_float)]
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = {}
    for name, kind, narr in (("read1_write1", 0, 2), ("read2_write1", 1, 3), ("write_only", 2, 1),
                             ("read_only", 3, 1)):
        nb = (int(nbytes_total // narr) // 4096) * 4096
        a = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        b = torch.ones(nb // 4, dtype=torch.float32, device="cuda") if kind == 1 else a
        c = torch.empty(nb // 4, dtype=torch.float32, device="cuda") if kind != 3 else \
            torch.empty(16384, dtype=torch.float32, device="cuda")
        best = None
        for blocks in (2048, 4096, 8192, 16384, 0):
            for nt in (1, 0):
                if kind == 3 and (blocks == 0 or nt == 0):
                    continue
                ms = C.c_float()
                rc = lib.dvm_stream_time(kind, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                                         C.c_void_p(c.data_ptr()), nb, blocks, nt, 3, 20, st, C.byref(ms))
                if rc != 0:
                    raise RuntimeError(f"stream reference kernel failed ({rc})")
                gbs = nb * narr / (ms.value * 1e-3) / 1e9
                if best is None or gbs > best["GB_per_s"]:
                    best = {"GB_per_s": gbs, "bytes_per_launch": nb * narr,
                            "workgroups": blocks or "one pass", "nontemporal_stores": bool(nt)}
        out[name] = best
        del a, b, c
    torch.cuda.empty_cache()
    return out


def oracle_rates(wl, seconds, nthreads):
    """The oracle's primal and adjoint Jacobi sweeps timed apart, each for
    about seconds/2 (at least one sweep) from the free stream and from
    phi = 0: pairs/s of each phase, and the rate of a 1:1 mix of sweeps (the
    GPU step's mix), 2 / (1/r_primal + 1/r_adjoint)."""
    import oracle
    p = oracle.Problem.from_workload(wl, nthreads=nthreads)
    p.primal_init()
    pairs = p.nc * p.nv
    out = {}
    for phase in ("primal", "adjoint"):
        if phase == "adjoint":
            p.adjoint_init()
        step = p.primal_iterate if phase == "primal" else p.adjoint_iterate
        done = 0
        t0 = time.perf_counter()
        while True:
            step(1)
            done += 1
            if time.perf_counter() - t0 > seconds / 2:
                break
        t = time.perf_counter() - t0
        out[phase] = {"value": pairs * done / t, "sweeps": done, "seconds": t}
    rp, ra = out["primal"]["value"], out["adjoint"]["value"]
    out["mix_1to1"] = 2.0 / (1.0 / rp + 1.0 / ra)
    return out


def cpu_baseline(wl, seconds):
    nthreads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    many = oracle_rates(wl, seconds, nthreads)
    one = oracle_rates(wl, seconds / 2, 1)
    pairs = wl.grid.ni * wl.grid.nj * wl.vgrid.n1 * wl.vgrid.n2

    def phases(r, cores):
        return {"cores": cores,
                "primal": {"value": r["primal"]["value"], "sweeps": r["primal"]["sweeps"],
                           "seconds": r["primal"]["seconds"]},
                "adjoint": {"value": r["adjoint"]["value"], "sweeps": r["adjoint"]["sweeps"],
                            "seconds": r["adjoint"]["seconds"]},
                "mix_1to1": r["mix_1to1"]}
    return {"value": many["mix_1to1"], "unit": "cell-velocity updates/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{wl.name}: {many['primal']['sweeps']} primal and {many['adjoint']['sweeps']} adjoint "
                      f"Jacobi sweeps of the full grid ({pairs} pairs), each phase timed apart, FP64, OpenMP over "
                      f"cells; value = the 1:1 primal:adjoint sweep mix of the GPU step",
            "all_cores": phases(many, nthreads), "single_core": phases(one, 1)}


def deform_scale():
    """RBF mesh motion (Sec. 3.4, Step 2) on O-grids from 192 to 8192 wall
    nodes (the library's limit): set-up (host Cholesky of the RBF system)
    and one motion and one transpose, host-inclusive, averaged over 5 calls
    after 2 warm-up calls.  Kernel times come from a kernel trace of this
    mode."""
    import numpy as np
    import torch

    from paper_2501_00923_amd import dvm, inputs as I
    from paper_2501_00923_amd.shape import Deformer

    rows = []
    for ni, nj, R in ((192, 128, 2.0), (2048, 128, 2.0), (8192, 64, 0.5), (8192, 64, 1.5)):
        g = I.ogrid(ni, nj, r_outer=10.0)
        mesh = dvm.Mesh.from_grid(g)
        t = time.perf_counter()
        D = Deformer(mesh, R)
        t_setup = time.perf_counter() - t
        wall = g.nodes[0, :ni] + 1e-4
        gvec = np.ones((nj + 1, ni + 1, 2))
        for _ in range(2):
            D.apply(wall)
            D.chain(gvec)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            D.apply(wall)
        t_apply = (time.perf_counter() - t) / 5
        t = time.perf_counter()
        for _ in range(5):
            D.chain(gvec)
        t_chain = (time.perf_counter() - t) / 5
        row = {"wall_nodes": ni, "mesh_nodes": (ni + 1) * (nj + 1), "radius": R, "setup_s": t_setup,
               "apply_ms": t_apply * 1e3, "chain_ms": t_chain * 1e3}
        print(f"[deform] {row}", file=sys.stderr, flush=True)
        rows.append(row)
        D.close()
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sweeps", type=int, default=20, help="primal and adjoint sweeps per step")
    ap.add_argument("--cpu-seconds", type=float, default=16.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-second-order", action="store_true",
                    help="skip the second-order leg (Green-Gauss slopes, Venkatakrishnan limiter)")
    ap.add_argument("--correction-every", type=int, default=40,
                    help="second-order leg: sweeps between evaluations of the held correction")
    ap.add_argument("--serving-requests", type=int, default=512,
                    help="requests in the solve-server leg (0 skips it; the default is the full stream)")
    ap.add_argument("--serving-cap", type=int, default=1000, help="sweep cap per phase per request")
    ap.add_argument("--accel-check", action="store_true",
                    help="the 256x128 C-grid with 64x64 sinh velocities at Kn 1e-3 .. 10: solves to --accel-tol with "
                         "the macroscopic prediction against the plain iteration, and exit")
    ap.add_argument("--accel-every", type=int, default=5)
    ap.add_argument("--accel-inner", type=int, default=200)
    ap.add_argument("--accel-tol", type=float, default=1e-8)
    ap.add_argument("--accel-cap", type=int, default=20000)
    ap.add_argument("--accel-plain-cap", type=int, default=3000)
    ap.add_argument("--accel-kn", type=str, default="1e-3,1e-2,0.1,1,10")
    ap.add_argument("--accel-precision", choices=("fp64", "mixed"), default="fp64")
    ap.add_argument("--serving-accel-below-kn", type=float, default=1.0,
                    help="requests below this Kn use the conservative equilibrium and the macroscopic prediction "
                         "(0: none)")
    ap.add_argument("--serving-accel-inner", type=int, default=75)
    ap.add_argument("--workload", choices=("c2", "c3"), default="c2",
                    help="the timed workload: c2 (the benchmark's: 48x48 Newton-Cotes velocities, Kn 0.1, Ma 0.8) "
                         "or c3 (64x64 sinh velocities, Kn 0.1, Ma 0.5) on the 256x128 NACA0012 C-grid; c3 is for "
                         "its counter runs")
    ap.add_argument("--no-c1", action="store_true",
                    help="skip the whole-solve latency of the circle O-grid 64x32 with 16x16 velocities")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the 256x128 C-grid with 64x64 sinh velocities (134 M pairs) leg")
    ap.add_argument("--batch-members", type=int, default=24,
                    help="requests of the serving stream in the batched-sweep roofline (0 skips it)")
    ap.add_argument("--serving-tol", type=float, default=1e-5)
    ap.add_argument("--serving-seed", type=int, default=0)
    ap.add_argument("--precision-sweep", action="store_true",
                    help="print the per-Kn mixed-vs-FP64 error table (256x128 C-grid, 64x64 sinh grid) and exit")
    ap.add_argument("--precision-sweeps", type=int, default=2000)
    ap.add_argument("--precision-order", type=int, default=1, choices=(1, 2),
                    help="spatial order of the scheme the --precision-sweep runs")
    ap.add_argument("--fd-check", action="store_true",
                    help="print the adjoint-vs-central-difference table of the 24-parameter B-spline NACA case and exit")
    ap.add_argument("--fd-h", type=float, default=1e-6)
    ap.add_argument("--fd-tol", type=float, default=1e-12)
    ap.add_argument("--fd-no-limiter", action="store_true",
                    help="second-order fd check without the limiter (the exact form is then exact)")
    ap.add_argument("--fd-order", type=int, default=1, choices=(1, 2),
                    help="spatial order of the scheme the --fd-check runs")
    ap.add_argument("--optimize", action="store_true",
                    help="run the shape-optimisation loop (CST, RBF mesh motion, SLSQP) instead of the bench")
    ap.add_argument("--opt-grid", type=str, default="16,48,64", help="n_wake,n_half,nj of the NACA0012 C-grid")
    ap.add_argument("--opt-nv", type=int, default=32)
    ap.add_argument("--opt-kn", type=float, default=1.0)
    ap.add_argument("--opt-ma", type=float, default=0.5)
    ap.add_argument("--opt-steps", type=int, default=20)
    ap.add_argument("--opt-gradient", choices=("paper", "exact"), default="paper")
    ap.add_argument("--opt-tol", type=float, default=1e-9)
    ap.add_argument("--opt-radius", type=float, default=2.0)
    ap.add_argument("--opt-sigma", type=float, default=0.1)
    ap.add_argument("--opt-max-sweeps", type=int, default=200000, help="sweep cap per solve")
    ap.add_argument("--opt-mixed", action="store_true", help="FP32 f and phi (FP64 moments, J, sensitivities)")
    ap.add_argument("--opt-no-limiter", action="store_true", help="second order without the limiter")
    ap.add_argument("--opt-adjoint-tol", type=float, default=None, help="adjoint solve tolerance (default: --opt-tol)")
    ap.add_argument("--cst-fd-check", action="store_true",
                    help="drag sensitivity to the CST variables (adjoint, both forms) vs central differences, "
                         "on the --opt-grid / --opt-nv / --opt-kn / --opt-ma case")
    ap.add_argument("--deform-scale", action="store_true",
                    help="RBF mesh motion timings on O-grids from 192 to 8192 wall nodes")
    ap.add_argument("--cst-fd-h", type=float, default=1e-4)
    ap.add_argument("--cst-fd-tol", type=float, default=1e-13)
    ap.add_argument("--opt-order", type=int, default=1, choices=(1, 2),
                    help="spatial order of the flow solves (2: Venkatakrishnan limiter, correction every 40 sweeps)")
    ap.add_argument("--no-optimize-leg", action="store_true",
                    help="skip the short shape optimisation (128x64 C-grid) of the default run")
    ap.add_argument("--no-stream-reference", action="store_true",
                    help="skip the streaming reference (its own copy and fill would sit beside a calibration copy)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (a kernel of known traffic "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: the solver runs on one GPU only (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE {world}); independent solves would shard one per GPU with no exchange.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2501_00923_amd import dvm
    from paper_2501_00923_amd import inputs as I

    torch.cuda.set_device(0)
    dvm.lib()
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {n} bytes read + {n} bytes written", file=sys.stderr, flush=True)
        del src, dst
    if args.precision_sweep:
        rows = precision_sweep(args.precision_sweeps, [1e-3, 1e-2, 0.1, 1.0, 10.0], order=args.precision_order)
        print(json.dumps({"precision_sweep": rows}))
        return
    if args.fd_check:
        print(json.dumps({"fd_check": fd_check(args.fd_h, args.fd_tol, order=args.fd_order,
                                               limiter=not args.fd_no_limiter)}))
        return
    if args.accel_check:
        kns = [float(x) for x in args.accel_kn.split(",")]
        print(json.dumps({"accel_check": accel_check(kns, args.accel_every, args.accel_inner, args.accel_cap,
                                                     args.accel_tol, args.accel_plain_cap, args.accel_precision)}))
        return
    if args.deform_scale:
        print(json.dumps({"deform_scale": deform_scale()}))
        return
    if args.cst_fd_check:
        nw_, nh_, nj_ = (int(x) for x in args.opt_grid.split(","))
        print(json.dumps({"cst_fd_check": cst_fd_check(nw_, nh_, nj_, args.opt_nv, args.opt_kn, args.opt_ma,
                                                       args.cst_fd_h, args.cst_fd_tol, args.opt_radius,
                                                       order=args.opt_order, limiter=not args.opt_no_limiter,
                                                       max_sweeps=args.opt_max_sweeps)}))
        return
    if args.optimize:
        nw_, nh_, nj_ = (int(x) for x in args.opt_grid.split(","))
        print(json.dumps({"optimize": optimize_leg(nw_, nh_, nj_, args.opt_nv, args.opt_kn, args.opt_ma,
                                                   args.opt_steps, args.opt_gradient, args.opt_tol,
                                                   args.opt_radius, args.opt_sigma, order=args.opt_order,
                                                   max_sweeps=args.opt_max_sweeps, mixed=args.opt_mixed,
                                                   adjoint_tol=args.opt_adjoint_tol)}))
        return
    wl = I.c2_naca(seed=0) if args.workload == "c2" else I.c3_naca_sinh(0.1)
    print(f"[bench] {wl.name}: FP64 steps={args.steps} warmup={args.warmup} sweeps={args.sweeps}",
          file=sys.stderr, flush=True)
    r64 = run_gpu(wl, dvm.FP64, args.sweeps, args.steps, args.warmup)
    print(f"[bench] fp64 {r64['updates_per_s']:.3e} upd/s, primal {r64['primal_sweep_ms']:.3f} ms, "
          f"adjoint {r64['adjoint_sweep_ms']:.3f} ms", file=sys.stderr, flush=True)
    mixed = None
    if not args.no_mixed:
        rm = run_gpu(wl, dvm.MIXED, args.sweeps, args.steps, args.warmup)
        mixed = {"value": rm["updates_per_s"], "ms_per_step": rm["ms_per_step"],
                 "speedup_vs_fp64": rm["updates_per_s"] / r64["updates_per_s"],
                 "primal_sweep_ms": rm["primal_sweep_ms"], "adjoint_sweep_ms": rm["adjoint_sweep_ms"],
                 "J_rel_err_vs_fp64": abs(rm["J"] - r64["J"]) / abs(r64["J"]),
                 "dtype": "f32 state / f64 moments"}
        print(f"[bench] mixed {rm['updates_per_s']:.3e} upd/s", file=sys.stderr, flush=True)

    pairs = r64["pairs"]
    t_adj = r64["adjoint_sweep_ms"] * 1e-3
    t_pri = r64["primal_sweep_ms"] * 1e-3
    b_adj = bytes_per_update("adjoint", False) * pairs
    b_pri = bytes_per_update("primal", False) * pairs
    achieved = b_adj / t_adj / 1e9
    tr = load_traffic(args.workload)
    traffic = tr.get("adjoint_fp64_bytes_per_launch")
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "k_adjoint_sweep<double>",
            "algorithmic_bytes_per_launch": b_adj,
            "avg_launch_ms": r64["adjoint_sweep_ms"],
            "primal": {"kernel": "k_primal_sweep<double>", "achieved": b_pri / t_pri / 1e9,
                       "frac": b_pri / t_pri / 1e9 / HBM_PEAK_GBS, "avg_launch_ms": r64["primal_sweep_ms"],
                       "algorithmic_bytes_per_launch": b_pri,
                       "traffic": tr.get("primal_fp64_bytes_per_launch")}}
    # what a plain streaming kernel reaches with the same read/write mix
    sref = None if args.no_stream_reference else stream_reference(b_adj)
    if sref is not None:
        roof["stream_reference"] = sref
        roof["frac_of_stream_reference"] = achieved / sref["read2_write1"]["GB_per_s"]
        roof["primal"]["frac_of_stream_reference"] = roof["primal"]["achieved"] / sref["read1_write1"]["GB_per_s"]
        print(f"[bench] stream reference: 2R1W {sref['read2_write1']['GB_per_s']:.0f} GB/s, "
              f"1R1W {sref['read1_write1']['GB_per_s']:.0f} GB/s", file=sys.stderr, flush=True)
    if mixed is not None:
        for kind, key in (("adjoint", "adjoint_sweep_ms"), ("primal", "primal_sweep_ms")):
            b = bytes_per_update(kind, True) * pairs
            t = mixed[key] * 1e-3
            roof[f"{kind}_mixed"] = {"kernel": f"k_{kind}_sweep<float>", "achieved": b / t / 1e9,
                                     "frac": b / t / 1e9 / HBM_PEAK_GBS, "avg_launch_ms": mixed[key],
                                     "algorithmic_bytes_per_launch": b,
                                     "traffic": tr.get(f"{kind}_mixed_bytes_per_launch")}
            if sref is not None:
                ref = sref["read2_write1" if kind == "adjoint" else "read1_write1"]["GB_per_s"]
                roof[f"{kind}_mixed"]["frac_of_stream_reference"] = b / t / 1e9 / ref
    second = None
    if not args.no_second_order:
        K = args.correction_every
        r2 = run_gpu(wl, dvm.FP64, args.sweeps, args.steps, args.warmup, order=2, correction_every=K)
        second = {"value": r2["updates_per_s"], "ms_per_step": r2["ms_per_step"], "dtype": "f64",
                  "limiter": "venkatakrishnan", "correction_every": K,
                  "vs_first_order": r2["updates_per_s"] / r64["updates_per_s"],
                  "J": r2["J"], "J_rel_diff_vs_first_order": abs(r2["J"] - r64["J"]) / abs(r64["J"]),
                  "roofline": {}}
        counted = tr.get("order2_bytes_per_launch", {})   # per kernel, from the counter runs
        kernels = {"primal": ("k_primal_sweep<double, true>", "k_so_slope<double, false>", "k_so_corr<double>"),
                   "adjoint": ("k_adjoint_sweep<double, true>", "k_so_adj_b<double>", "k_so_adj_e<double>")}
        cps = -(-args.sweeps // K) / args.sweeps     # corrections per sweep in a step from init
        second["corrections_per_sweep"] = cps
        for kind in ("primal", "adjoint"):
            t = r2[f"{kind}_sweep_ms"] * 1e-3
            bb = so_bytes_per_update(kind, False, cps)
            ks = kernels[kind]
            tb = [v for name in ks for k_, v in counted.items() if name in k_]
            second["roofline"][kind] = {
                "avg_sweep_ms": r2[f"{kind}_sweep_ms"],
                "note": "sweep plus its share of the correction kernels",
                "kernels": list(ks),
                "bytes_per_update": bb, "achieved": bb["per_sweep"] * pairs / t / 1e9,
                "frac": bb["per_sweep"] * pairs / t / 1e9 / HBM_PEAK_GBS,
                "traffic_per_sweep": (tb[0] + (tb[1] + tb[2]) * cps) if len(tb) == 3 else None}
        print(f"[bench] second order {r2['updates_per_s']:.3e} upd/s, primal {r2['primal_sweep_ms']:.3f} ms, "
              f"adjoint {r2['adjoint_sweep_ms']:.3f} ms per sweep", file=sys.stderr, flush=True)
        if not args.no_mixed:
            r2m = run_gpu(wl, dvm.MIXED, args.sweeps, args.steps, args.warmup, order=2, correction_every=K)
            second["mixed"] = {"value": r2m["updates_per_s"], "ms_per_step": r2m["ms_per_step"],
                               "speedup_vs_fp64": r2m["updates_per_s"] / r2["updates_per_s"],
                               "primal_sweep_ms": r2m["primal_sweep_ms"], "adjoint_sweep_ms": r2m["adjoint_sweep_ms"],
                               "J_rel_err_vs_fp64": abs(r2m["J"] - r2["J"]) / abs(r2["J"]),
                               "dtype": "f32 state / f64 moments and limiter"}
            print(f"[bench] second order mixed {r2m['updates_per_s']:.3e} upd/s", file=sys.stderr, flush=True)
    c3 = None
    if not args.no_c3 and args.workload == "c2":
        wl3 = I.c3_naca_sinh(0.1)
        tr3 = load_traffic("c3")
        print(f"[bench] {wl3.name}: FP64 and mixed", file=sys.stderr, flush=True)
        r3 = run_gpu(wl3, dvm.FP64, args.sweeps, max(2, args.steps // 2), args.warmup)
        r3m = run_gpu(wl3, dvm.MIXED, args.sweeps, max(2, args.steps // 2), args.warmup)
        p3 = r3["pairs"]
        c3 = {"workload": wl3.name, "cells": wl3.grid.ni * wl3.grid.nj, "velocities": wl3.vgrid.n1 * wl3.vgrid.n2,
              "pairs": p3, "fp64": {"value": r3["updates_per_s"], "ms_per_step": r3["ms_per_step"]},
              "mixed": {"value": r3m["updates_per_s"], "ms_per_step": r3m["ms_per_step"],
                        "J_rel_err_vs_fp64": abs(r3m["J"] - r3["J"]) / abs(r3["J"])}, "roofline": {}}
        for prec, rr, mixed_ in (("fp64", r3, False), ("mixed", r3m, True)):
            for kind in ("primal", "adjoint"):
                t = rr[f"{kind}_sweep_ms"] * 1e-3
                bb = bytes_per_update(kind, mixed_) * p3
                c3["roofline"][f"{kind}_{prec}"] = {
                    "kernel": f"k_{kind}_sweep<{'float' if mixed_ else 'double'}>", "avg_launch_ms": t * 1e3,
                    "algorithmic_bytes_per_launch": bb, "achieved": bb / t / 1e9, "frac": bb / t / 1e9 / HBM_PEAK_GBS,
                    "traffic": tr3.get(f"{kind}_{prec}_bytes_per_launch")}
        print(f"[bench] C3 fp64 {r3['updates_per_s']:.3e} upd/s, mixed {r3m['updates_per_s']:.3e} upd/s",
              file=sys.stderr, flush=True)
    c1 = None
    if not args.no_c1:
        c1 = c1_leg()
        print(f"[bench] C1 whole solve: {c1['primal_sweeps']} + {c1['adjoint_sweeps']} sweeps, "
              f"{c1['solve_ms_median']:.1f} ms (median of {c1['repeats']})", file=sys.stderr, flush=True)
    batch_roof = None
    if args.batch_members > 0:
        batch_roof = batch_roofline(args.batch_members, args.serving_seed)
    serving = None
    if args.serving_requests > 0:
        print(f"[bench] serving leg: {args.serving_requests} requests", file=sys.stderr, flush=True)
        serving = serving_leg(args.serving_requests, args.serving_seed, args.serving_cap, args.serving_tol,
                              64.0, 20, None if args.serving_accel_below_kn <= 0 else args.serving_accel_below_kn,
                              (args.accel_every, args.serving_accel_inner))
    optimization = None
    if not args.no_optimize_leg:
        # a whole optimisation (Sec. 3.4) on a 128x64 NACA0012 C-grid, 32x32 velocities, Kn 1, Ma 0.5
        print("[bench] optimisation leg", file=sys.stderr, flush=True)
        o = optimize_leg(16, 48, 64, 32, 1.0, 0.5, 20, "paper", 1e-9, 2.0, 0.1)
        optimization = {k: o[k] for k in ("workload", "gradient", "steps", "stop", "evaluations", "gradients",
                                          "unconverged_solves", "seconds", "sweeps", "stage_seconds",
                                          "deform_apply_ms", "deform_chain_ms")}
        optimization["Cd_initial"], optimization["Cd_final"] = o["Cd"][0], o["Cd"][-1]
        optimization["drag_change"] = o["drag_change"]
        optimization["Q_over_vmin_final"] = o["Q_over_vmin"][-1]
        optimization["paper_context"] = ("a full optimisation in 5-20 minutes on 40-160 CPU cores "
                                         "(the paper's channel and supersonic airfoil cases, Sec. 4)")
    cpu = None
    if not args.no_cpu_baseline:
        print(f"[bench] oracle on the host cores (~{args.cpu_seconds:.0f} s)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(wl, args.cpu_seconds)
    line = {
        "metric": "cell-velocity updates/s (primal+adjoint) vs plain FP64 path; p50/p99 solve ms",
        "value": r64["updates_per_s"], "unit": "cell-velocity updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded NACA0012 C-grid and Hicks-Henne bump positions)",
        "config": {"workload": wl.name, "cells": wl.grid.ni * wl.grid.nj, "velocities": wl.vgrid.n1 * wl.vgrid.n2,
                   "pairs": pairs,
                   "sweeps_per_step": {"primal": args.sweeps, "adjoint": args.sweeps},
                   "Kn": wl.flow.Kn, "Ma": wl.flow.Ma, "shape_params": int(wl.grid.wall_jac.shape[-1]),
                   "parallelism": "single GPU"},
        "roofline": roof, "cpu_baseline": cpu, "mixed": mixed, "c3": c3, "c1": c1, "batched_sweep_roofline": batch_roof,
        "second_order": second, "serving": serving,
        "optimization": optimization, "J": r64["J"], "Cd": r64["Cd"],
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
