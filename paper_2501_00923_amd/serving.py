"""Continuous batching of independent primal/adjoint solves on one GPU.

Requests (a shape, mesh and velocity-grid size, Kn, Ma, and whether the
adjoint sensitivities are wanted) arrive over time.  The server admits a
pending request as soon as its exact device footprint fits the memory
budget, keeps every admitted solve's state resident, and advances all
resident solves together: each sweep is two kernel launches, one over the
cells of every primal-phase solve and one over every adjoint-phase solve.
Requests are admitted in arrival order, except that a request that does not
fit yet lets later, smaller ones pass (it waits for memory to free).  Every
``q`` sweeps it reads the residuals; a converged (or capped) primal either
switches to its adjoint phase or finishes, a finished solve reads out J
(and dJ/dalpha), frees its memory, and the freed memory admits waiting
requests before the next launch.  Latency = finish time - arrival time.

The scheduler talks to a ``Backend``; ``GpuBackend`` runs libdvm batches,
``FakeBackend`` (CPU, synthetic convergence) exercises the policy in tests.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np


@dataclass
class SolveResult:
    rid: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    J: float = float("nan")
    Cd: float = float("nan")
    dJ: Optional[np.ndarray] = None
    primal_iters: int = 0
    adjoint_iters: int = 0
    primal_resid: float = float("nan")
    adjoint_resid: float = float("nan")
    status: str = "pending"      # pending, ok, notconv, failed
    error: str = ""

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class ServeConfig:
    memory_budget: int                   # device bytes for solver workspaces
    sweeps_per_check: int = 20           # q: sweeps between residual reads
    tol: float = 1e-5                    # primal residual target
    adjoint_tol: float = 1e-5
    max_iter: int = 4000                 # per phase
    max_resident: int = 64


class Backend:
    """What the scheduler needs from a solver implementation."""

    def footprint(self, req) -> int: ...
    def create(self, req): ...
    def release(self, h) -> None: ...
    def advance(self, handles: List, sweeps: int) -> None: ...
    def residuals(self, handles: List) -> np.ndarray: ...
    def start_adjoint(self, h) -> None: ...
    def finish(self, h, req, res: SolveResult) -> None: ...
    def sync(self) -> None: ...


class _Slot:
    __slots__ = ("req", "h", "res", "phase", "iters")

    def __init__(self, req, h, res):
        self.req, self.h, self.res = req, h, res
        self.phase = 0
        self.iters = 0


def serve(requests: List, backend: Backend, cfg: ServeConfig, clock=time.perf_counter,
          realtime: bool = True, sleep=time.sleep, on_finish=None) -> Dict:
    """Run the request stream to completion.  ``requests`` carry ``rid``,
    ``arrival`` (s after start) and ``want_adjoint``.  With realtime=False
    all requests are available at once (closed loop, capacity).
    on_finish(result, n_finished) is called as each request leaves."""
    order = sorted(requests, key=lambda r: r.arrival)
    results = {r.rid: SolveResult(r.rid, r.arrival if realtime else 0.0) for r in order}
    pending: List = []
    nxt = 0
    active: List[_Slot] = []
    used = 0
    t0 = clock()
    launches = 0
    peak_used = 0
    peak_resident = 0
    n_finished = 0

    def now():
        return clock() - t0

    while nxt < len(order) or pending or active:
        t = now()
        while nxt < len(order) and (not realtime or order[nxt].arrival <= t):
            pending.append(order[nxt])
            nxt += 1
        # admission by exact footprint, arrival order; a request larger than
        # the whole budget fails instead of blocking the queue
        still = []
        for req in pending:
            fp = backend.footprint(req)
            if fp > cfg.memory_budget:
                res = results[req.rid]
                res.status, res.error, res.finished = "failed", "footprint exceeds budget", now()
                n_finished += 1
                if on_finish is not None:
                    on_finish(res, n_finished)
                continue
            if used + fp <= cfg.memory_budget and len(active) < cfg.max_resident:
                try:
                    h = backend.create(req)
                except Exception as e:       # allocation or setup failure: fail this request only
                    res = results[req.rid]
                    res.status, res.error, res.finished = "failed", str(e), now()
                    n_finished += 1
                    if on_finish is not None:
                        on_finish(res, n_finished)
                    continue
                used += fp
                res = results[req.rid]
                res.admitted = now()
                active.append(_Slot(req, h, res))
            else:
                still.append(req)
        pending = still
        peak_used = max(peak_used, used)
        peak_resident = max(peak_resident, len(active))
        if not active:
            if nxt < len(order) and realtime:
                wait = order[nxt].arrival - now()
                if wait > 0:
                    sleep(min(wait, 0.01))
            continue
        handles = [s.h for s in active]
        backend.advance(handles, cfg.sweeps_per_check)
        launches += cfg.sweeps_per_check
        r = backend.residuals(handles)
        keep = []
        for slot, ri in zip(active, r):
            slot.iters += cfg.sweeps_per_check
            done = False
            if not math.isfinite(ri):
                slot.res.status, slot.res.error = "failed", "non-finite residual"
                done = True
            elif slot.phase == 0:
                slot.res.primal_resid = ri
                slot.res.primal_iters = slot.iters
                if ri < cfg.tol or slot.iters >= cfg.max_iter:
                    if ri >= cfg.tol:
                        slot.res.status = "notconv"
                    if slot.req.want_adjoint:
                        backend.start_adjoint(slot.h)
                        slot.phase, slot.iters = 1, 0
                    else:
                        done = True
            else:
                slot.res.adjoint_resid = ri
                slot.res.adjoint_iters = slot.iters
                if ri < cfg.adjoint_tol or slot.iters >= cfg.max_iter:
                    if ri >= cfg.adjoint_tol:
                        slot.res.status = "notconv"
                    done = True
            if done:
                if slot.res.status != "failed":
                    backend.finish(slot.h, slot.req, slot.res)
                    if slot.res.status == "pending":
                        slot.res.status = "ok"
                slot.res.finished = now()
                backend.release(slot.h)
                used -= backend.footprint(slot.req)
                n_finished += 1
                if on_finish is not None:
                    on_finish(slot.res, n_finished)
            else:
                keep.append(slot)
        active = keep
    backend.sync()
    wall = now()
    res = [results[r.rid] for r in order]

    def latency_stats(keep):
        lat = np.array([x.latency for x in res if keep(x)]) * 1e3
        return {"count": int(len(lat)),
                "solves_per_s": len(lat) / wall if wall > 0 else float("nan"),
                "p50_ms": float(np.percentile(lat, 50)) if len(lat) else float("nan"),
                "p99_ms": float(np.percentile(lat, 99)) if len(lat) else float("nan"),
                "mean_ms": float(lat.mean()) if len(lat) else float("nan")}

    finished = latency_stats(lambda x: x.status in ("ok", "notconv"))
    return {
        "results": res,
        "wall_s": wall,
        # every finished solve (converged or stopped at the sweep cap)
        "solves_per_s": finished["solves_per_s"],
        "p50_ms": finished["p50_ms"],
        "p99_ms": finished["p99_ms"],
        "mean_ms": finished["mean_ms"],
        "completed": finished["count"],
        # the solves that reached their tolerances, and those stopped at the cap
        "converged": latency_stats(lambda x: x.status == "ok"),
        "capped": latency_stats(lambda x: x.status == "notconv"),
        "capped_by_kn": capped_by_kn(order, res),
        "failed": sum(1 for x in res if x.status == "failed"),
        "notconv": sum(1 for x in res if x.status == "notconv"),
        "sweep_launches": launches,
        "peak_bytes": peak_used,
        "peak_resident": peak_resident,
    }


KN_DECADES = ((1e-3, 1e-2), (1e-2, 1e-1), (1e-1, 1.0), (1.0, 10.0 + 1e-9))


def capped_by_kn(requests: List, results: List[SolveResult]) -> Dict:
    """Requests and sweep-capped solves per decade of Kn (requests that carry
    a workload with a flow state; others are not counted)."""
    out = {}
    for lo, hi in KN_DECADES:
        n = capped = 0
        for req, r in zip(requests, results):
            kn = getattr(getattr(getattr(req, "workload", None), "flow", None), "Kn", None)
            if kn is None or not (lo <= kn < hi):
                continue
            n += 1
            capped += r.status == "notconv"
        out[f"[{lo:g},{min(hi, 10.0):g}]"] = {"requests": n, "capped": capped}
    return out


def serve_one_at_a_time(requests: List, backend: Backend, cfg: ServeConfig, clock=time.perf_counter,
                        realtime: bool = True, sleep=time.sleep, on_finish=None) -> Dict:
    """Baseline: one solve at a time in arrival order, each alone on the GPU."""
    big = ServeConfig(memory_budget=cfg.memory_budget, sweeps_per_check=cfg.sweeps_per_check, tol=cfg.tol,
                      adjoint_tol=cfg.adjoint_tol, max_iter=cfg.max_iter, max_resident=1)
    return serve(requests, backend, big, clock, realtime, sleep, on_finish)


# ---------------------------------------------------------------------------
# backends
# ---------------------------------------------------------------------------

class GpuBackend(Backend):
    """libdvm solvers on one GPU; all resident solves of one precision are
    advanced by one batch (rebuilt whenever the resident set or a phase
    changes)."""

    def __init__(self, precision, stream=None, shape_params: bool = True, accelerate_below_kn=None,
                 accelerate=(5, 75)):
        """accelerate_below_kn: requests below this Kn (first order) solve
        with the conservative equilibrium and the macroscopic prediction
        `accelerate` = (every, inner) of both phases; None: never."""
        import torch

        from . import dvm
        self.dvm, self.torch = dvm, torch
        self.precision = precision
        self.accelerate_below_kn = accelerate_below_kn
        self.accelerate = tuple(accelerate)
        self.shape_params = shape_params
        self.stream = stream
        self._batch = None
        self._key = None
        self._fp_cache: Dict = {}

    def _options(self, req):
        """Solver options of a request: second-order requests as asked; below
        the Kn threshold (first order), the conservative equilibrium and the
        macroscopic prediction."""
        order = getattr(req, "order", 1)
        if (self.accelerate_below_kn is not None and order == 1 and req.workload.flow.Kn < self.accelerate_below_kn):
            return dict(order=order, equilibrium=self.dvm.EQ_CONSERVATIVE, accelerate=self.accelerate)
        return dict(order=order)

    def footprint(self, req) -> int:
        key = req.rid
        if key not in self._fp_cache:
            wl = req.workload
            s = self.dvm.Solver(self.dvm.Mesh.from_grid(wl.grid), self.dvm.VGrid.from_spec(wl.vgrid), wl.flow.Kn,
                                wl.flow.Ma, wl.flow.Tw, wl.flow.objective, self.precision, req.want_adjoint,
                                bind=False, **self._options(req))
            self._fp_cache[key] = s.workspace_bytes
        return self._fp_cache[key]

    def create(self, req):
        wl = req.workload
        s = self.dvm.Solver(self.dvm.Mesh.from_grid(wl.grid), self.dvm.VGrid.from_spec(wl.vgrid), wl.flow.Kn,
                            wl.flow.Ma, wl.flow.Tw, wl.flow.objective, self.precision, req.want_adjoint,
                            stream=self.stream, **self._options(req))
        s.primal_init()
        return s

    def release(self, h) -> None:
        self._drop_batch()
        h.buffer = None

    def _drop_batch(self):
        if self._batch is not None:
            self._batch.close()
            self._batch = None
            self._key = None

    def advance(self, handles, sweeps):
        key = tuple((id(h), h.phase) for h in handles)
        if key != self._key:
            self._drop_batch()
            self._batch = self.dvm.Batch(handles, stream=self.stream)
            self._key = key
        self._batch.run(sweeps)

    def residuals(self, handles):
        return self._batch.residuals()

    def start_adjoint(self, h):
        self._drop_batch()
        h.adjoint_init()

    def finish(self, h, req, res):
        self._drop_batch()
        res.J, res.Cd = h.objective()
        if req.want_adjoint and self.shape_params:
            res.dJ = h.param_sensitivity(req.workload.grid.wall_jac)

    def sync(self):
        self._drop_batch()
        self.torch.cuda.synchronize()


class FakeBackend(Backend):
    """CPU stand-in: each solve's residual decays geometrically at a
    per-request rate; a sweep costs ``cost_per_pair`` seconds per (cell,
    velocity) pair of the batch (advanced on a virtual clock).  Requests
    whose workload name contains 'nan' produce a non-finite residual."""

    def __init__(self, cost_per_pair: float = 1e-12, fail_create=()):
        self.t = 0.0
        self.cost = cost_per_pair
        self.fail_create = set(fail_create)
        self.live = set()
        self.max_live_bytes = 0
        self.live_bytes = 0
        self.batches: List[int] = []

    def clock(self):
        return self.t

    def sleep(self, dt):
        self.t += dt

    def footprint(self, req) -> int:
        g = req.workload.grid
        return int(g.ni * g.nj * req.workload.vgrid.n1 * req.workload.vgrid.n2 * 16 * (4 if req.want_adjoint else 2))

    def create(self, req):
        if req.rid in self.fail_create:
            raise MemoryError("injected allocation failure")
        h = {"req": req, "r": 1.0, "phase": 0,
             "rate": 0.5 + 0.45 * ((req.rid * 7919) % 100) / 100.0}
        self.live.add(id(h))
        self.live_bytes += self.footprint(req)
        self.max_live_bytes = max(self.max_live_bytes, self.live_bytes)
        return h

    def release(self, h):
        self.live.discard(id(h))
        self.live_bytes -= self.footprint(h["req"])

    def advance(self, handles, sweeps):
        pairs = 0
        for h in handles:
            g = h["req"].workload.grid
            pairs += g.ni * g.nj * h["req"].workload.vgrid.n1 * h["req"].workload.vgrid.n2
            h["r"] *= h["rate"] ** sweeps
            if "nan" in h["req"].workload.name:
                h["r"] = float("nan")
        self.batches.append(len(handles))
        self.t += pairs * sweeps * self.cost + 1e-5

    def residuals(self, handles):
        return np.array([h["r"] for h in handles])

    def start_adjoint(self, h):
        h["phase"] = 1
        h["r"] = 1.0

    def finish(self, h, req, res):
        res.J = float(req.rid)

    def sync(self):
        pass
