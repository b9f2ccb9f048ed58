"""Gradient-based airfoil shape optimisation on libdvm (Sec. 3.4, Steps 1-6).

  Step 1  CST design fitted to the initial wall nodes (eq. cstini)
  Step 2  wall nodes from the design, bulk mesh by Wendland-C0 RBF motion
  Step 3  primal and adjoint solves; J (eq. numer_J) and Q (eq. formula_opt)
  Step 4  dJ/dalpha through the wall-node sensitivity (eq. sens_nod, the
          paper's form) or the exact discrete mesh sensitivity chained
          through the RBF motion (second order: limiter factors held
          fixed); dQ/dalpha by eq. (sens_con_nod)
  Step 5  SLSQP update (scipy's implementation of Kraft's algorithm, the one
          the paper uses through NLopt) under the bounds of eq.
          (cst_constraint) and Q <= 0
  Step 6  stop when |J_new - J_old| / |J_old| < 3e-5 (eq. criterion_opt)

Every flow solve, sensitivity, CST evaluation, constraint and mesh motion
runs in libdvm; this module orders the calls and hands the numbers to the
optimiser.  The optimiser works on the free design variables divided by
`sigma` and on J / J_0 (its first quasi-Newton step is the scaled gradient).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import dvm
from .shape import Deformer, cst_eval, cst_fit, n_params, volume_constraint


def airfoil_wall(grid):
    """Wall nodes of a C-grid airfoil with its leading edge at (0, 0) and
    trailing edge at (1, 0): positions, chord stations xi = x, and the upper
    flag (nodes after the leading edge in wall order)."""
    if grid.topology != dvm.TOPO_C:
        raise ValueError("the CST parameterisation needs a C-grid airfoil")
    nw = grid.ni - 2 * grid.n_wake
    wall = np.array(grid.nodes[0, grid.n_wake:grid.n_wake + nw], dtype=np.float64)
    le = int(np.argmin(wall[:, 0]))
    if abs(wall[le, 0]) > 1e-12 or abs(wall[0, 0] - 1.0) > 1e-12 or abs(wall[0, 1]) > 1e-12:
        raise ValueError("airfoil must have its leading edge at x = 0 and trailing edge at (1, 0)")
    return wall, wall[:, 0].copy(), np.arange(nw) > le


def cst_bounds(nb: int):
    """Bounds of eq. (cst_constraint): N1, N2 >= 0.01, A_u >= 0, A_l <= 0,
    trailing-edge offsets fixed at 0 (sharp trailing edge)."""
    lo = np.full(n_params(nb), -np.inf)
    hi = np.full(n_params(nb), np.inf)
    lo[:2] = 0.01
    lo[2:nb + 3] = 0.0
    hi[nb + 3:2 * nb + 4] = 0.0
    lo[2 * nb + 4:] = 0.0
    hi[2 * nb + 4:] = 0.0
    return lo, hi


@dataclass
class Evaluation:
    alpha: np.ndarray
    J: float
    Cd: float
    Q: float
    dQ: np.ndarray
    dJ: Optional[np.ndarray] = None
    primal: tuple = (0, 0.0)          # (sweeps, last residual)
    adjoint: tuple = (0, 0.0)
    seconds: float = 0.0
    times: dict = field(default_factory=dict)      # seconds per stage: deform, setup, primal, adjoint, sens
    solver: object = field(default=None, repr=False)
    deta: object = field(default=None, repr=False)     # d eta / d alpha at the wall stations


class _Stop(Exception):
    pass


class ShapeOptimizer:
    def __init__(self, wl, nb: int = 6, radius: float = 2.0, sigma: float = 0.1, gradient: str = "paper",
                 precision: int = dvm.FP64, order: int = 1, limiter: int = dvm.LIMITER_VENKAT,
                 solve_tol: float = 1e-10, adjoint_tol: Optional[float] = None,
                 max_sweeps: int = 200000, check_every: int = 50, warm_start: bool = True, progress=None):
        if gradient not in ("paper", "exact"):
            raise ValueError("gradient is 'paper' (wall nodes, eq. sens_nod) or 'exact' (mesh sensitivity)")
        self.wl, self.nb, self.sigma, self.gradient = wl, nb, float(sigma), gradient
        self.precision, self.order, self.limiter = precision, order, limiter
        self.solve_tol, self.max_sweeps, self.check_every = solve_tol, max_sweeps, check_every
        # the gradient only steers the optimiser: its solve may stop earlier
        self.adjoint_tol = solve_tol if adjoint_tol is None else adjoint_tol
        self.warm_start = warm_start
        self.progress = progress       # called with a line of text after each solve
        g = wl.grid
        self.grid = g
        self.wall0, self.xi, self.upper = airfoil_wall(g)
        self.vgrid = dvm.VGrid.from_spec(wl.vgrid)
        self.mesh0 = dvm.Mesh.from_grid(g)
        self.deform = Deformer(self.mesh0, radius)
        self.alpha0, self.fit_rms = cst_fit(nb, self.xi, self.upper, self.wall0[:, 1])       # Step 1
        self.v_min = -volume_constraint(self.wall0, 0.0)[0]
        self.lo, self.hi = cst_bounds(nb)
        self.free = np.nonzero(self.lo < self.hi)[0]
        self._cache = {}
        # two workspaces used in turn: a new design's solver binds one while
        # the previous design's solver keeps the other, whose f and phi seed
        # (device to device) the new solves
        self._buffers = [None, None]
        self._slots = [None, None]     # (solver, evaluation) bound to each workspace
        self._turn = 0
        self.evaluations = 0

    # -- Steps 2-4 --------------------------------------------------------
    def _solver(self, nodes):
        """A solver for these nodes in the workspace not holding the latest
        design; the evaluation that held that workspace loses its state."""
        g, fl = self.grid, self.wl.flow
        mesh = dvm.Mesh(g.topology, g.ni, g.nj, g.n_wake, nodes)
        s = dvm.Solver(mesh, self.vgrid, fl.Kn, fl.Ma, fl.Tw, fl.objective, self.precision, True,
                       bind=False, order=self.order, limiter=self.limiter)
        k = self._turn
        self._turn ^= 1
        if self._slots[k] is not None:
            self._slots[k][1].solver = None
            self._slots[k] = None
        if self._buffers[k] is None or self._buffers[k].numel() < s.workspace_bytes:
            self._buffers[k] = dvm.alloc_device(s.workspace_bytes)
        s.bind(self._buffers[k])
        return s, k

    def _latest(self, exclude):
        """The most recent other design's evaluation that still has its state."""
        other = self._slots[exclude ^ 1]
        return None if other is None else other[1]

    def evaluate(self, alpha, gradient: bool = True) -> Evaluation:
        alpha = np.array(alpha, dtype=np.float64)
        key = alpha.tobytes()
        ev = self._cache.get(key)
        if ev is None:
            t0 = time.perf_counter()
            eta, deta = cst_eval(self.nb, alpha, self.xi, self.upper, jacobian=True)
            wall = np.stack([self.xi, eta], axis=1)
            nodes = self.deform.apply(wall)                                                 # Step 2
            t1 = time.perf_counter()
            s, k = self._solver(nodes)
            prev = self._latest(k) if self.warm_start else None
            if prev is not None:
                s.state_copy_from(prev.solver, dvm.STATE_F)
            else:
                s.primal_init()
            t2 = time.perf_counter()
            ps = s.primal_iterate(self.max_sweeps, self.solve_tol, self.check_every, raise_notconv=False)  # Step 3
            J, Cd = s.objective()
            t3 = time.perf_counter()
            Q, dQ_dwall = volume_constraint(wall, self.v_min)
            ev = Evaluation(alpha, J, Cd, Q, deta.T @ dQ_dwall[:, 1], primal=ps,
                            seconds=time.perf_counter() - t0, solver=s, deta=deta,
                            times={"deform": t1 - t0, "setup": t2 - t1, "primal": t3 - t2})
            self._cache[key] = ev
            self._slots[k] = (s, ev)
            self.evaluations += 1
            if self.progress:
                self.progress(f"design {self.evaluations}: J {J:.10e} Q {Q:+.3e}, primal {ps[0]} sweeps "
                              f"(r {ps[1]:.1e}), {ev.seconds:.2f} s")
        if gradient and ev.dJ is None:
            t0 = time.perf_counter()
            if ev.solver is None:        # its state was dropped: solve again from the current state
                self._cache.pop(key)
                return self.evaluate(alpha, gradient)
            s = ev.solver
            s.adjoint_init()
            k = 0 if self._slots[0] is not None and self._slots[0][1] is ev else 1
            prev = self._latest(k) if self.warm_start else None
            if prev is not None and prev.dJ is not None:
                s.state_copy_from(prev.solver, dvm.STATE_PHI)
            ev.adjoint = s.adjoint_iterate(self.max_sweeps, self.adjoint_tol, self.check_every, raise_notconv=False)
            t1 = time.perf_counter()
            if self.gradient == "paper":                                                     # Step 4
                dJ_dwall = s.wall_sensitivity()["dJ_dnodes"]
            else:
                dJ_dwall = self.deform.chain(s.mesh_sensitivity())
            ev.dJ = ev.deta.T @ dJ_dwall[:, 1]
            t2 = time.perf_counter()
            ev.times.update(adjoint=t1 - t0, sens=t2 - t1)
            ev.seconds += t2 - t0
            if self.progress:
                self.progress(f"gradient: adjoint {ev.adjoint[0]} sweeps (r {ev.adjoint[1]:.1e}), {t2 - t0:.2f} s")
        return ev

    # -- Steps 5-6 --------------------------------------------------------
    def run(self, max_steps: int = 20, criterion: float = 3e-5) -> dict:
        from scipy.optimize import minimize

        a0, free, sig = self.alpha0, self.free, self.sigma
        t0 = time.perf_counter()

        def design(x):
            a = a0.copy()
            a[free] = np.asarray(x) * sig
            return a

        x0 = a0[free] / sig
        e0 = self.evaluate(design(x0), gradient=True)     # the design the optimiser starts from, bit for bit
        J0 = e0.J
        hist = [e0]

        def step_done(x):
            e = self.evaluate(design(x), gradient=False)
            hist.append(e)
            if abs(e.J - hist[-2].J) / abs(hist[-2].J) < criterion or len(hist) > max_steps:
                raise _Stop

        fun = lambda x: self.evaluate(design(x), gradient=False).J / J0
        jac = lambda x: self.evaluate(design(x)).dJ[free] * sig / J0
        cons = {"type": "ineq", "fun": lambda x: -self.evaluate(design(x), gradient=False).Q / self.v_min,
                "jac": lambda x: -self.evaluate(design(x), gradient=False).dQ[free] * sig / self.v_min}
        bounds = [(None if not np.isfinite(self.lo[p]) else self.lo[p] / sig,
                   None if not np.isfinite(self.hi[p]) else self.hi[p] / sig) for p in free]
        message = "iteration limit"
        try:
            r = minimize(fun, x0, jac=jac, method="SLSQP", bounds=bounds, constraints=[cons],
                         callback=step_done, options={"maxiter": max_steps + 5, "ftol": 1e-15})
            message = r.message
        except _Stop:
            message = "criterion" if abs(hist[-1].J - hist[-2].J) / abs(hist[-2].J) < criterion else "step limit"
        except dvm.DvmError as e:
            # a trial design the optimiser proposed moved the mesh into an
            # invalid one (a cell of non-positive area): stop with what was reached
            message = f"invalid trial design: {e}"
        # solves that stopped at the sweep cap above the tolerance (their J and
        # gradients carry the remaining iteration error)
        capped = sum(1 for e in self._cache.values() if e.primal[1] >= self.solve_tol
                     or (e.dJ is not None and e.adjoint[1] >= self.adjoint_tol))
        return dict(alpha0=a0, fit_rms=self.fit_rms, v_min=self.v_min, history=hist,
                    converged=message == "criterion", message=message, evaluations=self.evaluations,
                    unconverged_solves=capped, seconds=time.perf_counter() - t0)
