"""Differentiable drag: shape parameters -> J with a hand-written adjoint.

``ShapeCase`` describes a family of bodies (a grid generator taking the
shape parameters alpha), a velocity grid, a flow state and solve options.
``drag(alpha, case)`` returns J (FP64 scalar tensor); its backward runs the
adjoint sweep and the wall sensitivity of the paper (Sec. 2.5 eq. sens_shape,
Sec. 3.2) on the GPU and chains dJ/d(wall nodes) through d(wall nodes)/dalpha,
or, with ``exact=True``, the exact discrete derivative in every mesh node
chained through d(nodes)/dalpha.

The fixed-point adjoint needs only the converged primal state, so the
forward keeps that state on the device; with ``offload=True`` it instead
snapshots f to host memory and frees the device workspace between forward
and backward (for memory pressure), and ``checkpoint_every`` keeps host
snapshots of f during the primal solve (resume / inspection).
"""
from __future__ import annotations

import warnings
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import torch

from . import dvm
from . import inputs as I


@dataclass
class SolveOptions:
    max_iter: int = 20000
    tol: float = 1e-10
    check_every: int = 50
    adjoint_max_iter: int = 20000
    adjoint_tol: float = 1e-10
    fixed_iters: bool = False        # run exactly max_iter / adjoint_max_iter sweeps
    on_notconv: str = "warn"         # a solve left above its tolerance: "warn", "raise" or "ignore"


class NotConvergedWarning(RuntimeWarning):
    """A primal or adjoint solve stopped at its sweep cap above tolerance."""


def _unconverged(o: SolveOptions, what: str, iters: int, resid: float, tol: float):
    if o.fixed_iters or resid < tol or o.on_notconv == "ignore":
        return
    msg = f"{what} solve not converged: residual {resid:.3e} above {tol:.1e} after {iters} sweeps"
    if o.on_notconv == "raise":
        raise dvm.NotConverged(dvm.DVM_ENOTCONV, msg)
    warnings.warn(msg, NotConvergedWarning, stacklevel=3)


@dataclass
class ShapeCase:
    make_grid: Callable[[np.ndarray], I.GridInput]
    vgrid: I.VGridSpec
    flow: I.FlowSpec
    precision: int = dvm.FP64
    options: SolveOptions = field(default_factory=SolveOptions)
    checkpoint_every: int = 0
    keep_checkpoints: Optional[int] = None   # None: keep every snapshot; n: only the last n
    offload: bool = False
    exact: bool = False      # exact discrete derivative (every mesh node moves) instead of the wall-only form
    order: int = 1           # spatial scheme: 1, or 2 (exact form: limiter factors of f held fixed)
    limiter: int = dvm.LIMITER_VENKAT
    correction_every: int = 40


@dataclass
class ForwardRecord:
    iters: int = 0
    resid: float = float("nan")
    Cd: float = float("nan")
    checkpoints: List[np.ndarray] = field(default_factory=list)
    checkpoint_iters: List[int] = field(default_factory=list)   # sweeps done at each kept snapshot
    adjoint_iters: int = 0
    adjoint_resid: float = float("nan")


def _primal(case: ShapeCase, solver: dvm.Solver, rec: ForwardRecord):
    o = case.options
    if case.checkpoint_every > 0:
        left = o.max_iter
        while left > 0:
            m = min(case.checkpoint_every, left)
            it, r = solver.primal_iterate(m, 0.0 if o.fixed_iters else o.tol, m, raise_notconv=False)
            rec.iters += it
            rec.resid = r
            left -= it
            rec.checkpoints.append(solver.state_save(dvm.STATE_F))
            rec.checkpoint_iters.append(rec.iters)
            if case.keep_checkpoints is not None and len(rec.checkpoints) > case.keep_checkpoints:
                drop = len(rec.checkpoints) - case.keep_checkpoints
                del rec.checkpoints[:drop], rec.checkpoint_iters[:drop]
            if not o.fixed_iters and r < o.tol:
                break
    else:
        if o.fixed_iters:
            it, r = solver.primal_iterate(o.max_iter)
        else:
            it, r = solver.primal_iterate(o.max_iter, o.tol, o.check_every, raise_notconv=False)
        rec.iters, rec.resid = it, r


class _DragFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alpha: torch.Tensor, case: ShapeCase, rec: ForwardRecord):
        a = alpha.detach().cpu().double().numpy()
        grid = case.make_grid(a)
        solver = dvm.Solver(dvm.Mesh.from_grid(grid), dvm.VGrid.from_spec(case.vgrid), case.flow.Kn,
                            case.flow.Ma, case.flow.Tw, case.flow.objective, case.precision, True,
                            order=case.order, limiter=case.limiter, correction_every=case.correction_every)
        solver.primal_init()
        _primal(case, solver, rec)
        _unconverged(case.options, "primal", rec.iters, rec.resid, case.options.tol)
        J, Cd = solver.objective()
        rec.Cd = Cd
        ctx.case, ctx.rec, ctx.wall_jac, ctx.node_jac = case, rec, grid.wall_jac, grid.node_jac
        ctx.alpha_device, ctx.alpha_dtype = alpha.device, alpha.dtype
        if case.offload:
            ctx.f_host = solver.state_save(dvm.STATE_F)
            solver.buffer = None          # release the device workspace
            torch.cuda.empty_cache()
        ctx.solver = solver
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        case, solver = ctx.case, ctx.solver
        if case.offload:
            solver.bind()
            solver.state_load(dvm.STATE_F, ctx.f_host)
        solver.adjoint_init()
        o = case.options
        if o.fixed_iters:
            it, r = solver.adjoint_iterate(o.adjoint_max_iter)
        else:
            it, r = solver.adjoint_iterate(o.adjoint_max_iter, o.adjoint_tol, o.check_every, raise_notconv=False)
        ctx.rec.adjoint_iters, ctx.rec.adjoint_resid = it, r
        _unconverged(o, "adjoint", it, r, o.adjoint_tol)
        if case.exact:
            dJ = np.einsum("jid,jidp->p", solver.mesh_sensitivity(), ctx.node_jac)
        else:
            dJ = solver.param_sensitivity(ctx.wall_jac)
        ctx.solver = None
        grad = torch.from_numpy(dJ) * gJ.detach().cpu().double()
        return grad.to(device=ctx.alpha_device, dtype=ctx.alpha_dtype), None, None


def drag(alpha: torch.Tensor, case: ShapeCase, record: Optional[ForwardRecord] = None) -> torch.Tensor:
    """J(alpha) with dJ/dalpha from the adjoint (paper-mode wall sensitivity)."""
    rec = ForwardRecord() if record is None else record
    return _DragFn.apply(alpha, case, rec)


def naca_bspline_case(seed: int = 0, **kw) -> tuple:
    """The differentiation workload: seed-drawn NACA thickness / camber,
    192x96 C-grid, 48x48 Newton-Cotes grid on [-6, 6], Kn 0.5, Ma 2, 24
    B-spline control-point offsets drawn N(0, 1e-3).  Returns (case, alpha0)."""
    wl = I.c4_naca_bspline(seed)
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.08, 0.16)
    m = rng.uniform(0.0, 0.04)

    def make(alpha):
        return I.naca_cgrid(24, 72, 96, t=t, m=m, p=0.4,
                            perturb={"kind": "bspline", "n_ctrl": 14, "amp": np.asarray(alpha)})
    return ShapeCase(make, wl.vgrid, wl.flow, **kw), wl.grid.params.copy()


def circle_fourier_case(ni=64, nj=32, nv=16, vmax=5.0, Kn=1.0, Ma=0.5, r_outer=10.0, stretch=1.1,
                        **kw) -> tuple:
    """Circle with 8 radial Fourier modes (a0..a3, b1..b4)."""
    def make(alpha):
        alpha = np.asarray(alpha)
        return I.ogrid(ni, nj, r_outer, stretch, alpha[:4], alpha[4:])
    return (ShapeCase(make, I.VGridSpec(I.VG_MIDPOINT, nv, nv, vmax), I.FlowSpec(Kn, Ma), **kw),
            np.zeros(8))


def cst_case(wl, nb: int = 6, radius: float = 2.0, **kw) -> tuple:
    """The optimisation's own parameterisation as a differentiable family:
    the airfoil of workload `wl` (a C-grid with its leading edge at (0, 0)
    and trailing edge at (1, 0)) fitted by a CST design (Sec. 3.3, eq.
    cstini), bodies alpha -> wall nodes (xi_m, eta_CST(xi_m)) and the bulk
    mesh moved by the Wendland-C0 RBF interpolation (Sec. 3.4, Step 2).
    d(nodes)/d(alpha) is exact: the motion is linear in the wall
    displacement, so each column is one motion of the CST Jacobian's
    column.  Returns (case, alpha0)."""
    from .optimize import airfoil_wall
    from .shape import Deformer, cst_eval, cst_fit, n_params

    g0 = wl.grid
    wall0, xi, upper = airfoil_wall(g0)
    alpha0, _ = cst_fit(nb, xi, upper, wall0[:, 1])
    deform = Deformer(dvm.Mesh.from_grid(g0), radius)
    base = deform.apply(wall0)
    npar = n_params(nb)
    names = ["N1", "N2"] + [f"A_u{b}" for b in range(nb + 1)] + [f"A_l{b}" for b in range(nb + 1)] + ["eta_Tu", "eta_Tl"]

    def make(alpha):
        alpha = np.asarray(alpha, dtype=np.float64)
        eta, deta = cst_eval(nb, alpha, xi, upper, jacobian=True)
        nodes = deform.apply(np.stack([xi, eta], axis=1))
        wall_jac = np.zeros((len(xi), 2, npar))
        wall_jac[:, 1, :] = deta
        node_jac = np.zeros(nodes.shape + (npar,))
        for p in range(npar):
            if np.any(deta[:, p]):
                step = np.stack([np.zeros_like(xi), deta[:, p]], axis=1)
                node_jac[..., p] = deform.apply(wall0 + step) - base
        return I.GridInput(g0.topology, g0.ni, g0.nj, g0.n_wake, nodes, wall_jac, node_jac, alpha.copy(), names)

    return ShapeCase(make, wl.vgrid, wl.flow, **kw), alpha0
