"""ORACLE -- test infrastructure only: the shape-optimisation outer loop.

Plain FP64 numpy statement of the parts of the paper's optimisation that sit
around the flow solve, used to check the library's versions of them.  Only
the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module.  It shares no code with the library.

  CST surface eta(xi) = C(xi) S(xi) + xi eta_T     Sec. 3.3, eqs. (cstsuf),
    class function C = xi^N1 (1 - xi)^N2,                 (cst_classfunc),
    shape function S = sum_b A_b S_b(xi),                 (cst_shapefunc),
    S_b the Bernstein polynomials of order N_B       Sec. 3.3
  least-squares initial design                       Sec. 3.3, eq. (cstini)
  volume constraint Q = (1/D) sum x.n dGamma + V_min Sec. 2.4, eq. (formula_opt)
    and its node derivative                          Sec. 3.2, eq. (sens_con_nod)
  bulk-mesh motion by radial-basis-function
    interpolation, Wendland C0 basis                 Sec. 3.4, Step 2
  optimisation loop and stopping test               Sec. 3.4, Steps 1-6,
                                                     eq. (criterion_opt)
  design-variable bounds                             Sec. 4.2, eq. (cst_constraint)

Readings (where the paper leaves the detail open):
  * design vector order alpha = [N1, N2, A_u,0..N_B, A_l,0..N_B, eta_T,u,
    eta_T,l] (2 N_B + 6 entries, the count the paper gives);
  * the least-squares fit of eq. (cstini) runs over every design variable
    that is not held fixed, by damped Gauss-Newton from N1 = 0.5, N2 = 1
    (round nose, sharp tail) with the A's from the linear fit at that class;
  * the Wendland C0 function is phi(r) = (1 - r/R)^2 for r < R, 0 beyond, R
    the support radius; the interpolant has no polynomial part; its centres
    are the reference wall nodes, the bulk nodes move by the interpolated
    displacement of the reference mesh, and the wall nodes take their
    prescribed positions exactly;
  * the gradient optimiser is SLSQP (scipy's implementation of Kraft's
    algorithm, the one the paper names) on the free design variables divided
    by a scale sigma, with objective J / J_0.

Pins (tests/test_oracle_shape.py): Bernstein partition of unity and closed
forms of special designs; recovery of a CST surface's own parameters by the
fit; the polygon area against the shoelace formula and the analytic CST area
(beta functions) under refinement; eq. (sens_con_nod) against central
differences of Q; interpolation at the centres, compact support and positive
definiteness of the RBF system; the chain rule through the deformation
against the brute-force Jacobian.
"""
from __future__ import annotations

import math

import numpy as np


# ---------------------------------------------------------------------------
# CST parameterisation (Sec. 3.3)
# ---------------------------------------------------------------------------

def n_params(nb: int) -> int:
    return 2 * nb + 6


def bernstein(nb: int, xi: np.ndarray) -> np.ndarray:
    """S_b(xi), b = 0..nb, shape (len(xi), nb + 1)."""
    xi = np.asarray(xi, dtype=np.float64)
    return np.stack([math.comb(nb, b) * xi ** b * (1.0 - xi) ** (nb - b) for b in range(nb + 1)], axis=1)


def _xlogy(p, x):
    """x^p log x with its limit 0 at x = 0 (p > 0)."""
    out = np.zeros_like(x)
    pos = x > 0
    out[pos] = x[pos] ** p * np.log(x[pos])
    return out


def cst_eta(nb: int, alpha: np.ndarray, xi: np.ndarray, upper: np.ndarray) -> np.ndarray:
    """eta at stations xi of the upper (upper = True) or lower surface."""
    alpha = np.asarray(alpha, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    upper = np.asarray(upper, dtype=bool)
    N1, N2 = alpha[0], alpha[1]
    Au, Al = alpha[2:nb + 3], alpha[nb + 3:2 * nb + 4]
    Tu, Tl = alpha[2 * nb + 4], alpha[2 * nb + 5]
    C = xi ** N1 * (1.0 - xi) ** N2
    B = bernstein(nb, xi)
    S = np.where(upper, B @ Au, B @ Al)
    return C * S + xi * np.where(upper, Tu, Tl)


def cst_jacobian(nb: int, alpha: np.ndarray, xi: np.ndarray, upper: np.ndarray) -> np.ndarray:
    """d eta_m / d alpha, shape (len(xi), 2 nb + 6)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    upper = np.asarray(upper, dtype=bool)
    N1, N2 = alpha[0], alpha[1]
    Au, Al = alpha[2:nb + 3], alpha[nb + 3:2 * nb + 4]
    B = bernstein(nb, xi)
    S = np.where(upper, B @ Au, B @ Al)
    C = xi ** N1 * (1.0 - xi) ** N2
    Jm = np.zeros((len(xi), n_params(nb)))
    # d C / d N1 = C log xi, d C / d N2 = C log(1 - xi); both vanish where C does
    Jm[:, 0] = _xlogy(N1, xi) * (1.0 - xi) ** N2 * S
    Jm[:, 1] = xi ** N1 * _xlogy(N2, 1.0 - xi) * S
    Jm[:, 2:nb + 3] = np.where(upper[:, None], C[:, None] * B, 0.0)
    Jm[:, nb + 3:2 * nb + 4] = np.where(upper[:, None], 0.0, C[:, None] * B)
    Jm[:, 2 * nb + 4] = np.where(upper, xi, 0.0)
    Jm[:, 2 * nb + 5] = np.where(upper, 0.0, xi)
    return Jm


def cst_fit(nb: int, xi, upper, eta, fixed=None, alpha0=None, max_iter: int = 200):
    """Least-squares design of eq. (cstini): minimise sum_m (eta_CST(xi_m) -
    eta_m)^2 over the variables not in `fixed` (indices held at alpha0's
    values; default the two trailing-edge offsets, held at 0).  Returns
    (alpha, rms residual)."""
    xi = np.asarray(xi, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    upper = np.asarray(upper, dtype=bool)
    npar = n_params(nb)
    fixed = [2 * nb + 4, 2 * nb + 5] if fixed is None else list(fixed)
    free = np.array([p for p in range(npar) if p not in fixed], dtype=int)
    a = np.zeros(npar) if alpha0 is None else np.array(alpha0, dtype=np.float64)
    if alpha0 is None:
        a[0], a[1] = 0.5, 1.0
        # linear least squares for the A's (and free eta_T's) at this class
        lin = np.array([p for p in free if p >= 2], dtype=int)
        Jl = cst_jacobian(nb, a, xi, upper)[:, lin]
        r0 = eta - cst_eta(nb, a, xi, upper)
        a[lin] += np.linalg.lstsq(Jl, r0, rcond=None)[0]
    def cost(al):
        r = eta - cst_eta(nb, al, xi, upper)
        return float(r @ r)
    lam = 1e-3
    c = cost(a)
    for _ in range(max_iter):
        r = eta - cst_eta(nb, a, xi, upper)
        Jf = cst_jacobian(nb, a, xi, upper)[:, free]
        H = Jf.T @ Jf
        g = Jf.T @ r
        improved = False
        for _ in range(30):
            step = np.linalg.solve(H + lam * np.diag(np.diag(H)), g)
            trial = a.copy()
            trial[free] += step
            if trial[0] <= 0 or trial[1] <= 0:
                lam *= 10.0
                continue
            ct = cost(trial)
            if ct <= c:
                improved = c - ct > 1e-15 * c
                a, c = trial, ct
                lam = max(lam / 10.0, 1e-12)
                break
            lam *= 10.0
        if not improved:
            break
    return a, math.sqrt(c / len(xi))


def cst_area(nb: int, alpha) -> float:
    """Exact area between the two CST surfaces on [0, 1] (Beta functions):
    int xi^(N1+b) (1-xi)^(N2+nb-b) dxi = B(N1+b+1, N2+nb-b+1)."""
    a = np.asarray(alpha, dtype=np.float64)
    N1, N2 = a[0], a[1]
    Au, Al = a[2:nb + 3], a[nb + 3:2 * nb + 4]
    tot = 0.0
    for b in range(nb + 1):
        beta = math.exp(math.lgamma(N1 + b + 1) + math.lgamma(N2 + nb - b + 1)
                        - math.lgamma(N1 + N2 + nb + 2))
        tot += math.comb(nb, b) * beta * (Au[b] - Al[b])
    return tot + 0.5 * (a[2 * nb + 4] - a[2 * nb + 5])


# ---------------------------------------------------------------------------
# Volume constraint (Sec. 2.4, Sec. 3.2)
# ---------------------------------------------------------------------------

def volume_constraint(wall_xy: np.ndarray, v_min: float):
    """Q = (1/D) sum_l A_l n_l . x_l + V_min over the closed loop of wall
    elements l = (node l, node l+1), n_l the unit normal into the solid
    (taken as (dy, -dx)/A, which points into the body for the clockwise
    loops of body-fitted grids whose cells are counter-clockwise), x_l the
    element midpoint, D = 2.  Returns (Q, dQ/dx[nw][2] by eq. sens_con_nod)."""
    P = np.asarray(wall_xy, dtype=np.float64)
    Pn = np.roll(P, -1, axis=0)
    An = np.stack([Pn[:, 1] - P[:, 1], P[:, 0] - Pn[:, 0]], axis=1)      # A_l n_l
    mid = 0.5 * (P + Pn)
    Q = 0.5 * float(np.sum(An * mid)) + v_min
    # node m belongs to elements m (as first node) and m-1 (as second)
    dQ = 0.5 * (An + np.roll(An, 1, axis=0))
    return Q, dQ


def shoelace_area(wall_xy: np.ndarray) -> float:
    """Signed polygon area (positive for counter-clockwise order)."""
    P = np.asarray(wall_xy, dtype=np.float64)
    Pn = np.roll(P, -1, axis=0)
    return 0.5 * float(np.sum(P[:, 0] * Pn[:, 1] - Pn[:, 0] * P[:, 1]))


# ---------------------------------------------------------------------------
# Radial-basis-function mesh deformation (Sec. 3.4, Step 2)
# ---------------------------------------------------------------------------

def wendland_c0(r: np.ndarray) -> np.ndarray:
    r = np.asarray(r, dtype=np.float64)
    return np.where(r < 1.0, (1.0 - r) ** 2, 0.0)


def wall_node_index(topology: int, ni: int, nj: int, n_wake: int):
    """For every mesh node (index j*(ni+1) + i) the wall node it is (its
    distinct position on the j = 0 row, l = 0..nw-1), or -1."""
    nw = ni - 2 * n_wake
    idx = -np.ones((nj + 1) * (ni + 1), dtype=np.int64)
    for i in range(n_wake, n_wake + nw + 1):
        idx[i] = (i - n_wake) % nw
    return idx


def _distance(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """|a_i - b_j| for every pair of points: sqrt(dx^2 + dy^2)."""
    dx = a[:, None, 0] - b[None, :, 0]
    dy = a[:, None, 1] - b[None, :, 1]
    dx *= dx
    dy *= dy
    dx += dy
    return np.sqrt(dx, out=dx)


class RBFDeform:
    """Interpolated motion of every mesh node from the wall nodes' motion.

    Centres c_w: the reference wall nodes.  M[w, v] = phi(|c_w - c_v| / R);
    for wall displacements d[w] the weights solve M gamma = d, and node n
    moves by sum_w gamma_w phi(|x_n - c_w| / R) (reference positions);
    wall nodes are set to their prescribed positions."""

    def __init__(self, ref_nodes: np.ndarray, wall_idx: np.ndarray, radius: float):
        self.x0 = np.asarray(ref_nodes, dtype=np.float64).reshape(-1, 2).copy()
        self.widx = np.asarray(wall_idx)
        nw = int(self.widx.max()) + 1
        self.c = np.zeros((nw, 2))
        for n in np.nonzero(self.widx >= 0)[0]:
            self.c[self.widx[n]] = self.x0[n]
        self.R = float(radius)
        self.M = wendland_c0(_distance(self.c, self.c) / self.R)
        self.Phi = wendland_c0(_distance(self.x0, self.c) / self.R)

    def apply(self, wall_new: np.ndarray) -> np.ndarray:
        d = np.asarray(wall_new, dtype=np.float64) - self.c
        gamma = np.linalg.solve(self.M, d)
        x = self.x0 + self.Phi @ gamma
        on = self.widx >= 0
        x[on] = np.asarray(wall_new)[self.widx[on]]
        return x

    def chain(self, g: np.ndarray) -> np.ndarray:
        """dJ/d(wall node positions) from dJ/d(all node positions) g[n][2]."""
        g = np.asarray(g, dtype=np.float64).reshape(-1, 2)
        on = self.widx >= 0
        direct = np.zeros_like(self.c)
        np.add.at(direct, self.widx[on], g[on])
        h = self.Phi[~on].T @ g[~on]
        return direct + np.linalg.solve(self.M.T, h)


# ---------------------------------------------------------------------------
# Optimisation loop (Sec. 3.4)
# ---------------------------------------------------------------------------

def airfoil_stations(grid):
    """Wall nodes of a C-grid airfoil (leading edge at (0, 0), trailing edge
    at (1, 0), chord 1): their positions, xi = x, and which surface each is
    on (the nodes after the leading edge in wall order are upper)."""
    nw = grid.ni - 2 * grid.n_wake
    wall = grid.nodes[0, grid.n_wake:grid.n_wake + nw].copy()
    le = int(np.argmin(wall[:, 0]))
    if abs(wall[le, 0]) > 1e-12 or abs(wall[0, 0] - 1.0) > 1e-12:
        raise ValueError("airfoil must have its leading edge at x = 0 and trailing edge at x = 1")
    upper = np.arange(nw) > le
    return wall, wall[:, 0].copy(), upper


# Design-variable bounds of eq. (cst_constraint): N1, N2 >= 0.01, upper
# shape coefficients >= 0, lower <= 0, trailing-edge offsets held at 0.
def cst_bounds(nb: int):
    lo = np.full(n_params(nb), -np.inf)
    hi = np.full(n_params(nb), np.inf)
    lo[0] = lo[1] = 0.01
    lo[2:nb + 3] = 0.0
    hi[nb + 3:2 * nb + 4] = 0.0
    lo[2 * nb + 4:] = hi[2 * nb + 4:] = 0.0
    return lo, hi


class _Stop(Exception):
    pass


def optimise(wl, nb: int = 6, radius: float = 2.0, sigma: float = 0.01, max_steps: int = 20,
             criterion: float = 3e-5, gradient: str = "paper", solve_tol: float = 1e-12,
             max_sweeps: int = 200000, nthreads=None, order: int = 1, correction_every: int = 40):
    """Steps 1-6 of Sec. 3.4 with the oracle solver (spatial order 1, or 2
    with the Venkatakrishnan limiter and the given correction interval).
    Returns a dict with the initial fit, and per optimisation step the
    design, J, Q."""
    import oracle
    from scipy.optimize import minimize

    g, vg, fl = wl.grid, wl.vgrid, wl.flow
    wall0, xi, upper = airfoil_stations(g)
    alpha0, rms = cst_fit(nb, xi, upper, wall0[:, 1])                       # Step 1
    v_min = -volume_constraint(wall0, 0.0)[0]
    deform = RBFDeform(g.nodes, wall_node_index(g.topology, g.ni, g.nj, g.n_wake), radius)
    lo, hi = cst_bounds(nb)
    free = np.nonzero(lo < hi)[0]
    cache = {}

    def evaluate(alpha):
        key = alpha.tobytes()
        if key in cache:
            return cache[key]
        eta = cst_eta(nb, alpha, xi, upper)
        wall = np.stack([xi, eta], axis=1)
        nodes = deform.apply(wall).reshape(g.nj + 1, g.ni + 1, 2)         # Step 2
        p = oracle.Problem(g.topology, g.ni, g.nj, g.n_wake, nodes, vg.kind, vg.n1, vg.n2,
                           vg.vmax, vg.param, fl.Kn, fl.Ma, fl.Tw, fl.objective, nthreads)
        if order == 2:
            p.set_scheme(2, True, correction_every)
        p.primal_init()                                                      # Step 3
        p.primal_solve(solve_tol, max_sweeps, 50)
        J = p.objective()
        p.adjoint_init()
        p.adjoint_solve(solve_tol, max_sweeps, 50)
        if gradient == "paper":                                              # Step 4
            dJ_dwall = p.wall_sensitivity()["dJ_dnodes"]
        else:
            dJ_dwall = deform.chain(p.mesh_sensitivity())
        deta = cst_jacobian(nb, alpha, xi, upper)
        dJ = deta.T @ dJ_dwall[:, 1]
        Q, dQ_dwall = volume_constraint(wall, v_min)
        dQ = deta.T @ dQ_dwall[:, 1]
        cache[key] = (J, dJ, Q, dQ)
        return cache[key]

    def design(x):
        a = alpha0.copy()
        a[free] = x * sigma
        return a

    x0 = alpha0[free] / sigma
    a_start = design(x0)
    J0, _, Q0, _ = evaluate(a_start)
    hist = [(a_start, J0, Q0)]

    def step_done(x):                                                        # Step 6
        a = design(x)
        J, _, Q, _ = evaluate(a)
        hist.append((a, J, Q))
        if abs(J - hist[-2][1]) / abs(hist[-2][1]) < criterion:
            raise _Stop
        if len(hist) > max_steps:
            raise _Stop

    fun = lambda x: evaluate(design(x))[0] / J0
    jac = lambda x: evaluate(design(x))[1][free] * sigma / J0
    cons = {"type": "ineq", "fun": lambda x: -evaluate(design(x))[2] / v_min,
            "jac": lambda x: -evaluate(design(x))[3][free] * sigma / v_min}
    bounds = [(lo[p] / sigma, hi[p] / sigma) for p in free]
    bounds = [(None if not np.isfinite(b[0]) else b[0], None if not np.isfinite(b[1]) else b[1]) for b in bounds]
    converged = False
    try:                                                                     # Step 5
        minimize(fun, x0, jac=jac, method="SLSQP", bounds=bounds,
                 constraints=[cons], callback=step_done,
                 options={"maxiter": max_steps + 5, "ftol": 1e-15})
    except _Stop:
        converged = abs(hist[-1][1] - hist[-2][1]) / abs(hist[-2][1]) < criterion
    return dict(alpha0=alpha0, fit_rms=rms, v_min=v_min, history=hist, converged=converged)
