"""Pins of the oracle's discrete-conservative equilibrium (an option beside
the pointwise Maxwellian; the reading of Sec. 2.1 on a discrete velocity
grid: the equilibrium of a cell is the reduced Maxwellian whose moments on
the grid equal the cell's moments W).

* Definition: the grid moments of g(P'(W)) equal W to rounding on grids
  whose quadrature of the Maxwellian is off by up to 1e-2 (Newton-Cotes,
  sinh-stretched, coarse midpoint), where the pointwise Maxwellian's are
  measurably off.
* Where the grid integrates the Maxwellian exactly to rounding (32 midpoint
  cells on [-6, 6]), P'(W) is the primitive-variable vector of W.
* dP'/dW against central differences.
* A gas at rest at the wall temperature is a fixed point of a sweep with
  collisions on any grid (pointwise: it drifts by the quadrature defect).
* The adjoint with this equilibrium: dot-product identity against the
  complex-step twin of the residual and dJ/dKn against central differences
  of re-converged drags.
* The Jacobi iteration that diverges with the pointwise Maxwellian on a
  grid with a quadrature defect in the near-continuum regime (64x32 C-grid,
  24x24 Newton-Cotes velocities, Kn 0.01) converges with this one.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2501_00923_amd import inputs as I

GRIDS = [(I.VG_NEWTON_COTES, 28, 6.0, 0.0), (I.VG_NEWTON_COTES, 32, 6.0, 0.0), (I.VG_NEWTON_COTES, 48, 6.0, 0.0),
         (I.VG_SINH, 64, 6.0, 2.0), (I.VG_MIDPOINT, 8, 5.0, 0.0)]
STATES = [(1.0, 0.4564, 0.0, 0.5), (1.5, 0.2, 0.1, 0.3), (0.7, 1.8257, -0.3, 0.9), (1.0, 0.0, 0.0, 0.5)]


def _cons(rho, u1, u2, th):
    # conservative variables of a primitive state (gamma = 5/3): the input
    return np.array([rho, rho * u1, rho * u2, 0.5 * rho * (u1 * u1 + u2 * u2) + 1.5 * rho * th])


def _problem(kind, n, vmax, param, eq=1, Kn=1.0, Ma=0.5, Tw=1.0):
    wl = I.tiny_circle(nv=n, vmax=vmax, Kn=Kn, Ma=Ma, Tw=Tw, kind=kind)
    wl.vgrid.param = param
    p = oracle.Problem.from_workload(wl, nthreads=2)
    p.set_equilibrium(eq)
    return p


@pytest.mark.parametrize("grid", GRIDS, ids=lambda g: f"k{g[0]}n{g[1]}")
def test_equilibrium_moments_equal_W(grid):
    p = _problem(*grid)
    v, w = p.vgrid()
    worst_pointwise = 0.0
    for st in STATES:
        W = _cons(*st)
        P, _ = p.eq_params(W)
        m = oracle.moments(v, w, oracle.maxwell(*P, v))
        assert np.max(np.abs(m - W)) <= 1e-13 * np.max(np.abs(W)), (grid, st, m - W)
        mp = oracle.moments(v, w, oracle.maxwell(*st, v))
        worst_pointwise = max(worst_pointwise, np.max(np.abs(mp - W)) / np.max(np.abs(W)))
    assert worst_pointwise > 1e-6            # the grid's quadrature of the Maxwellian is not exact


def test_equals_primitive_variables_where_the_quadrature_is_exact():
    p = _problem(I.VG_MIDPOINT, 32, 6.0, 0.0)
    for st in STATES[:2] + STATES[3:]:
        P, _ = p.eq_params(_cons(*st))
        assert np.max(np.abs(P - np.array(st))) <= 1e-12, (st, P)
    q = _problem(I.VG_NEWTON_COTES, 28, 6.0, 0.0, eq=0)
    for st in STATES:
        P, _ = q.eq_params(_cons(*st))
        assert np.max(np.abs(P - np.array(st))) <= 1e-14


@pytest.mark.parametrize("eq", [0, 1])
def test_derivative_matches_central_differences(eq):
    p = _problem(I.VG_NEWTON_COTES, 28, 6.0, 0.0, eq=eq)
    for st in STATES:
        W = _cons(*st)
        _, M = p.eq_params(W)
        for m in range(4):
            h = 1e-6 * max(1.0, abs(W[m]))
            e = np.zeros(4)
            e[m] = h
            fd = (p.eq_params(W + e)[0] - p.eq_params(W - e)[0]) / (2 * h)
            assert np.max(np.abs(fd - M[:, m])) <= 1e-7 * max(1.0, np.max(np.abs(M[:, m]))), (st, m)


def test_gas_at_rest_is_stationary_with_collisions():
    """u_inf = 0 and T_w = 1: f = g(1, 0, 1/2) everywhere; one sweep with
    collisions (Kn 0.3) leaves it unchanged to rounding with the
    conservative equilibrium, and moves it by the quadrature defect with the
    pointwise one (28x28 Newton-Cotes grid)."""
    change = {}
    for eq in (0, 1):
        p = _problem(I.VG_NEWTON_COTES, 28, 6.0, 0.0, eq=eq, Kn=0.3, Ma=0.0)
        p.primal_init()
        f0 = p.f
        p.primal_iterate(1)
        change[eq] = np.max(np.abs(p.f - f0)) / np.max(f0)
    assert change[1] <= 1e-14
    assert change[0] > 1e-6


def _solved(wl, eq, **kw):
    p = oracle.Problem.from_workload(wl, nthreads=4, **kw)
    p.set_equilibrium(eq)
    p.primal_init()
    it, r = p.primal_solve(1e-15, 30000)
    assert r < 1e-13
    return p


def test_adjoint_is_the_transpose_with_the_conservative_equilibrium():
    wl = I.tiny_circle(Kn=0.5, Ma=0.6)                  # 8x8 midpoint cells on [-5, 5]: defect ~1e-3
    p = _solved(wl, 1)
    rng = np.random.default_rng(5)
    u = rng.standard_normal((p.nc, p.nv, 2))
    phi = rng.standard_normal((p.nc, p.nv, 2))
    _, w = p.vgrid()
    dR, _ = p.complex_step(u)
    lhs = np.sum(w[None, :, None] * phi * dR)
    rhs = np.sum(w[None, :, None] * u * p.adjoint_operator(phi, with_source=False))
    assert abs(lhs - rhs) < 1e-13 * np.sum(np.abs(w[None, :, None] * phi * dR))
    # dJ/dKn from the adjoint against central differences of re-converged drags
    p.adjoint_init()
    p.adjoint_solve(1e-15, 30000)
    h = 1e-5
    fd = (_solved(wl, 1, Kn=wl.flow.Kn + h).objective() - _solved(wl, 1, Kn=wl.flow.Kn - h).objective()) / (2 * h)
    assert abs(p.adjoint_dJdp(oracle.KN) - fd) < 1e-8 * abs(fd)
    # the two equilibria give different drags on this grid (the option matters)
    assert abs(_solved(wl, 0).objective() - p.objective()) > 1e-8 * abs(p.objective())


def test_near_continuum_iteration_converges_with_the_conservative_equilibrium():
    g = I.naca_cgrid(8, 24, 32, t=0.12, m=0.0)
    wl = I.Workload("c64x32_nc24_kn0.01", g, I.VGridSpec(I.VG_NEWTON_COTES, 24, 24, 6.0), I.FlowSpec(0.01, 0.5), 0)
    res = {}
    for eq in (0, 1):
        p = oracle.Problem.from_workload(wl, nthreads=8)
        p.set_equilibrium(eq)
        p.primal_init()
        rs = [p.primal_iterate(25) for _ in range(4)]
        res[eq] = rs
    assert not all(math.isfinite(r) and r < 1e-2 for r in res[0])       # pointwise: blows up
    r1 = res[1]
    assert all(b < a for a, b in zip(r1, r1[1:])) and r1[-1] < 1e-3     # conservative: steady decrease
