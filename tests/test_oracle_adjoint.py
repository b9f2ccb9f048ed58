"""Oracle pins of the adjoint (Sec. 2.5, eq. formula_adjointbgk; Sec. 3.1,
eq. numerad_gov).

* Dot-product identity: the homogeneous adjoint operator is the transpose of
  the linearised primal residual under sum_k w_k, where the linearisation is
  a complex-step derivative of an independently written complex-valued twin
  of the primal residual (so an error in dg/dW, the wall coupling or the
  face upwinding on either side shows up).
* At the converged adjoint, -sum w phi . (dR/df u) equals dJ/df u.
* dJ/dp from the adjoint equals central finite differences of J from fully
  re-converged primal solves, for p = Kn, Ma, T_w.
"""
import numpy as np
import pytest

import oracle
from paper_2501_00923_amd import inputs as I

CASES = [I.tiny_circle(Kn=1.0, Ma=0.5), I.tiny_naca(Kn=0.7, Ma=1.2)]


def _solved(wl, **kw):
    p = oracle.Problem.from_workload(wl, nthreads=4, **kw)
    p.primal_init()
    it, r = p.primal_solve(1e-15, 30000)
    assert r < 1e-13
    return p


@pytest.mark.parametrize("wl", CASES, ids=lambda w: w.name)
def test_dot_product_identity(wl):
    p = _solved(wl)
    rng = np.random.default_rng(1)
    u = rng.standard_normal((p.nc, p.nv, 2))
    phi = rng.standard_normal((p.nc, p.nv, 2))
    _, w = p.vgrid()
    dR, _ = p.complex_step(u)
    lhs = np.sum(w[None, :, None] * phi * dR)
    rhs = np.sum(w[None, :, None] * u * p.adjoint_operator(phi, with_source=False))
    assert abs(lhs - rhs) < 1e-13 * (abs(lhs) + np.sum(np.abs(w[None, :, None] * phi * dR)) * 1e-3)


@pytest.mark.parametrize("wl", CASES, ids=lambda w: w.name)
def test_converged_adjoint_identity(wl):
    p = _solved(wl)
    p.adjoint_init()
    it, r = p.adjoint_solve(1e-15, 30000)
    assert r < 1e-13
    phi = p.phi
    _, w = p.vgrid()
    rng = np.random.default_rng(2)
    for _ in range(2):
        u = rng.standard_normal((p.nc, p.nv, 2))
        dR, dJ = p.complex_step(u)
        lhs = -np.sum(w[None, :, None] * phi * dR)
        assert abs(lhs - dJ) < 1e-11 * max(1.0, abs(dJ))
    # the fixed point zeroes the adjoint equation
    assert np.max(np.abs(p.adjoint_operator(phi))) < 1e-11


@pytest.mark.parametrize("which,name,h", [(oracle.KN, "Kn", 1e-5), (oracle.MA, "Ma", 1e-5),
                                          (oracle.TW, "Tw", 1e-5)])
def test_adjoint_gradient_matches_finite_differences(which, name, h):
    wl = CASES[0]
    p = _solved(wl)
    p.adjoint_init()
    p.adjoint_solve(1e-15, 30000)
    base = {"Kn": wl.flow.Kn, "Ma": wl.flow.Ma, "Tw": wl.flow.Tw}[name]
    Jp = _solved(wl, **{name: base + h}).objective()
    Jm = _solved(wl, **{name: base - h}).objective()
    fd = (Jp - Jm) / (2 * h)
    adj = p.adjoint_dJdp(which)
    assert abs(adj - fd) < 1e-8 * abs(fd)


def test_adjoint_gradient_naca_kn():
    wl = CASES[1]
    p = _solved(wl)
    p.adjoint_init()
    p.adjoint_solve(1e-15, 30000)
    h = 1e-5
    fd = (_solved(wl, Kn=wl.flow.Kn + h).objective() - _solved(wl, Kn=wl.flow.Kn - h).objective()) / (2 * h)
    assert abs(p.adjoint_dJdp(oracle.KN) - fd) < 1e-8 * abs(fd)
