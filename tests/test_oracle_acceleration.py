"""Pins of the oracle's macroscopic prediction (the reading of Sec. 3.1's
prediction acceleration: every K sweeps a linearised macroscopic system
driven by the moments of the kinetic residual predicts the moments the next
sweep relaxes towards).

* The system is the linearisation of the scheme's transport restricted to
  local equilibria plus a pseudo-time term on the diagonal: for a
  perturbation dW of the moments, the cell moments of the complex-step
  derivative of the residual (the independently written complex twin) in
  the direction of the equilibrium perturbation dg/dW dW equal
  (D - lam I) dW_c + sum_q O_q dW_nbr (conservative equilibrium: the
  collision part's moments vanish), wall coupling included; r is the moment
  vector of the residual.  The prediction is refused with the pointwise
  Maxwellian.
* The discrete solution is a fixed point of the accelerated iteration, and
  the plain and accelerated iterations converge to the same state.
* The first prediction changes rho and theta by at most 20% in any cell.
* Near the continuum limit the accelerated iteration reaches 1e-8 in a few
  hundred sweeps where the plain one is still above 1e-5.
* Adjoint: the Gauss-Seidel map's transpose passes the dot-product test;
  two accelerated adjoint sweeps F1 F1 and three primal sweeps P1 P1 P0
  (plain, then two after a prediction; central differences of the oracle's
  own primal iteration) satisfy <F1 F1 a, R' P0 b> = <a, R' P1 P1 P0 b>
  under sum_k w_k, R' the complex-step derivative of the residual -- the
  identity that makes the accelerated adjoint cycle share the primal
  cycle's eigenvalues; the accelerated and plain adjoint iterations reach
  the same phi and the same sensitivities.
"""
import numpy as np
import pytest

import oracle
from paper_2501_00923_amd import inputs as I


def _theta(W):
    u1, u2 = W[..., 1] / W[..., 0], W[..., 2] / W[..., 0]
    return (2.0 / 3.0) * (W[..., 3] / W[..., 0] - 0.5 * (u1 * u1 + u2 * u2))


@pytest.mark.parametrize("wl", [I.tiny_circle(Kn=0.05, Ma=0.6), I.tiny_naca(Kn=0.02, Ma=0.9)],
                         ids=lambda w: w.name)
def test_macroscopic_system_is_the_linearised_transport(wl):
    p = oracle.Problem.from_workload(wl, nthreads=4)
    p.set_equilibrium(1)
    p.primal_init()
    p.primal_iterate(7)
    r, Dinv, O, lam = p.macro_system()
    assert np.all(lam > 0)
    v, w = p.vgrid()
    # r: the moments of the residual at the current f
    R = p.primal_residual()
    psi = np.stack([np.ones(p.nv), v[:, 0], v[:, 1], 0.5 * (v[:, 0] ** 2 + v[:, 1] ** 2)], -1)
    rm = np.einsum("k,ka,ck->ca", w, psi, R[..., 0])
    rm[:, 3] += np.einsum("k,ck->c", w, R[..., 1])
    assert np.max(np.abs(r - rm)) <= 1e-12 * np.max(np.abs(rm))
    # A dW against the complex-step derivative in the direction dg/dW dW
    rng = np.random.default_rng(3)
    W = p.W
    dW = rng.standard_normal(W.shape) * np.abs(W) * 1e-2
    u = np.zeros((p.nc, p.nv, 2))
    for c in range(p.nc):
        P, M = p.eq_params(W[c])
        for k in range(p.nv):
            # dg/dP' at (P', v_k), then through dP'/dW
            rho, u1, u2, th = P
            c1, c2 = v[k, 0] - u1, v[k, 1] - u2
            g1 = oracle.maxwell(rho, u1, u2, th, v[k:k + 1])[0, 0]
            d1 = np.array([g1 / rho, g1 * c1 / th, g1 * c2 / th, g1 * ((c1 * c1 + c2 * c2) / (2 * th * th) - 1 / th)])
            d2 = 0.5 * th * d1
            d2[3] += 0.5 * g1
            u[c, k, 0] = d1 @ (M @ dW[c])
            u[c, k, 1] = d2 @ (M @ dW[c])
    dR, _ = p.complex_step(u)
    lin = np.einsum("k,ka,ck->ca", w, psi, dR[..., 0])
    lin[:, 3] += np.einsum("k,ck->c", w, dR[..., 1])
    m = p.mesh()
    Ad = np.einsum("cab,cb->ca", np.linalg.inv(Dinv) - lam[:, None, None] * np.eye(4), dW)
    for q in range(4):
        nb = m["nbr"][:, q]
        Ad += np.where((nb >= 0)[:, None], np.einsum("cab,cb->ca", O[:, q], dW[np.maximum(nb, 0)]), 0.0)
    assert np.max(np.abs(Ad - lin)) <= 1e-10 * np.max(np.abs(lin))


def test_solution_is_a_fixed_point_and_both_iterations_agree():
    wl = I.tiny_circle(Kn=0.3, Ma=0.5)
    plain = oracle.Problem.from_workload(wl, nthreads=4)
    plain.set_equilibrium(1)
    plain.primal_init()
    it_p, r_p = plain.primal_solve(1e-14, 40000)
    acc = oracle.Problem.from_workload(wl, nthreads=4)
    acc.set_equilibrium(1)
    acc.set_acceleration(5, 50)
    acc.primal_init()
    it_a, r_a = acc.primal_solve(1e-14, 40000, check_every=5)
    assert r_p < 1e-14 and r_a < 1e-14 and it_a < it_p
    assert np.max(np.abs(acc.f - plain.f)) <= 1e-10 * np.max(plain.f)
    assert abs(acc.objective() - plain.objective()) <= 1e-10 * abs(plain.objective())
    # the converged state: the residual's moments vanish, the prediction
    # does not move it
    r, _, _, _ = acc.macro_system()
    assert np.max(np.abs(r)) <= 1e-10 * np.max(np.abs(acc.W))
    f0 = acc.f
    acc.primal_iterate(5)
    assert np.max(np.abs(acc.f - f0)) <= 1e-11 * np.max(f0)


def test_prediction_is_limited_and_accelerates_near_the_continuum():
    g = I.naca_cgrid(8, 24, 32, t=0.12, m=0.0)
    wl = I.Workload("c64x32_v16_kn0.001", g, I.VGridSpec(I.VG_MIDPOINT, 16, 16, 6.0), I.FlowSpec(1e-3, 0.5), 0)
    p = oracle.Problem.from_workload(wl, nthreads=8)
    p.set_equilibrium(1)
    p.set_acceleration(5, 50)
    p.primal_init()
    p.primal_iterate(4)
    W4 = p.W
    p.primal_iterate(1)                 # sweep 5, then the first prediction
    q = oracle.Problem.from_workload(wl, nthreads=8)
    q.set_equilibrium(1)
    q.primal_init()
    q.primal_iterate(5)                 # the same 5 sweeps, no prediction
    Wp, Ws = p.W, q.W
    assert np.max(np.abs(Wp - Ws)) > 1e-3 * np.max(np.abs(Ws))     # the prediction moved W
    assert np.max(np.abs(Wp[:, 0] - Ws[:, 0]) / Ws[:, 0]) <= 0.2 + 1e-12
    assert np.max(np.abs(_theta(Wp) - _theta(Ws)) / _theta(Ws)) <= 0.2 + 1e-12
    del W4
    it, r = p.primal_solve(1e-8, 400, check_every=5)
    it_q = 300
    r_q = q.primal_iterate(it_q - 5)
    assert r < 1e-8 and it + 5 <= 300, (it, r)
    assert r_q > 1e-5, r_q


def test_adjoint_is_taken_at_the_moments_of_f():
    """A prediction leaves the predicted moments in W for the next sweep;
    the adjoint linearises about f, so its start puts the moments of f back."""
    p = oracle.Problem.from_workload(I.tiny_naca(Kn=0.02, Ma=0.9), nthreads=2)
    p.set_equilibrium(1)
    p.set_acceleration(5, 20)
    p.primal_init()
    p.primal_iterate(10)                 # ends with a prediction
    v, w = p.vgrid()
    f = p.f
    Wf = np.array([oracle.moments(v, w, f[c]) for c in range(p.nc)])
    assert np.max(np.abs(p.W - Wf)) > 1e-6 * np.max(np.abs(Wf))
    p.adjoint_init()
    assert np.max(np.abs(p.W - Wf)) <= 1e-14 * np.max(np.abs(Wf))


def test_prediction_needs_the_conservative_equilibrium():
    p = oracle.Problem.from_workload(I.tiny_circle(), nthreads=1)
    with pytest.raises(ValueError):
        p.set_acceleration(5, 20)
    p.set_equilibrium(1)
    p.set_acceleration(5, 20)
    with pytest.raises(ValueError):
        p.set_equilibrium(0)


def _adjoint_case(wl, acc, tol=1e-13, max_iter=40000):
    p = oracle.Problem.from_workload(wl, nthreads=4)
    p.set_equilibrium(1)
    if acc:
        p.set_acceleration(*acc)
    p.primal_init()
    p.primal_solve(1e-14, 40000, check_every=5)
    p.adjoint_init()
    it, r = p.adjoint_solve(tol, max_iter, check_every=5)
    return p, it, r


@pytest.mark.parametrize("wl", [I.tiny_circle(Kn=0.05, Ma=0.6), I.tiny_naca(Kn=0.02, Ma=0.9)],
                         ids=lambda w: w.name)
def test_gauss_seidel_transpose(wl):
    p = oracle.Problem.from_workload(wl, nthreads=4)
    p.set_equilibrium(1)
    p.set_acceleration(5, 7)
    p.primal_init()
    p.primal_iterate(9)
    p.adjoint_init()
    rng = np.random.default_rng(11)
    r, s = rng.standard_normal((p.nc, 4)), rng.standard_normal((p.nc, 4))
    lhs, rhs = np.sum(p.macro_gs(r) * s), np.sum(r * p.macro_gs_adj(s))
    assert abs(lhs - rhs) <= 1e-13 * np.sum(np.abs(p.macro_gs(r) * s))
    # linear, and not the identity or a scaling of it
    assert np.allclose(p.macro_gs(2.0 * r), 2.0 * p.macro_gs(r), rtol=1e-14, atol=0)
    assert not np.allclose(p.macro_gs_adj(s), p.macro_gs(s))


def _wdot(w, x, y):
    return float(np.sum(w[None, :, None] * x * y))


@pytest.mark.parametrize("wl", [I.tiny_circle(Kn=0.05, Ma=0.6), I.tiny_naca(Kn=0.02, Ma=0.9)],
                         ids=lambda w: w.name)
def test_accelerated_adjoint_sweeps_transpose_the_primal_cycle(wl):
    conv = oracle.Problem.from_workload(wl, nthreads=4)
    conv.set_equilibrium(1)
    conv.primal_init()
    conv.primal_solve(1e-15, 40000)
    fs = conv.f
    _, w = conv.vgrid()
    rng = np.random.default_rng(4)
    a = rng.standard_normal(fs.shape)
    b = rng.standard_normal(fs.shape) * fs       # a relative perturbation of f
    h = 1e-6

    def sweeps(every, n, f0):
        q = oracle.Problem.from_workload(wl, nthreads=4)
        q.set_equilibrium(1)
        if every:
            q.set_acceleration(every, 6)
        q.primal_init()
        q.f = f0
        q.primal_iterate(n)
        return q.f
    u = (sweeps(0, 1, fs + h * b) - sweeps(0, 1, fs - h * b)) / (2 * h)          # P0 b
    v = (sweeps(1, 3, fs + h * b) - sweeps(1, 3, fs - h * b)) / (2 * h)          # P1 P1 P0 b
    p = oracle.Problem.from_workload(wl, nthreads=4)
    p.set_equilibrium(1)
    p.set_acceleration(1, 6)
    p.primal_init()
    p.f = fs
    p.adjoint_init()
    p.phi = a
    p.adjoint_iterate(2)
    pa = p.phi
    p.phi = np.zeros_like(a)
    p.adjoint_iterate(2)
    F = pa - p.phi                                                              # F1 F1 a
    Ru, _ = p.complex_step(u)
    Rv, _ = p.complex_step(v)
    lhs, rhs = _wdot(w, F, Ru), _wdot(w, a, Rv)
    scale = _wdot(w, np.abs(a), np.abs(Rv))
    assert abs(lhs - rhs) <= 1e-7 * scale, (lhs, rhs, scale)
    # the prediction matters here: without the correction the identity fails
    p2 = oracle.Problem.from_workload(wl, nthreads=4)
    p2.set_equilibrium(1)
    p2.primal_init()
    p2.f = fs
    p2.adjoint_init()
    p2.phi = a
    p2.adjoint_iterate(2)
    pa = p2.phi
    p2.phi = np.zeros_like(a)
    p2.adjoint_iterate(2)
    assert abs(_wdot(w, pa - p2.phi, Ru) - rhs) > 1e-4 * scale


def test_adjoint_prediction_shares_the_solution_and_accelerates():
    wl = I.tiny_circle(Kn=0.02, Ma=0.5)
    plain, it_p, r_p = _adjoint_case(wl, None)
    acc, it_a, r_a = _adjoint_case(wl, (5, 50))
    assert r_p < 1e-13 and r_a < 1e-13 and it_a < it_p / 3, (it_p, it_a)
    assert np.max(np.abs(acc.phi - plain.phi)) <= 1e-9 * np.max(np.abs(plain.phi))
    sa, sp = acc.wall_sensitivity(), plain.wall_sensitivity()
    assert np.max(np.abs(sa["dJ_dnodes"] - sp["dJ_dnodes"])) <= 1e-9 * np.max(np.abs(sp["dJ_dnodes"]))
