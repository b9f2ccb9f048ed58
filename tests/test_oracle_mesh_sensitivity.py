"""Oracle pins for the exact discrete shape derivative (the Lagrangian of
Sec. 2.5 differentiated in every mesh node coordinate by complex step), for
the first-order scheme and for the second-order one (limiter factors of f
held fixed: exact with the limiter off):

- translation invariance: moving every node by the same vector changes no
  face vector, volume, normal or length, so the node derivatives sum to
  zero at any state;
- at converged primal and adjoint states, the derivative chained through
  d(nodes)/d(alpha) equals central differences of the re-converged drag
  J(alpha +- h e_p) (O-grid with Fourier modes; C-grid with Hicks-Henne
  bumps, wake cut and far field on all sides) to the finite-difference
  error, while the paper's wall-only derivative differs at the
  discretisation level."""
import numpy as np
import pytest

import oracle
from paper_2501_00923_amd import inputs as I


def _problem(g, vg, fl, order=1, limiter=False):
    o = oracle.Problem(g.topology, g.ni, g.nj, g.n_wake, g.nodes, vg.kind, vg.n1, vg.n2, vg.vmax, vg.param,
                       fl.Kn, fl.Ma, fl.Tw, fl.objective, nthreads=8)
    if order == 2:
        o.set_scheme(2, limiter, 5)
    return o


def _converge(o, adjoint=False, tol=1e-14, chunk=200, max_iter=40000):
    it = 0
    while it < max_iter:
        r = (o.adjoint_iterate if adjoint else o.primal_iterate)(chunk)
        it += chunk
        if r < tol:
            return r
    raise AssertionError(f"not converged: {r}")


def _J(make, a, vg, fl, order=1, limiter=False):
    o = _problem(make(a), vg, fl, order, limiter)
    o.primal_init()
    _converge(o)
    return o.objective()


def _exact_and_fd(make, a0, vg, fl, h, order=1, limiter=False):
    g = make(a0)
    o = _problem(g, vg, fl, order, limiter)
    o.primal_init()
    _converge(o)
    o.adjoint_init()
    _converge(o, adjoint=True)
    exact = np.einsum("jid,jidp->p", o.mesh_sensitivity(), g.node_jac)
    wall = np.einsum("md,mdp->p", o.wall_sensitivity()["dJ_dnodes"], g.wall_jac)
    fd = np.zeros(len(a0))
    for p in range(len(a0)):
        e = np.zeros(len(a0))
        e[p] = h
        fd[p] = (_J(make, a0 + e, vg, fl, order, limiter) - _J(make, a0 - e, vg, fl, order, limiter)) / (2 * h)
    return exact, wall, fd


def test_translation_invariance_at_any_state():
    wl = I.tiny_naca(nv=16, Kn=0.5, Ma=1.1)
    o = oracle.Problem.from_workload(wl, nthreads=8)
    o.primal_init()
    o.primal_iterate(17)
    o.adjoint_init()
    o.adjoint_iterate(9)
    g = o.mesh_sensitivity()
    assert np.abs(g).max() > 1e-3
    assert np.all(np.abs(g.reshape(-1, 2).sum(axis=0)) <= 1e-12 * np.abs(g).max() * g.size)


def test_exact_gradient_matches_fd_circle():
    vg = I.VGridSpec(I.VG_MIDPOINT, 16, 16, 5.0)
    fl = I.FlowSpec(1.0, 0.5)

    def make(a):
        return I.ogrid(16, 8, 5.0, 1.2, a[:4], a[4:])

    a0 = np.array([0.01, -0.02, 0.015, 0.005, 0.0, 0.01, -0.005, 0.0])
    exact, wall, fd = _exact_and_fd(make, a0, vg, fl, 1e-5)
    scale = np.abs(fd).max()
    assert np.abs(exact - fd).max() <= 1e-8 * scale
    assert np.abs(wall - fd).max() >= 1e-3 * scale      # the wall-only derivative is an approximation


def test_exact_gradient_matches_fd_naca_cgrid():
    vg = I.VGridSpec(I.VG_MIDPOINT, 16, 16, 5.0)
    fl = I.FlowSpec(0.6, 1.3)
    hs = [0.2, 0.5, 0.8, 0.3, 0.7]

    def make(a):
        return I.naca_cgrid(4, 8, 6, t=0.12, m=0.02, p=0.4, r_outer=4.0, h1=0.05,
                            perturb={"kind": "hicks_henne", "h": hs, "n_up": 3, "amp": a})

    a0 = np.array([0.004, -0.003, 0.002, 0.001, -0.002])
    exact, wall, fd = _exact_and_fd(make, a0, vg, fl, 1e-5)
    scale = np.abs(fd).max()
    assert np.abs(exact - fd).max() <= 1e-8 * scale
    assert np.abs(wall - fd).max() >= 1e-3 * scale


@pytest.mark.parametrize("limiter", [False, True], ids=["unlimited", "venkatakrishnan"])
def test_second_order_translation_invariance(limiter):
    wl = I.tiny_naca(nv=16, Kn=0.5, Ma=1.1)
    o = oracle.Problem.from_workload(wl, nthreads=8)
    o.set_scheme(2, limiter, 5)
    o.primal_init()
    o.primal_iterate(17)
    o.adjoint_init()
    o.adjoint_iterate(9)
    g = o.mesh_sensitivity()
    assert np.abs(g).max() > 1e-3
    assert np.all(np.abs(g.reshape(-1, 2).sum(axis=0)) <= 1e-12 * np.abs(g).max() * g.size)


def test_second_order_exact_gradient_matches_fd_circle():
    vg = I.VGridSpec(I.VG_MIDPOINT, 16, 16, 5.0)
    fl = I.FlowSpec(1.0, 0.5)

    def make(a):
        return I.ogrid(16, 8, 5.0, 1.2, a[:4], a[4:])

    a0 = np.array([0.01, -0.02, 0.015, 0.005, 0.0, 0.01, -0.005, 0.0])
    exact, wall, fd = _exact_and_fd(make, a0, vg, fl, 1e-5, order=2)
    scale = np.abs(fd).max()
    assert np.abs(exact - fd).max() <= 1e-8 * scale
    assert np.abs(wall - fd).max() >= 1e-3 * scale


def test_second_order_exact_gradient_matches_fd_naca_cgrid():
    """Wall, wake cut and far field on all sides; with the limiter on, the
    frozen-limiter derivative is an approximation at the percent level."""
    vg = I.VGridSpec(I.VG_MIDPOINT, 16, 16, 5.0)
    fl = I.FlowSpec(0.6, 1.3)
    hs = [0.2, 0.5, 0.8, 0.3, 0.7]

    def make(a):
        return I.naca_cgrid(4, 8, 6, t=0.12, m=0.02, p=0.4, r_outer=4.0, h1=0.05,
                            perturb={"kind": "hicks_henne", "h": hs, "n_up": 3, "amp": a})

    a0 = np.array([0.004, -0.003, 0.002, 0.001, -0.002])
    exact, _, fd = _exact_and_fd(make, a0, vg, fl, 1e-5, order=2)
    scale = np.abs(fd).max()
    assert np.abs(exact - fd).max() <= 1e-8 * scale
    exact_l, _, fd_l = _exact_and_fd(make, a0, vg, fl, 1e-5, order=2, limiter=True)
    assert np.abs(exact_l - fd_l).max() <= 0.1 * np.abs(fd_l).max()
