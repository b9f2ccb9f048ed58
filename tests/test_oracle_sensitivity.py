"""Oracle pins of the wall shape sensitivity (Sec. 3.2).

* Element derivatives (eqs. sens_J_itf, sens_B_itf with eq. gaussgrad)
  against central differences of the discrete J_l + B_w,l expressions
  (eqs. numer_J, numer_B) evaluated at perturbed element attributes with f
  and phi frozen; for the first- and the second-order scheme.
* Node transform (eq. sens_nod) against central differences of the
  element geometry (length, midpoint, unit normal into the solid) as
  functions of the two end nodes.
* Mirror symmetry: sine modes of a circle in a symmetric stream have zero
  sensitivity; mirrored bumps on a symmetric profile have equal ones.
* Agreement with finite differences of J under shape change is a
  discretisation-level trend (the paper's formula ignores volume-mesh
  motion, Sec. 2.5); the observed gap shrinks under mesh refinement.
"""
import numpy as np
import pytest

import oracle
from paper_2501_00923_amd import inputs as I


def _solved(wl, adjoint=True, order=1):
    p = oracle.Problem.from_workload(wl, nthreads=4)
    if order == 2:
        p.set_scheme(2, True, 5)
    p.primal_init()
    p.primal_solve(1e-14, 30000)
    if adjoint:
        p.adjoint_init()
        p.adjoint_solve(1e-14, 30000)
    return p


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("wl", [I.tiny_circle(Kn=1.0, Ma=0.5), I.tiny_naca(Kn=0.7, Ma=1.2)],
                         ids=lambda w: w.name)
def test_element_derivatives_match_discrete_definitions(wl, order):
    """order 2: the same formulas with the second-order scheme's values
    (reconstructed wall and face values, F_l + dF_l)."""
    p = _solved(wl, order=order)
    s = p.wall_sensitivity()
    m = p.mesh()
    for l in range(0, p.nw, 3):
        A, x, n = m["wall_A"][l], m["wall_x"][l], m["wall_n"][l]
        base = p.wall_JB(l, A, x, n)
        h = 1e-6 * max(1.0, A)
        dA = (p.wall_JB(l, A + h, x, n) - p.wall_JB(l, A - h, x, n)) / (2 * h)
        assert abs(dA - s["S_A"][l]) < 1e-8 * (abs(s["S_A"][l]) + abs(base / A) + 1e-12)
        for d in range(2):
            e = np.zeros(2)
            e[d] = 1e-6
            dx = (p.wall_JB(l, A, x + e, n) - p.wall_JB(l, A, x - e, n)) / 2e-6
            dn = (p.wall_JB(l, A, x, n + e) - p.wall_JB(l, A, x, n - e)) / 2e-6
            sc = np.max(np.abs(s["S_x"][l])) + np.max(np.abs(s["S_n"][l])) + 1e-12
            assert abs(dx - s["S_x"][l, d]) < 1e-7 * sc
            assert abs(dn - s["S_n"][l, d]) < 1e-7 * sc


def _elem_geom(a, b):
    t = b - a
    A = np.linalg.norm(t)
    return A, 0.5 * (a + b), np.array([t[1], -t[0]]) / A


def test_node_transform_matches_geometry_differences():
    wl = I.tiny_naca(Kn=0.7, Ma=1.2)
    p = _solved(wl)
    s = p.wall_sensitivity()
    g = wl.grid
    nodes = g.wall_nodes()
    nw = p.nw

    def lam(X):
        tot = 0.0
        for l in range(nw):
            A, x, n = _elem_geom(X[l], X[(l + 1) % nw])
            tot += s["S_A"][l] * A + s["S_x"][l] @ x + s["S_n"][l] @ n
        return tot
    m = p.mesh()
    for l in range(nw):                      # geometry agrees with the mesh
        A, x, n = _elem_geom(nodes[l], nodes[(l + 1) % nw])
        assert abs(A - m["wall_A"][l]) < 1e-14 and np.allclose(n, m["wall_n"][l], atol=1e-14)
    for mm in range(nw):
        for d in range(2):
            Xp, Xm = nodes.copy(), nodes.copy()
            Xp[mm, d] += 1e-7
            Xm[mm, d] -= 1e-7
            fd = (lam(Xp) - lam(Xm)) / 2e-7
            assert abs(fd - s["dJ_dnodes"][mm, d]) < 1e-6 * (np.max(np.abs(s["dJ_dnodes"])) + 1e-12)


@pytest.mark.parametrize("order", [1, 2])
def test_circle_sine_modes_have_zero_sensitivity(order):
    wl = I.tiny_circle(Kn=1.0, Ma=0.5)
    p = _solved(wl, order=order)
    s = p.wall_sensitivity()
    dJ = np.einsum("md,mdp->p", s["dJ_dnodes"], wl.grid.wall_jac)
    assert np.max(np.abs(dJ[4:])) < 1e-12 * abs(dJ[0])
    assert abs(dJ[0]) > 0.1


@pytest.mark.parametrize("order", [1, 2])
def test_symmetric_profile_mirrored_bumps_equal(order):
    h = np.array([0.3, 0.6, 0.3, 0.6])
    wl = I.tiny_naca(Kn=0.7, Ma=1.2, perturb={"kind": "hicks_henne", "h": h, "n_up": 2,
                                              "amp": np.zeros(4)})
    g = I.naca_cgrid(4, 8, 6, t=0.12, m=0.0, r_outer=4.0, h1=0.05,
                     perturb={"kind": "hicks_henne", "h": h, "n_up": 2, "amp": np.zeros(4)})
    wl.grid = g
    p = _solved(wl, order=order)
    s = p.wall_sensitivity()
    dJ = np.einsum("md,mdp->p", s["dJ_dnodes"], g.wall_jac)
    np.testing.assert_allclose(dJ[:2], dJ[2:], rtol=1e-11)


@pytest.mark.slow
def test_shape_sensitivity_fd_gap_shrinks_under_refinement():
    gaps = []
    for ni, nj in ((16, 8), (32, 16)):
        mk = lambda a: I.circle_case(ni, nj, 8, 5.0, 1.0, 0.5, 1.0, a, np.zeros(4), r_outer=5.0,
                                     stretch=1.2 ** (8.0 / nj))
        a0 = np.zeros(4)
        p = _solved(mk(a0))
        s = p.wall_sensitivity()
        adj = np.einsum("md,mdp->p", s["dJ_dnodes"], mk(a0).grid.wall_jac)[0]
        h = 1e-6
        e = np.array([h, 0, 0, 0])
        fd = (_solved(mk(a0 + e), False).objective() - _solved(mk(a0 - e), False).objective()) / (2 * h)
        gaps.append(abs(adj - fd) / abs(fd))
    assert gaps[1] < gaps[0] < 0.2
