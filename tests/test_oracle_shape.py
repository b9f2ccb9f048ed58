"""Pins of the oracle's outer-loop pieces (Sec. 2.4 volume constraint, Sec.
3.2 eq. sens_con_nod, Sec. 3.3 CST, Sec. 3.4 RBF deformation).

Each pin fixes the oracle against something other than itself: closed
forms of special designs, the Bernstein partition of unity, recovery of a
CST surface's own parameters by the fit, the shoelace formula and the
analytic (beta-function) area of a CST profile, central differences, and the
brute-force Jacobian of the deformation.
"""

import numpy as np

from oracle import shape as S
from paper_2501_00923_amd import inputs as I

NB = 6


def _stations(n=200):
    """Cosine-clustered stations, lower surface from the trailing edge to
    the leading edge, then the upper surface back (the wall order of the
    C-grids)."""
    q = np.arange(2 * n)
    lower = q <= n
    beta = np.where(lower, np.pi * (1 - q / n), np.pi * (q - n) / n)
    xi = 0.5 * (1 - np.cos(beta))
    return xi, ~lower


def test_bernstein_partition_of_unity_and_closed_forms():
    xi = np.linspace(0, 1, 41)
    assert np.allclose(S.bernstein(NB, xi).sum(axis=1), 1.0, atol=1e-15)
    # all shape coefficients equal a: eta = a xi^N1 (1 - xi)^N2 + xi eta_T
    a, N1, N2, Tu, Tl = 0.17, 0.5, 1.0, 0.003, -0.002
    alpha = np.r_[N1, N2, np.full(NB + 1, a), np.full(NB + 1, -a), Tu, Tl]
    up = xi > 0.3
    eta = S.cst_eta(NB, alpha, xi, up)
    ref = np.where(up, a, -a) * np.sqrt(xi) * (1 - xi) + xi * np.where(up, Tu, Tl)
    assert np.max(np.abs(eta - ref)) < 1e-15
    # a single coefficient: C(xi) * binom(nb, b) xi^b (1 - xi)^(nb - b)
    alpha = np.zeros(S.n_params(NB))
    alpha[:2] = 0.7, 1.3
    alpha[2 + 2] = 1.0
    eta = S.cst_eta(NB, alpha, xi, np.ones_like(xi, dtype=bool))
    ref = xi ** 0.7 * (1 - xi) ** 1.3 * 15 * xi ** 2 * (1 - xi) ** 4
    assert np.max(np.abs(eta - ref)) < 1e-15


def test_cst_jacobian_against_central_differences():
    xi, up = _stations(40)
    rng = np.random.default_rng(1)
    alpha = np.r_[0.55, 0.9, rng.uniform(0.1, 0.2, NB + 1), -rng.uniform(0.1, 0.2, NB + 1), 0.01, -0.004]
    Jm = S.cst_jacobian(NB, alpha, xi, up)
    for p in range(S.n_params(NB)):
        h = 1e-6
        e = np.zeros_like(alpha)
        e[p] = h
        fd = (S.cst_eta(NB, alpha + e, xi, up) - S.cst_eta(NB, alpha - e, xi, up)) / (2 * h)
        assert np.max(np.abs(Jm[:, p] - fd)) < 1e-9, p
    # the leading- and trailing-edge stations do not move with N1, N2 or A
    ends = (xi == 0) | (xi == 1)
    assert np.all(Jm[ends, :2 * NB + 4] == 0)


def test_fit_recovers_a_cst_surface():
    xi, up = _stations(120)
    rng = np.random.default_rng(2)
    true = np.r_[0.62, 0.85, rng.uniform(0.1, 0.25, NB + 1), -rng.uniform(0.05, 0.2, NB + 1), 0.0, 0.0]
    eta = S.cst_eta(NB, true, xi, up)
    alpha, rms = S.cst_fit(NB, xi, up, eta)
    assert rms < 1e-12
    assert np.max(np.abs(alpha - true)) < 1e-7


def test_fit_of_naca0012_and_its_area():
    g = I.naca_cgrid(32, 96, 128)
    wall, xi, up = S.airfoil_stations(g)
    alpha, rms = S.cst_fit(NB, xi, up, wall[:, 1])
    assert rms < 5e-5                       # order-6 CST reproduces NACA0012 to ~1e-5 chord
    assert 0.3 < alpha[0] < 0.7 and 0.7 < alpha[1] < 1.3
    assert np.all(alpha[2:NB + 3] > 0) and np.all(alpha[NB + 3:2 * NB + 4] < 0)
    # NACA 4-digit area ~ 0.685 t c^2
    V = -S.volume_constraint(wall, 0.0)[0]
    assert abs(V - 0.685 * 0.12) < 2e-3


def test_volume_constraint_area_and_gradient():
    rng = np.random.default_rng(4)
    alpha = np.r_[0.5, 1.0, rng.uniform(0.1, 0.2, NB + 1), -rng.uniform(0.1, 0.2, NB + 1), 0.0, 0.0]
    exact = S.cst_area(NB, alpha)
    errs = []
    for n in (50, 100, 200):
        xi, up = _stations(n)
        P = np.stack([xi[:-1], S.cst_eta(NB, alpha, xi, up)[:-1]], axis=1)   # closed loop
        Q, dQ = S.volume_constraint(P, 0.25)
        # the loop is clockwise: Q = V_min - area
        assert abs(Q - (0.25 + S.shoelace_area(P))) < 1e-15
        assert S.shoelace_area(P) < 0
        errs.append(abs(0.25 - Q - exact))
        if n == 50:
            # Q is quadratic in the nodes, so central differences are exact
            for m in rng.choice(len(P), 8, replace=False):
                for d in range(2):
                    h = 1e-4
                    Pp, Pm = P.copy(), P.copy()
                    Pp[m, d] += h
                    Pm[m, d] -= h
                    fd = (S.volume_constraint(Pp, 0.25)[0] - S.volume_constraint(Pm, 0.25)[0]) / (2 * h)
                    assert abs(fd - dQ[m, d]) < 1e-12
    # cosine clustering of a sqrt(xi) nose: the area error falls ~4x per halving
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0
    assert errs[2] < 1e-4 * exact


def _tiny_grid():
    return I.naca_cgrid(4, 12, 8, t=0.12, r_outer=4.0, h1=0.05)


def test_rbf_interpolates_and_is_compact():
    g = _tiny_grid()
    widx = S.wall_node_index(g.topology, g.ni, g.nj, g.n_wake)
    for R in (0.5, 2.0):
        D = S.RBFDeform(g.nodes, widx, R)
        # Wendland C0 is positive definite in two dimensions
        assert np.linalg.eigvalsh(D.M).min() > 0
        rng = np.random.default_rng(5)
        d = 1e-3 * rng.standard_normal(D.c.shape)
        gamma = np.linalg.solve(D.M, d)
        # the interpolant takes the prescribed displacement at every centre
        at_c = S.wendland_c0(np.linalg.norm(D.c[:, None] - D.c[None], axis=-1) / R) @ gamma
        assert np.max(np.abs(at_c - d)) < 1e-14 * max(1.0, np.linalg.cond(D.M))
        x = D.apply(D.c + d)
        moved = np.linalg.norm(x - D.x0, axis=1) > 0
        dist = np.min(np.linalg.norm(D.x0[:, None] - D.c[None], axis=-1), axis=1)
        assert not np.any(moved & (dist >= R))
        assert np.any(moved & (widx < 0))
        # wall nodes exactly at their prescribed positions, both copies of
        # the trailing-edge node included
        on = widx >= 0
        assert np.array_equal(x[on], (D.c + d)[widx[on]])


def test_rbf_chain_is_the_transposed_jacobian():
    g = _tiny_grid()
    widx = S.wall_node_index(g.topology, g.ni, g.nj, g.n_wake)
    D = S.RBFDeform(g.nodes, widx, 1.0)
    nw = D.c.shape[0]
    Jac = np.zeros((D.x0.size, 2 * nw))       # brute force, one wall coordinate at a time
    for w in range(nw):
        for d in range(2):
            e = np.zeros_like(D.c)
            e[w, d] = 1.0
            Jac[:, 2 * w + d] = (D.apply(D.c + e) - D.apply(D.c)).ravel()
    rng = np.random.default_rng(6)
    gvec = rng.standard_normal(D.x0.shape)
    got = D.chain(gvec).ravel()
    want = Jac.T @ gvec.ravel()
    assert np.max(np.abs(got - want)) < 1e-11 * np.max(np.abs(want))


def test_fit_with_free_trailing_edge_offsets():
    xi, up = _stations(80)
    rng = np.random.default_rng(8)
    true = np.r_[0.55, 0.95, rng.uniform(0.1, 0.2, NB + 1), -rng.uniform(0.1, 0.2, NB + 1), 0.004, -0.003]
    eta = S.cst_eta(NB, true, xi, up)
    alpha, rms = S.cst_fit(NB, xi, up, eta, fixed=[])
    assert rms < 1e-12 and np.max(np.abs(alpha - true)) < 1e-7


def test_volume_constraint_normals_are_the_meshes_wall_normals():
    """The (dy, -dx) element vectors of the volume constraint are A_l n_l of
    the oracle's own mesh (normal into the solid), element by element."""
    import oracle
    for g in (I.naca_cgrid(4, 12, 8, t=0.12, r_outer=4.0, h1=0.05), I.ogrid(16, 8)):
        nw = g.ni - 2 * g.n_wake
        wall = g.nodes[0, g.n_wake:g.n_wake + nw]
        p = oracle.Problem(g.topology, g.ni, g.nj, g.n_wake, g.nodes, I.VG_MIDPOINT, 4, 4, 3.0, 0.0, 1.0, 0.5)
        m = p.mesh()
        An = m["wall_A"][:, None] * m["wall_n"]
        Q, dQ = S.volume_constraint(wall, 0.0)
        # dQ/dx_m = (A n_{m-1} + A n_m) / 2
        assert np.max(np.abs(dQ - 0.5 * (An + np.roll(An, 1, axis=0)))) < 1e-14
        # Q = -area of the body: the shoelace area of the clockwise wall
        assert abs(Q - S.shoelace_area(wall)) < 1e-14 and Q < 0
