"""Pins of the oracle's Green-Gauss wall-cell gradient (Sec. 3.2, eq.
gaussgrad) with the first-order scheme's upwind face values.

On a grid of equal parallelograms (cell centroids a lattice with edge
vectors e1, e2; face vectors S_E = -S_W, S_N = -S_S; volume |e1 x e2|), the
upwind Green-Gauss sum (1/V) sum_q f_q S_q takes, on each pair of opposite
faces, the neighbour value on the inflow face and the cell's own on the
outflow face, so it equals (1/V) sum over the two inflow faces of
(f_nbr - f_c) S_q, a one-sided difference.  Closed forms follow:

* a linear field f = a + b.x gives exactly b (the identity
  e1 S_E^T + e2 S_N^T = V I of a parallelogram);
* on a Cartesian grid of spacing h, a quadratic field gives the textbook
  upwind-difference error: grad f(x_c) - (h/2) (f_xx sgn v1, f_yy sgn v2);
* at a wall cell, the inflow value of the wall face is the diffuse value
  F_l gbar_k (eq. barg); a field linear in y whose incoming-velocity values
  continue, at the mirror cell below the wall, to exactly F_l gbar_k keeps the
  gradient exact there as well.

A wrong face choice (downwind or central: those differ on the quadratic),
a sign of S, the volume, a swapped component or direction index, or the
wrong wall value on either side of the wall face fails one of these.
"""
import numpy as np

import oracle

NI, NJ, H = 10, 5, 0.3


def _problem(shear):
    """C-grid block (one wake cell at either end) of equal parallelograms
    with the wall on y = 0: nodes (i h + j s, j h)."""
    nodes = np.zeros((NJ + 1, NI + 1, 2))
    for j in range(NJ + 1):
        for i in range(NI + 1):
            nodes[j, i] = (i * H + j * shear, j * H)
    p = oracle.Problem(1, NI, NJ, 1, nodes, 0, 8, 8, 5.0, 0.0, 0.5, 0.7, 1.3, 0, nthreads=2)
    return p


def _centroids(p):
    return p.mesh()["cen"]


def test_linear_field_exact_on_parallelograms():
    p = _problem(0.11)
    cen = _centroids(p)
    rng = np.random.default_rng(1)
    nv = p.nv
    a = rng.uniform(1.0, 2.0, (nv, 2))
    b = rng.normal(0.0, 1.0, (nv, 2, 2))          # gradient [k, component, direction]
    f = a[None] + np.einsum("kmd,cd->ckm", b, cen)
    p.f = f
    for j in range(1, NJ - 1):
        for i in range(1, NI - 1):
            g = p.gauss_grad(i + NI * j)
            assert np.max(np.abs(g - b)) <= 1e-13 * np.max(np.abs(b)), (i, j)


def test_quadratic_field_upwind_error_on_cartesian_grid():
    p = _problem(0.0)
    cen = _centroids(p)
    v, _ = p.vgrid()
    rng = np.random.default_rng(2)
    nv = p.nv
    a = rng.uniform(1.0, 2.0, (nv, 2))
    b = rng.normal(0.0, 1.0, (nv, 2, 2))
    Hs = rng.normal(0.0, 1.0, (nv, 2, 2, 2))
    Hs = 0.5 * (Hs + np.swapaxes(Hs, 2, 3))       # symmetric Hessian per velocity and component
    f = a[None] + np.einsum("kmd,cd->ckm", b, cen) + 0.5 * np.einsum("cd,kmde,ce->ckm", cen, Hs, cen)
    p.f = f
    sg = np.sign(v)                                # no velocity node has a zero component
    for j in range(1, NJ - 1):
        for i in range(1, NI - 1):
            c = i + NI * j
            grad = b + np.einsum("kmde,e->kmd", Hs, cen[c])
            diag = np.stack([Hs[:, :, 0, 0], Hs[:, :, 1, 1]], axis=-1)
            want = grad - 0.5 * H * diag * sg[:, None, :]
            g = p.gauss_grad(c)
            assert np.max(np.abs(g - want)) <= 1e-12 * np.max(np.abs(want)), (i, j)


def test_wall_cell_gradient_with_the_diffuse_wall_value():
    shear = 0.11
    p = _problem(shear)
    cen = _centroids(p)
    v, _ = p.vgrid()
    rng = np.random.default_rng(3)
    nv = p.nv
    beta = rng.normal(0.0, 1.0, (nv, 2))           # d f / d y per velocity and component
    a = rng.uniform(1.0, 2.0, (nv, 2))
    y = cen[:, 1]
    out = v[:, 1] < 0                              # towards the wall (v . n > 0, n = (0, -1)): Xi^+
    p.f = a[None] + beta[None] * y[:, None, None]
    D, F = p.wall()
    # every wall cell has the same y and normal, hence the same F_l; set the
    # incoming-velocity values so that the field continued to the mirror
    # cell below the wall (y = -h/2) is the diffuse wall value there
    assert np.max(np.abs(F - F[0])) <= 1e-14 * abs(F[0])
    th_w = p.flow()["theta_w"]
    gM = oracle.maxwell(1.0, 0.0, 0.0, th_w, v)[:, 0]
    gbar1 = gM / D[0]
    wall_val = np.stack([F[0] * gbar1, F[0] * 0.5 * th_w * gbar1], axis=-1)
    a_in = wall_val + 0.5 * H * beta
    a = np.where(out[:, None], a, a_in)
    p.f = a[None] + beta[None] * y[:, None, None]
    D2, F2 = p.wall()
    assert np.array_equal(F2, F)                   # F sums the outgoing velocities only
    want = np.zeros((nv, 2, 2))
    want[:, :, 1] = beta
    m = p.mesh()
    for l in range(p.nw):
        c = int(m["wall_cell"][l])
        g = p.gauss_grad(c)
        assert np.max(np.abs(g - want)) <= 1e-12 * np.max(np.abs(beta)), l
