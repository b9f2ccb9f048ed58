"""Oracle pins of the second-order scheme (Sec. 3.1 states second-order
accuracy in physical space for the primal and adjoint balances; the
reconstruction, limiter and iteration are readings, stated in the oracle's
header of that part).

* Green-Gauss slopes are exact for a linear field on a grid of equal
  parallelograms (the face mean of the two cell values is then the value at
  the face midpoint), the limiter factor of a linear field is 1, and
  the reconstructed face values are the field's values at the face
  midpoints.
* Venkatakrishnan limiter: a limited face value leaves the range of the
  cell and its interior neighbours by at most e / (2 sqrt 2), e = 1e-3 |f_c|
  (a bound derived from the limiter function), and psi moves smoothly with f.
* Defect correction: the converged state solves the second-order balance
  R2 = 0 and does not depend on the correction interval K.
* Order of accuracy: under refinement of the circle's O-grid the drag's
  successive differences shrink about 4x per halving for order 2 and 2x for
  order 1.
* Adjoint: dot-product identity of the frozen-limiter adjoint operator
  against a complex-step linearisation of an independently written
  complex twin of R2 and J; with the limiter off, dJ/dp from the adjoint
  equals central finite differences of re-converged order-2 drags.
"""
import numpy as np
import pytest

import oracle
from paper_2501_00923_amd import inputs as I


def _problem(wl, limiter=True, K=5, **kw):
    p = oracle.Problem.from_workload(wl, nthreads=4, **kw)
    p.set_scheme(2, limiter, K)
    return p


def _corners(nodes, i, j):
    return np.array([nodes[j, i], nodes[j, i + 1], nodes[j + 1, i + 1], nodes[j + 1, i]])


def test_linear_field_is_reconstructed_exactly():
    # equal parallelograms, O-grid connectivity (seam and ring boundaries
    # only affect cells next to them, which are left out)
    ni, nj, h1, h2, sh = 12, 9, 0.3, 0.2, 0.35
    jj, ii = np.meshgrid(np.arange(nj + 1), np.arange(ni + 1), indexing="ij")
    nodes = np.stack([1.0 + ii * h1 + jj * h2 * sh, 2.0 + jj * h2], axis=-1)
    p = oracle.Problem(I.TOPO_O, ni, nj, 0, nodes, I.VG_MIDPOINT, 4, 4, 3.0, 0.0, 1.0, 0.5)
    p.set_scheme(2, True, 5)
    cen = p.mesh()["cen"]
    rng = np.random.default_rng(3)
    a = rng.uniform(1.0, 2.0, (p.nv, 2))
    b = rng.standard_normal((p.nv, 2, 2))
    f = a[None] + np.einsum("kmd,cd->ckm", b, cen)
    G, psi = p.so_slopes(f)
    faces = p.so_faces(f)
    for j in range(1, nj - 1):
        for i in range(1, ni - 1):
            c = i + ni * j
            assert np.max(np.abs(G[c] - b)) < 1e-12 * np.max(np.abs(b))
            assert np.all(psi[c] >= 1.0 - 1e-14)
            if 2 <= i <= ni - 3 and 2 <= j <= nj - 3:
                Q = _corners(nodes, i, j)
                for q in range(4):
                    mid = 0.5 * (Q[q] + Q[(q + 1) % 4])
                    exact = a + np.einsum("kmd,d->km", b, mid)
                    assert np.max(np.abs(faces[c, q] - exact)) < 1e-13 * np.max(np.abs(exact))


KAPPA = 1e-3      # Venkatakrishnan smoothing relative to the cell value


@pytest.mark.parametrize("wl", [I.tiny_circle(), I.tiny_naca()], ids=lambda w: w.name)
def test_limiter_bounds_and_smoothness(wl):
    """Venkatakrishnan: with D the room to the neighbourhood's max (min) and
    d the unlimited increment, phi d - D = (e^2 (d - D) - D^3) / den with
    den >= 2 d^2 + e^2, so a limited face value leaves [lo, hi] by at most
    e / (2 sqrt 2), e = kappa |f_c|; and psi is a smooth function of f."""
    p = _problem(wl)
    m = p.mesh()
    nbr, cen = m["nbr"], m["cen"]
    g = wl.grid
    rng = np.random.default_rng(5)
    f = np.exp(rng.standard_normal((p.nc, p.nv, 2)))
    G, psi = p.so_slopes(f)
    assert np.all(psi >= 0.0) and np.all(psi <= 1.0)
    assert np.mean(psi < 0.5) > 0.3          # a rough field is limited strongly in many cells
    for c in range(p.nc):
        i, j = c % g.ni, c // g.ni
        Q = _corners(g.nodes, i, j)
        mids = 0.5 * (Q + np.roll(Q, -1, axis=0))
        nb = [n for n in nbr[c] if n >= 0]
        lo = np.minimum(f[c], f[nb].min(axis=0))
        hi = np.maximum(f[c], f[nb].max(axis=0))
        vals = f[c][None] + np.einsum("kmd,qd->qkm", G[c], mids - cen[c])    # [q, k, m]
        slack = KAPPA * np.abs(f[c])[None] / (2 * np.sqrt(2)) * (1 + 1e-9) + 1e-14 * np.abs(f[c]).max()
        assert np.all(vals >= lo[None] - slack) and np.all(vals <= hi[None] + slack)
    # smooth: a relative perturbation of 1e-12 moves psi by O(1e-12 / kappa) at most
    f2 = f * (1 + 1e-12 * rng.standard_normal(f.shape))
    _, psi2 = p.so_slopes(f2)
    assert np.max(np.abs(psi2 - psi)) < 1e-7


@pytest.mark.parametrize("wl", [I.tiny_circle(Kn=1.0, Ma=0.5), I.tiny_naca(Kn=0.7, Ma=1.2)],
                         ids=lambda w: w.name)
def test_defect_correction_fixed_point(wl):
    Js = []
    for K in (3, 5, 10):
        p = _problem(wl, limiter=False, K=K)
        p.primal_init()
        it, r = p.primal_solve(1e-14, 20000, 100)
        assert r < 1e-14
        R = p.primal_residual()
        assert np.max(np.abs(R)) < 1e-13 * np.max(np.abs(p.f))
        Js.append(p.objective())
    assert max(Js) - min(Js) < 1e-12 * abs(Js[0])
    q = oracle.Problem.from_workload(wl, nthreads=4)
    q.primal_init()
    q.primal_solve(1e-14, 20000, 100)
    assert abs(q.objective() - Js[0]) > 1e-3 * abs(Js[0])     # the reconstruction is active
    # with the (smooth) limiter the iteration converges as well, to a state
    # that differs from the unlimited one
    p = _problem(wl, limiter=True, K=5)
    p.primal_init()
    it, r = p.primal_solve(1e-14, 20000, 100)
    assert r < 1e-14
    assert np.max(np.abs(p.primal_residual())) < 1e-13 * np.max(np.abs(p.f))
    assert abs(p.objective() - Js[0]) > 1e-5 * abs(Js[0])


def test_grid_convergence_order():
    Cd = {}
    for ni, nj in ((16, 8), (32, 16), (64, 32)):
        wl = I.circle_case(ni=ni, nj=nj, nv=8, Kn=1.0, Ma=0.5)
        for order in (1, 2):
            p = oracle.Problem.from_workload(wl, nthreads=8)
            p.set_scheme(order, False, 5)
            p.primal_init()
            it, r = p.primal_solve(1e-12, 20000, 100)
            assert r < 1e-12
            Cd[(ni, order)] = p.objective() / p.cd_scale()
    ratio = {o: (Cd[(16, o)] - Cd[(32, o)]) / (Cd[(32, o)] - Cd[(64, o)]) for o in (1, 2)}
    assert 1.6 < ratio[1] < 2.4, ratio
    assert 3.4 < ratio[2] < 6.0, ratio


@pytest.mark.parametrize("limiter", [False, True], ids=["unlimited", "venkatakrishnan"])
@pytest.mark.parametrize("wl", [I.tiny_circle(Kn=1.0, Ma=0.5), I.tiny_naca(Kn=0.7, Ma=1.2)],
                         ids=lambda w: w.name)
def test_adjoint_dot_product_identity(wl, limiter):
    p = _problem(wl, limiter=limiter)
    p.primal_init()
    p.primal_iterate(600)
    p.adjoint_init()                          # freezes the limiter factors of this f
    rng = np.random.default_rng(7)
    u = rng.standard_normal((p.nc, p.nv, 2))
    phi = rng.standard_normal((p.nc, p.nv, 2))
    _, w = p.vgrid()
    W = w[None, :, None]
    dR, dJ = p.complex_step(u)
    lhs = np.sum(W * phi * dR)
    rhs = np.sum(W * u * p.adjoint_operator(phi, with_source=False))
    assert abs(lhs - rhs) < 1e-13 * np.sum(np.abs(W * phi * dR))
    # the objective's part of the operator is dJ/df
    src = np.sum(W * u * (p.adjoint_operator(phi, True) - p.adjoint_operator(phi, False)))
    assert abs(src - dJ) < 1e-12 * max(abs(dJ), 1.0)
    # the frozen-limiter adjoint iteration converges to the operator's zero
    p.adjoint_init()
    it, r = p.adjoint_solve(1e-14, 20000, 100)
    assert r < 1e-14
    assert np.max(np.abs(p.adjoint_operator(p.phi))) < 1e-12 * np.max(np.abs(p.phi))


@pytest.mark.parametrize("which,name", [(oracle.KN, "Kn"), (oracle.MA, "Ma"), (oracle.TW, "Tw")])
def test_adjoint_gradient_matches_finite_differences(which, name):
    wl = I.tiny_circle(Kn=1.0, Ma=0.5)
    p = _problem(wl, limiter=False)
    p.primal_init()
    p.primal_solve(1e-15, 30000, 100)
    p.adjoint_init()
    p.adjoint_solve(1e-15, 30000, 100)
    h = 1e-5
    base = {"Kn": wl.flow.Kn, "Ma": wl.flow.Ma, "Tw": wl.flow.Tw}[name]
    Js = []
    for sgn in (1, -1):
        q = _problem(wl, limiter=False, **{name: base + sgn * h})
        q.primal_init()
        q.primal_solve(1e-15, 30000, 100)
        Js.append(q.objective())
    fd = (Js[0] - Js[1]) / (2 * h)
    assert abs(p.adjoint_dJdp(which) - fd) < 1e-8 * abs(fd)
