"""Oracle pins: velocity quadrature, reduced Maxwellian, dg/dW.

Velocity grids (Sec. 2.2: d Xi = dv1 dv2) must integrate what their rule
class guarantees; the reduced Maxwellian of eq. (maxwell_reduce) must carry
the moments (rho, rho u, rho |u|^2/2 + 3/2 rho RT) that eq. (macint_reduce)
and the specific energy of Sec. 2.1 with gamma = 5/3 fix.
"""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("kind,n,vmax,param", [(0, 16, 5.0, 0.0), (0, 48, 6.0, 0.0),
                                               (1, 48, 6.0, 0.0), (1, 8, 3.0, 0.0),
                                               (2, 64, 6.0, 2.0)])
def test_quadrature_symmetry_and_length(kind, n, vmax, param):
    x, w = oracle.vgrid_1d(kind, n, vmax, param)
    assert np.all(np.diff(x) > 0)
    np.testing.assert_allclose(x, -x[::-1], rtol=0, atol=1e-15 * vmax)
    np.testing.assert_allclose(w, w[::-1], rtol=1e-15, atol=0)
    assert np.all(np.abs(x) > 0)                          # no node at v = 0
    assert abs(w.sum() - 2 * vmax) <= 1e-13 * vmax
    assert abs(np.sum(w * x)) <= 1e-14 * vmax ** 2
    assert abs(np.sum(w * x ** 3)) <= 1e-13 * vmax ** 4


@pytest.mark.parametrize("n", [8, 16, 48])
def test_newton_cotes_exact_to_degree_3(n):
    # composite Simpson + 3/8 is exact for cubics on every panel
    x, w = oracle.vgrid_1d(1, n, 2.5, 0.0)
    for deg in range(4):
        exact = (2.5 ** (deg + 1) - (-2.5) ** (deg + 1)) / (deg + 1)
        assert abs(np.sum(w * x ** deg) - exact) <= 1e-13 * max(1.0, abs(exact))
    # a shifted cubic too (not odd/even)
    f = lambda t: 3 * t ** 3 - t ** 2 + 0.5 * t + 2
    F = lambda t: 0.75 * t ** 4 - t ** 3 / 3 + 0.25 * t ** 2 + 2 * t
    assert abs(np.sum(w * f(x)) - (F(2.5) - F(-2.5))) < 1e-12


def test_newton_cotes_rejects_unsupported_count():
    with pytest.raises(ValueError):
        oracle.vgrid_1d(1, 10, 3.0, 0.0)


def test_sinh_grid_denser_near_origin():
    x, w = oracle.vgrid_1d(2, 64, 6.0, 2.0)
    assert w[32] < w[0] / 3
    # mapped-cell rule: second-order convergence on a Gaussian
    errs = []
    for n in (32, 64, 128):
        xx, ww = oracle.vgrid_1d(2, n, 6.0, 2.0)
        errs.append(abs(np.sum(ww * np.exp(-xx ** 2)) - np.sqrt(np.pi)))
    assert errs[1] < 5e-4 and 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def _grid2d(kind, n, vmax, param=0.0):
    x, w = oracle.vgrid_1d(kind, n, vmax, param)
    v1, v2 = np.meshgrid(x, x, indexing="xy")
    v = np.stack([v1.ravel(), v2.ravel()], axis=1)
    wt = np.outer(w, w).ravel()
    return v, wt


@pytest.mark.parametrize("rho,u1,u2,th", [(1.0, 0.0, 0.0, 0.5), (1.3, 0.45, -0.2, 0.6),
                                          (0.7, -0.9, 0.3, 0.35)])
def test_maxwellian_moments_closed_form(rho, u1, u2, th):
    # a wide, fine midpoint grid integrates a Gaussian spectrally
    v, w = _grid2d(0, 160, 9.0)
    g = oracle.maxwell(rho, u1, u2, th, v)
    W = oracle.moments(v, w, g)
    exact = np.array([rho, rho * u1, rho * u2, 0.5 * rho * (u1 * u1 + u2 * u2) + 1.5 * rho * th])
    np.testing.assert_allclose(W, exact, rtol=1e-11, atol=1e-12)
    # g2 = RT/2 g1 exactly (eq. maxwell_reduce)
    np.testing.assert_allclose(g[:, 1], 0.5 * th * g[:, 0], rtol=1e-15)
    # second moments: pressure tensor rho*th*I + rho u u
    P11 = np.sum(w * v[:, 0] ** 2 * g[:, 0])
    assert abs(P11 - (rho * th + rho * u1 * u1)) < 1e-10


def test_conservation_defect_recorded_on_coarse_grid():
    """The BGK collision term conserves W only to quadrature error on a
    finite grid (pointwise discrete Maxwellian); record its size on the
    circle workload's 16x16 grid on [-5, 5] at Ma 0.5."""
    v, w = _grid2d(0, 16, 5.0)
    u = 0.5 * np.sqrt(5.0 / 6.0)
    g = oracle.maxwell(1.0, u, 0.0, 0.5, v)
    W = oracle.moments(v, w, g)
    exact = np.array([1.0, u, 0.0, 0.5 * u * u + 0.75])
    defect = np.max(np.abs(W - exact))
    assert defect < 1e-6


def _prim(W):
    rho = W[0]
    u1, u2 = W[1] / rho, W[2] / rho
    th = (2.0 / 3.0) * (W[3] / rho - 0.5 * (u1 * u1 + u2 * u2))
    return rho, u1, u2, th


@pytest.mark.parametrize("W", [np.array([1.0, 0.3, -0.1, 1.0]), np.array([0.6, -0.5, 0.2, 0.9])])
def test_dg_dW_and_dtau_dW_by_central_differences(W):
    rho, u1, u2, th = _prim(W)
    for v1, v2 in [(0.4, -1.2), (-2.0, 0.7), (1.5, 1.5)]:
        dg, dtt = oracle.dg_dW(rho, u1, u2, th, v1, v2)
        for m in range(4):
            h = 1e-6
            Wp, Wm = W.copy(), W.copy()
            Wp[m] += h
            Wm[m] -= h
            gp = oracle.maxwell(*_prim(Wp), np.array([[v1, v2]]))[0]
            gm = oracle.maxwell(*_prim(Wm), np.array([[v1, v2]]))[0]
            fd = (gp - gm) / (2 * h)
            np.testing.assert_allclose(dg[:, m], fd, rtol=1e-8, atol=1e-11)
            # tau ~ 1/(rho sqrt(theta)) (hard sphere, Sec. 2.1)
            tp = 1.0 / (_prim(Wp)[0] * np.sqrt(_prim(Wp)[3]))
            tm = 1.0 / (_prim(Wm)[0] * np.sqrt(_prim(Wm)[3]))
            t0 = 1.0 / (rho * np.sqrt(th))
            assert abs(dtt[m] - (tp - tm) / (2 * h) / t0) < 1e-8
