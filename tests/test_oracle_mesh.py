"""Oracle pins: mesh connectivity and geometry (Sec. 3.1: A_ij, n_ij, V_i).

Closure sum_j A_ij n_ij = 0 for every cell, total volume equal to the
polygon area between the far-field boundary and the wall, reciprocity of
neighbour faces, wall elements with normals into the solid (Sec. 3.2).
"""
import numpy as np
import pytest

import oracle
from paper_2501_00923_amd import inputs as I


def _shoelace(P):
    x, y = P[:, 0], P[:, 1]
    return 0.5 * np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y)


CASES = [I.tiny_circle(), I.tiny_naca(), I.circle_case(32, 16, 4), I.tiny_naca(n_wake=3, n_half=6, nj=5)]


@pytest.mark.parametrize("wl", CASES, ids=lambda w: w.name)
def test_closure_volume_reciprocity(wl):
    p = oracle.Problem.from_workload(wl, nthreads=1)
    m = p.mesh()
    S, nbr, vol = m["S"], m["nbr"], m["vol"]
    per = np.sum(np.linalg.norm(S, axis=2), axis=1)
    assert np.max(np.abs(S.sum(axis=1)).max(axis=1) / per) < 1e-14
    g = wl.grid
    # boundary of the union of all cells walked counter-clockwise: j = 0
    # line (wall and both sides of any cut), i = ni line, j = nj line back,
    # i = 0 line down; the cut and the O-grid seam cancel in the sum.
    n = g.nodes
    loop = np.concatenate([n[0, :], n[1:, g.ni], n[g.nj, g.ni - 1::-1], n[g.nj - 1:0:-1, 0]])
    area = _shoelace(loop)
    assert area > 0
    assert abs(vol.sum() - abs(area)) < 1e-12 * abs(area)
    nc = p.nc
    for c in range(nc):
        for q in range(4):
            d = nbr[c, q]
            if d >= 0:
                back = [r for r in range(4) if nbr[d, r] == c]
                assert back, (c, q, d)
                assert any(np.allclose(S[d, r], -S[c, q], rtol=0, atol=1e-14) for r in back)
    # wall elements: one per wall face, normal = face normal of the wall cell
    assert np.sum(nbr <= -2) == p.nw
    np.testing.assert_allclose(np.linalg.norm(m["wall_n"], axis=1), 1.0, rtol=1e-15)
    for l in range(p.nw):
        c = m["wall_cell"][l]
        assert nbr[c, 0] == -2 - l
        np.testing.assert_allclose(m["wall_A"][l] * m["wall_n"][l], S[c, 0], rtol=0, atol=1e-15)
        # into the solid: points from the element centroid towards the body
        # side, i.e. away from the wall cell's centroid
        assert np.dot(m["wall_n"][l], m["cen"][c] - m["wall_x"][l]) < 0


def test_cgrid_wake_cut_pairs_cells():
    wl = I.tiny_naca()
    g = wl.grid
    p = oracle.Problem.from_workload(wl, nthreads=1)
    nbr = p.mesh()["nbr"]
    for i in range(g.n_wake):
        assert nbr[i, 0] == g.ni - 1 - i
        assert nbr[g.ni - 1 - i, 0] == i
    assert nbr[0, 3] == -1 and nbr[g.ni - 1, 1] == -1


def test_ogrid_periodic_and_farfield():
    wl = I.tiny_circle()
    g = wl.grid
    p = oracle.Problem.from_workload(wl, nthreads=1)
    nbr = p.mesh()["nbr"]
    for j in range(g.nj):
        assert nbr[j * g.ni, 3] == j * g.ni + g.ni - 1
        assert nbr[j * g.ni + g.ni - 1, 1] == j * g.ni
    assert np.all(nbr[(g.nj - 1) * g.ni:, 2] == -1)


def test_invalid_mesh_rejected():
    g = I.tiny_circle().grid
    bad = g.nodes[:, ::-1].copy()                 # reversed walk -> negative areas
    with pytest.raises(ValueError):
        oracle.Problem(g.topology, g.ni, g.nj, 0, bad, 0, 8, 8, 5.0, 0.0, 1.0, 0.5)
