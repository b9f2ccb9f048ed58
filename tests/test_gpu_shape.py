"""GPU parity of the optimisation's outer loop (Sec. 3.4): the RBF mesh
motion and its transpose against the oracle, the whole SLSQP loop against
the oracle's loop, and the exact design gradient against finite
differences of re-converged drags."""
import numpy as np
import pytest

from oracle import shape as OS
from paper_2501_00923_amd import dvm, inputs as I

pytestmark = pytest.mark.gpu


def _grids():
    return [("tiny_c", I.naca_cgrid(4, 12, 8, t=0.12, r_outer=4.0, h1=0.05), 1.0),
            ("small_c", I.naca_cgrid(4, 24, 10, t=0.12, r_outer=4.0, h1=0.02), 0.5),
            ("c256x128", I.naca_cgrid(32, 96, 128), 2.0),
            ("o64x32", I.ogrid(64, 32), 3.0),
            # walls of 400 and 301 nodes: the host factor of the RBF system
            # then runs threaded, over several column blocks, with ragged edges
            ("c_wall400", I.naca_cgrid(8, 200, 16, t=0.12, r_outer=4.0, h1=0.01), 1.5),
            ("o301x8", I.ogrid(301, 8), 2.0)]


def _deform_parity(name, g, R, cond=None):
    from paper_2501_00923_amd.shape import Deformer
    print(f"[deform] {name} R={R}", flush=True)
    mesh = dvm.Mesh.from_grid(g)
    D = Deformer(mesh, R)
    O = OS.RBFDeform(g.nodes, OS.wall_node_index(g.topology, g.ni, g.nj, g.n_wake), R)
    rng = np.random.default_rng(11)
    scale = np.max(np.abs(g.nodes))
    # the weights solve M gamma = d: both sides agree to about cond(M) eps
    # relative (Cholesky here, LU in the oracle)
    kappa = (np.linalg.cond(O.M) if cond is None else cond(O.M)) * np.finfo(np.float64).eps
    for call in range(2):                                     # two calls in a row, different inputs
        c = O.c
        if call == 0:                                         # rough: independent normal offsets
            d = 2e-3 * rng.standard_normal(c.shape)
        else:                                                 # smooth, as a design change moves a wall
            d = 5e-4 * np.stack([np.sin(3 * c[:, 0] + 1) * np.cos(2 * c[:, 1]), np.cos(2 * c[:, 0]) + c[:, 1]], 1)
        wall = c + d
        x = D.apply(wall)
        xo = O.apply(wall).reshape(x.shape)
        assert np.max(np.abs(x - xo)) < 1e-14 * scale + 4 * kappa * np.max(np.abs(d)), call
        assert np.array_equal(x[0, g.n_wake:g.n_wake + mesh.nw], wall)
        gvec = rng.standard_normal(x.shape)
        h = D.chain(gvec)
        ho = O.chain(gvec)
        assert np.max(np.abs(h - ho)) < max(1e-13, 4 * kappa) * np.max(np.abs(ho)), call
    # the moved mesh is a valid mesh
    dvm.Mesh(g.topology, g.ni, g.nj, g.n_wake, x)


@pytest.mark.parametrize("name,g,R", _grids(), ids=[x[0] for x in _grids()])
def test_deform_apply_and_chain_match_oracle(name, g, R):
    _deform_parity(name, g, R)


def test_deform_at_the_wall_node_limit():
    """8192 wall nodes, the most the library takes.  The wall is a circle of
    equally spaced nodes, so the RBF matrix is circulant and its condition
    number is exactly that of the FFT of one row."""
    g = I.ogrid(8192, 1, r_outer=2.0)
    assert dvm.Mesh.from_grid(g).nw == 8192

    def circulant_cond(M):
        lam = np.abs(np.fft.fft(M[0]).real)
        return lam.max() / lam.min()
    _deform_parity("o8192x1", g, 1.5, circulant_cond)


def _small_workload(Kn=1.0):
    g = I.naca_cgrid(4, 24, 10, t=0.12, r_outer=4.0, h1=0.02)
    return I.Workload("small_naca", g, I.VGridSpec(I.VG_MIDPOINT, 8, 8, 5.0), I.FlowSpec(Kn, 0.5, 1.0), 0)


@pytest.mark.parametrize("gradient", ["paper", "exact"])
def test_optimiser_matches_oracle_loop(gradient):
    from paper_2501_00923_amd.optimize import ShapeOptimizer
    print(f"[optimise] small_naca gradient={gradient}", flush=True)
    wl = _small_workload()
    ro = OS.optimise(wl, radius=1.0, sigma=0.1, max_steps=3, gradient=gradient, solve_tol=1e-12, nthreads=8)
    opt = ShapeOptimizer(wl, radius=1.0, sigma=0.1, gradient=gradient, solve_tol=1e-12, warm_start=False)
    r = opt.run(max_steps=3)
    assert abs(r["v_min"] - ro["v_min"]) < 1e-15
    assert np.max(np.abs(r["alpha0"] - ro["alpha0"])) < 1e-9
    assert len(r["history"]) == len(ro["history"]) == 4
    for e, (ao, Jo, Qo) in zip(r["history"], ro["history"]):
        assert abs(e.J - Jo) < 1e-9 * abs(Jo)
        assert np.max(np.abs(e.alpha - ao)) < 1e-7
        assert abs(e.Q - Qo) < 1e-9 * ro["v_min"]
    assert r["history"][-1].J < r["history"][0].J
    # warm-started solves (the default) follow the same path
    rw = ShapeOptimizer(wl, radius=1.0, sigma=0.1, gradient=gradient, solve_tol=1e-12).run(max_steps=3)
    for e, f in zip(rw["history"], r["history"]):
        assert abs(e.J - f.J) < 1e-9 * abs(f.J)


def test_exact_design_gradient_matches_finite_differences():
    from paper_2501_00923_amd.optimize import ShapeOptimizer
    print("[optimise] exact gradient vs FD", flush=True)
    wl = _small_workload(Kn=0.5)
    opt = ShapeOptimizer(wl, radius=1.0, gradient="exact", solve_tol=1e-14, warm_start=False)
    a0 = opt.alpha0
    dJ = opt.evaluate(a0).dJ
    nb = opt.nb
    for p in (0, 1, 2 + 3, nb + 3 + 2):
        h = 1e-6
        e = np.zeros_like(a0)
        e[p] = h
        Jp = opt.evaluate(a0 + e, gradient=False).J
        Jm = opt.evaluate(a0 - e, gradient=False).J
        fd = (Jp - Jm) / (2 * h)
        assert abs(fd - dJ[p]) < 2e-6 * np.max(np.abs(dJ)), (p, fd, dJ[p])


def test_state_copy_matches_save_and_load():
    print("[state copy] device-to-device vs host round trip", flush=True)
    from paper_2501_00923_amd.shape import Deformer
    wl = _small_workload()
    g, vg, fl = wl.grid, wl.vgrid, wl.flow
    mesh = dvm.Mesh.from_grid(g)
    D = Deformer(mesh, 1.0)
    wall = g.nodes[0, g.n_wake:g.n_wake + mesh.nw]
    moved = D.apply(wall + np.stack([np.zeros(mesh.nw), 1e-3 * np.sin(np.pi * wall[:, 0])], 1))
    V = dvm.VGrid.from_spec(vg)

    def solver(nodes):
        return dvm.Solver(dvm.Mesh(g.topology, g.ni, g.nj, g.n_wake, nodes), V, fl.Kn, fl.Ma, fl.Tw)

    s1, s2, s3 = solver(g.nodes), solver(moved), solver(moved)
    s1.primal_init()
    s1.primal_sweeps(200)
    s1.adjoint_init()
    s1.adjoint_sweeps(100)
    s2.state_copy_from(s1, dvm.STATE_F)
    s3.state_load(dvm.STATE_F, s1.state_save(dvm.STATE_F))
    assert np.array_equal(s2.state_save(dvm.STATE_F), s3.state_save(dvm.STATE_F))
    assert np.array_equal(s2.moments(), s3.moments())
    for s in (s2, s3):
        s.primal_sweeps(10)
        s.adjoint_init()
    assert np.array_equal(s2.moments(), s3.moments())
    s2.state_copy_from(s1, dvm.STATE_PHI)
    s3.state_load(dvm.STATE_PHI, s1.state_save(dvm.STATE_PHI))
    for s in (s2, s3):
        s.adjoint_sweeps(10)
    assert np.array_equal(s2.state_save(dvm.STATE_PHI), s3.state_save(dvm.STATE_PHI))
    # refused: different grid size; phi into a solver not in the adjoint phase
    other = dvm.Solver.from_workload(I.tiny_naca())
    other.primal_init()
    with pytest.raises(dvm.DvmError):
        other.state_copy_from(s1, dvm.STATE_F)
    s4 = solver(moved)
    s4.primal_init()
    with pytest.raises(dvm.DvmError):
        s4.state_copy_from(s1, dvm.STATE_PHI)


@pytest.mark.parametrize("gradient", ["paper", "exact"])
def test_second_order_optimiser_matches_oracle_loop(gradient):
    """The loop with the second-order scheme (limited reconstruction,
    correction every 40 sweeps), with the paper's wall-node gradient with the
    second-order values or the exact one (limiter factors fixed); every
    solve runs to the same sweep cap or tolerance on both sides."""
    from paper_2501_00923_amd.optimize import ShapeOptimizer
    print(f"[optimise] small_naca second order gradient={gradient}", flush=True)
    wl = _small_workload()
    ro = OS.optimise(wl, radius=1.0, sigma=0.1, max_steps=3, solve_tol=1e-11, max_sweeps=6000, nthreads=8,
                     order=2, correction_every=40, gradient=gradient)
    opt = ShapeOptimizer(wl, radius=1.0, sigma=0.1, solve_tol=1e-11, max_sweeps=6000, warm_start=False, order=2,
                         gradient=gradient)
    r = opt.run(max_steps=3)
    assert len(r["history"]) == len(ro["history"])
    for e, (ao, Jo, Qo) in zip(r["history"], ro["history"]):
        assert abs(e.J - Jo) < 1e-9 * abs(Jo)
        assert np.max(np.abs(e.alpha - ao)) < 1e-7


def test_full_optimisation_matches_oracle():
    """A whole optimisation, to the 3e-5 stopping test of eq. (criterion_opt),
    on the library and on the oracle: same number of steps, same optimum."""
    from paper_2501_00923_amd.optimize import ShapeOptimizer
    print("[optimise] small_naca to the stopping test", flush=True)
    wl = _small_workload()
    ro = OS.optimise(wl, radius=1.0, sigma=0.1, max_steps=20, solve_tol=1e-12, nthreads=8)
    r = ShapeOptimizer(wl, radius=1.0, sigma=0.1, solve_tol=1e-12).run(max_steps=20)
    assert ro["converged"] and r["converged"]
    assert len(r["history"]) == len(ro["history"])
    Jf, Jo = r["history"][-1].J, ro["history"][-1][1]
    assert abs(Jf - Jo) < 1e-8 * abs(Jo)
    assert np.max(np.abs(r["history"][-1].alpha - ro["history"][-1][0])) < 1e-5
    assert Jf < 0.97 * r["history"][0].J


def test_mixed_precision_optimiser_follows_fp64():
    """FP32 f and phi (FP64 moments, J and sensitivities) in every solve of
    the loop: the same design path as FP64, J within the mixed solves'
    accuracy."""
    from paper_2501_00923_amd.optimize import ShapeOptimizer
    print("[optimise] small_naca mixed vs fp64", flush=True)
    wl = _small_workload()
    r64 = ShapeOptimizer(wl, radius=1.0, sigma=0.1, solve_tol=1e-7).run(max_steps=3)
    r32 = ShapeOptimizer(wl, radius=1.0, sigma=0.1, solve_tol=1e-7, precision=dvm.MIXED,
                         max_sweeps=20000).run(max_steps=3)
    assert len(r32["history"]) == len(r64["history"])
    for a, b in zip(r32["history"], r64["history"]):
        assert abs(a.J - b.J) < 1e-5 * abs(b.J)
        assert np.max(np.abs(a.alpha - b.alpha)) < 1e-3


@pytest.mark.parametrize("exact", [False, True], ids=["wall_nodes", "exact"])
def test_autograd_cst_case_matches_oracle(exact):
    """drag(alpha) over the CST design with the RBF motion: forward J and
    backward dJ/dalpha against the oracle's solve on the same moved mesh."""
    import torch
    from paper_2501_00923_amd import autograd as AG
    print(f"[autograd] CST case exact={exact}", flush=True)
    wl = _small_workload()
    opts = AG.SolveOptions(max_iter=60000, tol=1e-13, adjoint_max_iter=60000, adjoint_tol=1e-13, check_every=50)
    case, a0 = AG.cst_case(wl, radius=1.0, options=opts, exact=exact)
    alpha = a0.copy()
    alpha[2 + 2] += 0.01                                   # a design away from the fit
    t = torch.tensor(alpha, requires_grad=True)
    J = AG.drag(t, case)
    J.backward()
    g = t.grad.numpy()
    # oracle on the same design
    g0 = wl.grid
    wall0, xi, up = OS.airfoil_stations(g0)
    D = OS.RBFDeform(g0.nodes, OS.wall_node_index(g0.topology, g0.ni, g0.nj, g0.n_wake), 1.0)
    eta = OS.cst_eta(6, alpha, xi, up)
    nodes = D.apply(np.stack([xi, eta], axis=1)).reshape(g0.nj + 1, g0.ni + 1, 2)
    import oracle
    vg, fl = wl.vgrid, wl.flow
    p = oracle.Problem(g0.topology, g0.ni, g0.nj, g0.n_wake, nodes, vg.kind, vg.n1, vg.n2, vg.vmax, vg.param,
                       fl.Kn, fl.Ma, fl.Tw, fl.objective, 8)
    p.primal_init()
    p.primal_solve(1e-13, 60000, 50)
    Jo = p.objective()
    p.adjoint_init()
    p.adjoint_solve(1e-13, 60000, 50)
    dwall = D.chain(p.mesh_sensitivity()) if exact else p.wall_sensitivity()["dJ_dnodes"]
    go = OS.cst_jacobian(6, alpha, xi, up).T @ dwall[:, 1]
    assert abs(J.item() - Jo) < 1e-10 * abs(Jo)
    assert np.max(np.abs(g - go)) < 1e-8 * np.max(np.abs(go))
