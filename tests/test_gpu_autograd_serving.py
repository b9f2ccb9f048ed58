"""GPU: the differentiable drag (torch.autograd.Function over the HIP adjoint)
against the oracle's adjoint gradient and finite differences; the solve
server's results alone vs in a mix of concurrently resident solves."""
import sys

import numpy as np
import pytest

import oracle
from paper_2501_00923_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2501_00923_amd import autograd as AG  # noqa: E402
from paper_2501_00923_amd import dvm  # noqa: E402
from paper_2501_00923_amd import serving as S  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle_grad(grid, vg, flow, n_primal, n_adjoint, order=1, correction_every=10):
    o = oracle.Problem(grid.topology, grid.ni, grid.nj, grid.n_wake, grid.nodes, vg.kind, vg.n1, vg.n2,
                       vg.vmax, vg.param, flow.Kn, flow.Ma, flow.Tw, flow.objective, nthreads=16)
    if order == 2:
        o.set_scheme(2, True, correction_every)
    o.primal_init()
    o.primal_iterate(n_primal)
    J = o.objective()
    o.adjoint_init()
    o.adjoint_iterate(n_adjoint)
    g = np.einsum("md,mdp->p", o.wall_sensitivity()["dJ_dnodes"], grid.wall_jac)
    return J, g


def test_autograd_matches_oracle_adjoint_and_offload_is_identical():
    case, a0 = AG.circle_fourier_case(16, 8, 8, 5.0, Kn=1.0, Ma=0.5, r_outer=5.0, stretch=1.2,
                                      options=AG.SolveOptions(max_iter=300, adjoint_max_iter=300, fixed_iters=True))
    alpha = torch.tensor(a0 + np.array([0.02, -0.01, 0.015, 0.0, 0.0, 0.01, 0.0, 0.0]), requires_grad=True)
    _say("[gpu] autograd circle 16x8")
    J = AG.drag(alpha, case)
    J.backward()
    Jo, go = _oracle_grad(case.make_grid(alpha.detach().numpy()), case.vgrid, case.flow, 300, 300)
    assert abs(J.item() - Jo) <= 1e-10 * abs(Jo)
    assert np.max(np.abs(alpha.grad.numpy() - go)) <= 1e-10 * np.max(np.abs(go))
    case.offload = True
    case.checkpoint_every = 100
    rec = AG.ForwardRecord()
    alpha2 = alpha.detach().clone().requires_grad_(True)
    J2 = AG.drag(alpha2, case, rec)
    (3.0 * J2).backward()
    assert J2.item() == J.item()
    assert np.array_equal(alpha2.grad.numpy(), 3.0 * alpha.grad.numpy())
    assert len(rec.checkpoints) == 3 and rec.iters == 300


def test_autograd_second_order_matches_oracle_and_offload_is_identical():
    """The autograd wrapper with the second-order scheme (correction every 5
    sweeps): J and dJ/dalpha equal the oracle's after the same sweeps; the
    offloaded backward (f reloaded, correction re-evaluated) is bitwise the
    same when the checkpoint falls on a multiple of K."""
    opts = AG.SolveOptions(max_iter=300, adjoint_max_iter=300, fixed_iters=True)
    case, a0 = AG.circle_fourier_case(16, 8, 8, 5.0, Kn=1.0, Ma=0.5, r_outer=5.0, stretch=1.2, options=opts)
    case.order, case.correction_every = 2, 5
    alpha = torch.tensor(a0 + np.array([0.02, -0.01, 0.015, 0.0, 0.0, 0.01, 0.0, 0.0]), requires_grad=True)
    _say("[gpu] autograd circle 16x8, order 2")
    J = AG.drag(alpha, case)
    J.backward()
    Jo, go = _oracle_grad(case.make_grid(alpha.detach().numpy()), case.vgrid, case.flow, 300, 300,
                          order=2, correction_every=5)
    assert abs(J.item() - Jo) <= 1e-10 * abs(Jo)
    assert np.max(np.abs(alpha.grad.numpy() - go)) <= 1e-10 * np.max(np.abs(go))
    case.offload = True
    case.checkpoint_every = 100
    alpha2 = alpha.detach().clone().requires_grad_(True)
    J2 = AG.drag(alpha2, case)
    J2.backward()
    assert J2.item() == J.item()
    assert np.array_equal(alpha2.grad.numpy(), alpha.grad.numpy())


def test_autograd_fd_agreement_paper_mode():
    """Central differences (h = 1e-6) of fully converged J against the
    adjoint gradient: sine modes vanish on both sides; the a0 and a2 modes
    agree to the discretisation level of the wall-only shape derivative, and
    to the differences' own error with the exact discrete derivative."""
    case, a0 = AG.circle_fourier_case(32, 16, 8, 5.0, Kn=1.0, Ma=0.5, r_outer=5.0, stretch=1.2 ** 0.5,
                                      options=AG.SolveOptions(max_iter=30000, tol=1e-13, adjoint_tol=1e-13,
                                                              check_every=100))
    alpha = torch.tensor(a0, requires_grad=True)
    J = AG.drag(alpha, case)
    J.backward()
    g = alpha.grad.numpy()
    h = 1e-6
    fd = {}
    for p in (0, 2, 5):
        e = np.zeros(8)
        e[p] = h
        Jp = AG.drag(torch.tensor(a0 + e), case).item()
        Jm = AG.drag(torch.tensor(a0 - e), case).item()
        fd[p] = (Jp - Jm) / (2 * h)
    _say(f"[gpu] fd {fd}  adjoint {g[[0, 2, 5]]}")
    assert abs(fd[5]) < 1e-6 and abs(g[5]) < 1e-10
    assert abs(g[0] - fd[0]) < 0.1 * abs(fd[0])
    assert abs(g[2] - fd[2]) < 0.05 * abs(fd[2])
    # the exact discrete derivative (every mesh node moves with alpha) equals
    # the differences to their own error
    case.exact = True
    alpha = torch.tensor(a0, requires_grad=True)
    AG.drag(alpha, case).backward()
    ge = alpha.grad.numpy()
    _say(f"[gpu] exact {ge[[0, 2, 5]]}")
    for p in (0, 2, 5):
        assert abs(ge[p] - fd[p]) <= 1e-4 * max(abs(fd[0]), abs(fd[2]))


def test_differentiation_workload_matches_oracle():
    """Seeded NACA (thickness/camber drawn), 192x96 C-grid, 48x48
    Newton-Cotes grid, Kn 0.5, Ma 2, 24 B-spline offsets: gradient after 12
    primal + 12 adjoint sweeps equals the oracle's."""
    case, a0 = AG.naca_bspline_case(seed=0, options=AG.SolveOptions(max_iter=12, adjoint_max_iter=12,
                                                                    fixed_iters=True))
    alpha = torch.tensor(a0, requires_grad=True)
    _say("[gpu] autograd naca 192x96 v48")
    J = AG.drag(alpha, case)
    J.backward()
    Jo, go = _oracle_grad(case.make_grid(a0), case.vgrid, case.flow, 12, 12)
    assert abs(J.item() - Jo) <= 1e-10 * abs(Jo)
    assert np.max(np.abs(alpha.grad.numpy() - go)) <= 1e-10 * np.max(np.abs(go))


def _small_stream(n, seed, rate):
    # velocity grids of 16 and 24 points on [-6, 6]: coarser grids do not
    # resolve the thermal width and the pointwise Maxwellian then diverges
    return I.poisson_stream(n, rate, seed=seed, mesh_choices=[(32, 16), (64, 32)], vgrid_choices=[16, 24])


@pytest.mark.parametrize("precision", [dvm.MIXED, dvm.FP64])
def test_server_results_alone_equal_mix(precision):
    reqs = _small_stream(10, 11, 1e6)
    for r in reqs:       # keep the solves short: moderate Kn
        r.workload.flow.Kn = max(r.workload.flow.Kn, 0.3)
    for r in reqs[::3]:  # some requests ask for the second-order scheme
        r.order = 2
    cfg = S.ServeConfig(memory_budget=1 << 34, sweeps_per_check=10, tol=1e-4, adjoint_tol=1e-4, max_iter=400)
    _say(f"[gpu] server mix precision={precision}")
    mix = S.serve(reqs, S.GpuBackend(precision), cfg, realtime=False)
    assert mix["peak_resident"] > 1
    one = S.serve_one_at_a_time(reqs, S.GpuBackend(precision), cfg, realtime=False)
    assert one["peak_resident"] == 1
    for a, b in zip(mix["results"], one["results"]):
        assert a.status == b.status and a.status in ("ok", "notconv")
        assert a.J == b.J and a.primal_iters == b.primal_iters and a.adjoint_iters == b.adjoint_iters
        if a.dJ is not None:
            assert np.array_equal(a.dJ, b.dJ)


@pytest.mark.parametrize("precision", [dvm.FP64, dvm.MIXED])
def test_server_with_prediction_alone_equals_mix(precision):
    """Requests below Kn 0.5 solve with the conservative equilibrium and the
    macroscopic prediction: their batched results (shared Gauss-Seidel
    launches, equilibrium parameters per member group) equal one-at-a-time
    results bit for bit, and both reach the tolerance."""
    reqs = _small_stream(8, 13, 1e6)
    for i, r in enumerate(reqs):        # half near the continuum, half not
        r.workload.flow.Kn = 0.02 if i % 2 == 0 else 0.6
    cfg = S.ServeConfig(memory_budget=1 << 34, sweeps_per_check=10, tol=1e-5, adjoint_tol=1e-5, max_iter=2000)
    _say(f"[gpu] server with prediction, precision={precision}")
    mix = S.serve(reqs, S.GpuBackend(precision, accelerate_below_kn=0.5, accelerate=(5, 20)), cfg, realtime=False)
    assert mix["peak_resident"] > 1
    one = S.serve_one_at_a_time(reqs, S.GpuBackend(precision, accelerate_below_kn=0.5, accelerate=(5, 20)), cfg,
                                realtime=False)
    for a, b in zip(mix["results"], one["results"]):
        assert a.status == b.status == "ok", (a.rid, a.status, a.error)
        assert a.J == b.J and a.primal_iters == b.primal_iters and a.adjoint_iters == b.adjoint_iters
        if a.dJ is not None:
            assert np.array_equal(a.dJ, b.dJ)


def test_server_admission_respects_budget():
    reqs = _small_stream(8, 5, 1e6)
    for r in reqs:
        r.workload.flow.Kn = max(r.workload.flow.Kn, 0.3)
    be = S.GpuBackend(dvm.MIXED)
    fps = [be.footprint(r) for r in reqs]
    budget = int(sum(sorted(fps)[-3:]))
    out = S.serve(reqs, be, S.ServeConfig(memory_budget=budget, sweeps_per_check=10, tol=1e-4, adjoint_tol=1e-4,
                                          max_iter=200), realtime=False)
    assert out["peak_bytes"] <= budget and out["completed"] == len(reqs)


def test_autograd_device_alpha_and_unconverged_solves():
    """A CUDA alpha gets its gradient on its own device and dtype (equal to
    the host one); a solve left above its tolerance warns, or raises when
    asked to."""
    case, a0 = AG.circle_fourier_case(16, 8, 8, 5.0, Kn=1.0, Ma=0.5, r_outer=5.0, stretch=1.2,
                                      options=AG.SolveOptions(max_iter=200, adjoint_max_iter=200, fixed_iters=True))
    a_host = torch.tensor(a0 + 0.01, requires_grad=True)
    AG.drag(a_host, case).backward()
    a_dev = torch.tensor(a0 + 0.01, device="cuda", requires_grad=True)
    AG.drag(a_dev, case).backward()
    assert a_dev.grad.device == a_dev.device and a_dev.grad.dtype == a_dev.dtype
    assert np.array_equal(a_dev.grad.cpu().numpy(), a_host.grad.numpy())
    case.options = AG.SolveOptions(max_iter=40, adjoint_max_iter=40, tol=1e-12, adjoint_tol=1e-12, check_every=20)
    a = torch.tensor(a0, requires_grad=True)
    with pytest.warns(AG.NotConvergedWarning):
        J = AG.drag(a, case)
    with pytest.warns(AG.NotConvergedWarning):
        J.backward()
    case.options.on_notconv = "raise"
    with pytest.raises(dvm.NotConverged):
        AG.drag(torch.tensor(a0, requires_grad=True), case)
