"""GPU parity of the second-order scheme (Sec. 3.1; readings in the oracle):
the HIP path through the C ABI against the FP64 oracle, both running the
same defect-correction iteration (correction every K sweeps) for a number of
sweeps that is not a multiple of K.

Bars as for the first-order scheme: FP64 f, phi element-wise <= 1e-11 of
max|.|, W <= 1e-11, J <= 1e-10 relative; mixed (FP32 f, phi, slopes and
corrections; FP64 moments and limiter arithmetic) f, J, phi <= 5e-5 (the
velocity grids reach f ~ 1e-22, where the limiter's squares would underflow
in FP32).  Cases: several velocity passes
with ragged tails, partial patches and tiles, the wake cut, one cell row
(every cell on the wall and the far field), odd n1, tau = infinity, the heat
objective on a hot wall, the largest velocity grid, limiter on and off.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2501_00923_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2501_00923_amd import dvm  # noqa: E402
from _parity import _rel, _say, check_resid, check_sens  # noqa: E402

NTHREADS = 16
K = 5


def _case(name):
    if name == "tiny_circle":
        return I.tiny_circle(Kn=1.0, Ma=0.5)
    if name == "tiny_naca":
        return I.tiny_naca(Kn=0.7, Ma=1.2)
    if name == "o24x12_v20":
        return I.circle_case(24, 12, 20, 5.0, 0.3, 0.9, r_outer=6.0, stretch=1.15)
    if name == "c_odd":
        g = I.naca_cgrid(5, 9, 7, t=0.12, m=0.03, r_outer=4.0, h1=0.03)
        return I.Workload("c_odd", g, I.VGridSpec(I.VG_MIDPOINT, 20, 20, 6.0), I.FlowSpec(0.3, 1.1), 0)
    if name == "c_sinh36":
        g = I.naca_cgrid(4, 8, 6, t=0.10, m=0.0, r_outer=4.0, h1=0.02)
        return I.Workload("c_sinh36", g, I.VGridSpec(I.VG_SINH, 36, 36, 6.0, 2.0), I.FlowSpec(0.05, 2.0), 0)
    if name == "o70x20_tiles":
        return I.circle_case(70, 20, 12, 5.0, 0.5, 0.9, r_outer=6.0, stretch=1.12)
    if name == "o12x6_v17":
        return I.circle_case(12, 6, 17, 5.0, 0.7, 0.8, r_outer=4.0, stretch=1.2)
    if name == "one_row":
        return I.circle_case(12, 1, 10, 5.0, 1.0, 0.5, r_outer=2.0, stretch=1.0)
    if name == "freemol":
        return I.tiny_circle(Kn=math.inf, Ma=0.7)
    if name == "heat_hotwall":
        w = I.tiny_naca(Kn=0.4, Ma=0.6)
        w.flow = I.FlowSpec(0.4, 0.6, Tw=1.6, objective=1)
        return w
    if name == "v128_max":
        return I.circle_case(6, 3, 128, 6.0, 0.8, 0.9, r_outer=3.0, stretch=1.3)
    raise KeyError(name)


def _run(wl, precision, n_primal, n_adjoint, limiter=True, k=K):
    _say(f"[gpu-so] {wl.name} precision={precision} limiter={limiter} K={k} primal={n_primal} adjoint={n_adjoint}")
    s = dvm.Solver.from_workload(wl, precision=precision, order=2,
                                 limiter=dvm.LIMITER_VENKAT if limiter else dvm.LIMITER_NONE, correction_every=k)
    s.primal_init()
    _, rps = s.primal_iterate(n_primal)
    o = oracle.Problem.from_workload(wl, nthreads=NTHREADS)
    o.set_scheme(2, limiter, k)
    o.primal_init()
    rpo = o.primal_iterate(n_primal)
    J, _ = s.objective()
    Jo = o.objective()
    res = dict(s=s, o=o, J=J, Jo=Jo, f=s.state_array(dvm.STATE_F), W=s.moments(), rp=(rps, rpo))
    if n_adjoint:
        s.adjoint_init()
        _, ras = s.adjoint_iterate(n_adjoint)
        o.adjoint_init()
        rao = o.adjoint_iterate(n_adjoint)
        res["ra"] = (ras, rao)
        res["phi"] = s.state_array(dvm.STATE_PHI)
        res["gs"], res["go"] = s.wall_sensitivity(), o.wall_sensitivity()
        res["msens"] = _rel(s.mesh_sensitivity(), o.mesh_sensitivity())
    return res


CASES = [("tiny_circle", True), ("tiny_circle", False), ("tiny_naca", True), ("o24x12_v20", True),
         ("c_odd", True), ("c_sinh36", True), ("o70x20_tiles", True), ("o12x6_v17", True), ("one_row", True),
         ("freemol", True), ("heat_hotwall", True), ("heat_hotwall", False), ("v128_max", True)]


@pytest.mark.parametrize("name,limiter", CASES, ids=[f"{n}-{'vk' if l else 'none'}" for n, l in CASES])
def test_fp64_second_order_parity(name, limiter):
    wl = _case(name)
    r = _run(wl, dvm.FP64, 23, 17, limiter)
    o = r["o"]
    ef, eW, ep = _rel(r["f"], o.f), _rel(r["W"], o.W), _rel(r["phi"], o.phi)
    eJ = abs(r["J"] - r["Jo"]) / max(abs(r["Jo"]), 1e-300)
    _say(f"[fp64-so] {name}: f {ef:.1e} W {eW:.1e} J {eJ:.1e} phi {ep:.1e} mesh sens {r['msens']:.1e}")
    check_resid(*r["rp"], label=f"{name} order-2 primal")
    check_resid(*r["ra"], label=f"{name} order-2 adjoint")
    check_sens(r["gs"], r["go"], 1e-10, f"{name} order 2")
    assert ef <= 1e-11 and eW <= 1e-11 and ep <= 1e-11 and r["msens"] <= 1e-10
    assert abs(r["J"] - r["Jo"]) <= 1e-10 * abs(r["Jo"]) + 1e-14


@pytest.mark.parametrize("name", ["tiny_circle", "o24x12_v20", "c_sinh36", "o12x6_v17"])
def test_mixed_second_order_parity(name):
    wl = _case(name)
    r = _run(wl, dvm.MIXED, 23, 17)
    o = r["o"]
    ef, ep = _rel(r["f"], o.f), _rel(r["phi"], o.phi)
    eJ = abs(r["J"] - r["Jo"]) / abs(r["Jo"])
    _say(f"[mixed-so] {name}: f {ef:.2e} J {eJ:.2e} phi {ep:.2e} mesh sens {r['msens']:.2e}")
    check_sens(r["gs"], r["go"], 1e-3, f"{name} order 2 mixed")
    assert ef <= 5e-5 and eJ <= 5e-5 and ep <= 5e-5 and r["msens"] <= 1e-3


def test_second_order_checkpoint_continues_bitwise():
    """A state saved after a multiple of K sweeps and loaded into a fresh
    solver continues bit for bit (the correction is re-evaluated at the
    first sweep after the load, as the uninterrupted run does there)."""
    wl = _case("o24x12_v20")
    a = dvm.Solver.from_workload(wl, order=2, correction_every=K)
    a.primal_init()
    a.primal_iterate(2 * K)
    snap = a.state_save(dvm.STATE_F)
    a.primal_iterate(7)
    b = dvm.Solver.from_workload(wl, order=2, correction_every=K)
    b.state_load(dvm.STATE_F, snap)
    b.primal_iterate(7)
    assert np.array_equal(a.state_array(dvm.STATE_F), b.state_array(dvm.STATE_F))


def test_second_order_argument_and_state_errors():
    wl = _case("tiny_circle")
    s = dvm.Solver.from_workload(wl, order=2)
    with pytest.raises(dvm.DvmError) as e:
        dvm._check(dvm.lib().dvm_solver_set_scheme(s._h, 1, 0, 5))
    assert e.value.code == dvm.DVM_ESTATE          # set before bind only
    s.primal_init()
    s.primal_iterate(6)
    s.adjoint_init()
    s.adjoint_iterate(3)
    # the wall and mesh sensitivities reuse the slope buffer; the adjoint
    # continues as if they had not run (the held term is kept, the slopes
    # are recomputed)
    s.mesh_sensitivity()
    t = dvm.Solver.from_workload(wl, order=2)
    t.primal_init()
    t.primal_iterate(6)
    t.adjoint_init()
    t.adjoint_iterate(3)
    s.wall_sensitivity()
    s.adjoint_iterate(9)
    t.adjoint_iterate(9)
    assert np.array_equal(s.state_array(dvm.STATE_PHI), t.state_array(dvm.STATE_PHI))


def test_c1_circle_second_order_converged():
    """Circle O-grid 64x32, 16x16 velocities, Kn 1, Ma 0.5, FP64, order 2 with
    the limiter (correction every 10 sweeps): the GPU converges the primal
    and the adjoint to 1e-8; the oracle runs the same numbers of sweeps;
    drag and the 8 Fourier-mode wall sensitivities agree to 1e-10."""
    wl = I.c1_circle()
    s = dvm.Solver.from_workload(wl, order=2, correction_every=10)
    s.primal_init()
    itp, rp = s.primal_iterate(20000, tol=1e-8, check_every=100)
    J, Cd = s.objective()
    s.adjoint_init()
    ita, ra = s.adjoint_iterate(20000, tol=1e-8, check_every=100)
    g = s.param_sensitivity(wl.grid.wall_jac)
    _say(f"[c1-so] primal {itp} sweeps (resid {rp:.2e}), adjoint {ita} sweeps (resid {ra:.2e}), C_d {Cd:.10f}")
    assert rp < 1e-8 and ra < 1e-8
    o = oracle.Problem.from_workload(wl, nthreads=NTHREADS)
    o.set_scheme(2, True, 10)
    o.primal_init()
    rpo = o.primal_iterate(itp)
    Jo = o.objective()
    o.adjoint_init()
    rao = o.adjoint_iterate(ita)
    go = np.einsum("md,mdp->p", o.wall_sensitivity()["dJ_dnodes"], wl.grid.wall_jac)
    check_resid(rp, rpo, "c1 order-2 primal")
    check_resid(ra, rao, "c1 order-2 adjoint")
    assert abs(J - Jo) <= 1e-10 * abs(Jo)
    assert abs(Cd - Jo / o.cd_scale()) <= 1e-10 * abs(Cd)
    assert _rel(g, go) <= 1e-10
