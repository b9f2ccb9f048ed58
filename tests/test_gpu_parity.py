"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Both sides run the same number of Jacobi sweeps from the same start, so
their iterates agree to rounding.  Bars:
  FP64   f, phi element-wise <= 1e-11 of max|.|;  W <= 1e-11;  J, C_d and every
         sensitivity output <= 1e-10 relative (max-norm of the array)
  MIXED  (FP32 f / phi, FP64 moments and integrals) J <= 2e-5, f <= 2e-5 of
         max|f|, sensitivities <= 1e-3 (FP32 rounding of ~1e-7 per sweep,
         growing with the sweep count; measured errors are reported by the
         precision tests and the benchmark)
Cases span several 64-velocity wave steps with a ragged tail, fewer
velocities than a wave, odd grid sizes (partial 2x2 patches and tiles), the
largest velocity grid (128 x 128), both topologies (wake cut), tau =
infinity, the heat objective and a hot wall.
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


def _case(name):
    if name == "tiny_circle":
        return I.tiny_circle(Kn=1.0, Ma=0.5)
    if name == "tiny_naca":
        return I.tiny_naca(Kn=0.7, Ma=1.2)
    if name == "o24x12_v20":                       # nv = 400: one full pass + ragged tail
        return I.circle_case(24, 12, 20, 5.0, 0.3, 0.9, r_outer=6.0, stretch=1.15)
    if name == "c_nc24":                           # nv = 576: two passes + a 64-velocity tail
        g = I.naca_cgrid(6, 10, 8, t=0.12, m=0.02, r_outer=5.0, h1=0.02)
        return I.Workload("c_nc24", g, I.VGridSpec(I.VG_NEWTON_COTES, 24, 24, 5.0), I.FlowSpec(0.2, 0.8), 0)
    if name == "c_sinh36":                         # nv = 1296: five passes + tail
        g = I.naca_cgrid(4, 8, 6, t=0.10, m=0.0, r_outer=4.0, h1=0.02)
        return I.Workload("c_sinh36", g, I.VGridSpec(I.VG_SINH, 36, 36, 6.0, 2.0), I.FlowSpec(0.05, 2.0), 0)
    if name == "freemol":
        return I.tiny_circle(Kn=math.inf, Ma=0.7)
    if name == "heat_hotwall":
        w = I.tiny_naca(Kn=0.4, Ma=0.6)
        w.flow = I.FlowSpec(0.4, 0.6, Tw=1.6, objective=1)
        return w
    if name == "one_row":                          # nj = 1, nv = 100; patches of 2 cells
        return I.circle_case(12, 1, 10, 5.0, 1.0, 0.5, r_outer=2.0, stretch=1.0)
    if name == "o13x7_odd":                        # odd ni, nj: patches of 1, 2 and 4 cells; nv = 324
        return I.circle_case(13, 7, 18, 5.0, 0.5, 0.6, r_outer=4.0, stretch=1.2)
    if name == "c_odd":                            # C-grid 28 x 7: odd nj, wake cut; nv = 400
        g = I.naca_cgrid(5, 9, 7, t=0.12, m=0.03, r_outer=4.0, h1=0.03)
        return I.Workload("c_odd", g, I.VGridSpec(I.VG_MIDPOINT, 20, 20, 6.0), I.FlowSpec(0.3, 1.1), 0)
    if name == "o12x6_v17":                        # odd n1: one velocity per lane in FP32 as well
        return I.circle_case(12, 6, 17, 5.0, 0.7, 0.8, r_outer=4.0, stretch=1.2)
    if name == "o70x20_tiles":                     # 3 x 2 sweep tiles of 32 x 16 with ragged last ones
        return I.circle_case(70, 20, 12, 5.0, 0.5, 0.9, r_outer=6.0, stretch=1.12)
    if name == "v128_max":                         # the largest velocity grid, 128 x 128 = 16384
        return I.circle_case(6, 3, 128, 6.0, 0.8, 0.9, r_outer=3.0, stretch=1.3)
    raise KeyError(name)


CASES = ["tiny_circle", "tiny_naca", "o24x12_v20", "c_nc24", "c_sinh36", "freemol", "heat_hotwall", "one_row",
         "o13x7_odd", "c_odd", "o12x6_v17", "o70x20_tiles", "v128_max"]


def _run(wl, precision, n_primal, n_adjoint, n_params_jac=None):
    _say(f"[gpu] {wl.name} precision={precision} primal={n_primal} adjoint={n_adjoint}")
    s = dvm.Solver.from_workload(wl, precision=precision)
    s.primal_init()
    _, rps = s.primal_iterate(n_primal)
    o = oracle.Problem.from_workload(wl, nthreads=NTHREADS)
    o.primal_init()
    rpo = o.primal_iterate(n_primal)
    res = dict(s=s, o=o, rp=(rps, rpo))
    if n_adjoint is not None:
        s.adjoint_init()
        _, ras = s.adjoint_iterate(n_adjoint)
        o.adjoint_init()
        rao = o.adjoint_iterate(n_adjoint)
        res["ra"] = (ras, rao)
    return res


@pytest.mark.parametrize("name", CASES)
def test_fp64_primal_adjoint_sensitivity_parity(name):
    wl = _case(name)
    r = _run(wl, dvm.FP64, 37, 29)
    s, o = r["s"], r["o"]
    check_resid(*r["rp"], label=f"{name} primal")
    check_resid(*r["ra"], label=f"{name} adjoint")
    assert _rel(s.state_array(dvm.STATE_F), o.f) <= 1e-11
    assert _rel(s.moments(), o.W) <= 1e-11
    J, Cd = s.objective()
    Jo = o.objective()
    assert abs(J - Jo) <= 1e-10 * abs(Jo) + 1e-14
    if not math.isnan(Cd) and wl.flow.Ma > 0:
        assert abs(Cd - Jo / o.cd_scale()) <= 1e-10 * abs(Jo / o.cd_scale()) + 1e-14
    assert _rel(s.state_array(dvm.STATE_PHI), o.phi) <= 1e-11
    gs, go = s.wall_sensitivity(), o.wall_sensitivity()
    check_sens(gs, go, 1e-10, name)
    jac = wl.grid.wall_jac
    if jac.shape[-1]:
        da = s.param_sensitivity(jac)
        do = np.einsum("md,mdp->p", go["dJ_dnodes"], jac)
        assert _rel(da, do) <= 1e-10
    # exact discrete derivative in every node coordinate
    ms, mo = s.mesh_sensitivity(), o.mesh_sensitivity()
    assert _rel(ms, mo) <= 1e-10


@pytest.mark.parametrize("name", ["tiny_circle", "o24x12_v20", "c_sinh36", "o13x7_odd", "o12x6_v17"])
def test_mixed_precision_parity(name):
    wl = _case(name)
    r = _run(wl, dvm.MIXED, 37, 29)
    s, o = r["s"], r["o"]
    ef = _rel(s.state_array(dvm.STATE_F), o.f)
    J, _ = s.objective()
    Jo = o.objective()
    eJ = abs(J - Jo) / abs(Jo)
    gs, go = s.wall_sensitivity(), o.wall_sensitivity()
    eS = check_sens(gs, go, 1e-3, f"{name} mixed")
    eM = _rel(s.mesh_sensitivity(), o.mesh_sensitivity())
    _say(f"[mixed] {name}: f {ef:.2e}  J {eJ:.2e}  sens {eS:.2e}  mesh sens {eM:.2e}")
    assert ef <= 2e-5 and eJ <= 2e-5 and eS <= 1e-3 and eM <= 1e-3


def test_param_sensitivity_at_the_parameter_limit():
    """64 shape parameters, the most the library takes, against the
    oracle's wall-node derivative contracted with the same Jacobian (a dense
    random one); 65 parameters are refused before any device work."""
    wl = I.tiny_naca()
    r = _run(wl, dvm.FP64, 37, 29)
    s, o = r["s"], r["o"]
    nw = wl.grid.wall_jac.shape[0]
    jac = np.random.default_rng(64).standard_normal((nw, 2, dvm.MAX_PARAMS))
    da = s.param_sensitivity(jac)
    do = np.einsum("md,mdp->p", o.wall_sensitivity()["dJ_dnodes"], jac)
    assert _rel(da, do) <= 1e-10
    # fewer parameters give the leading entries of the same contraction
    assert _rel(s.param_sensitivity(jac[..., :5]), do[:5]) <= 1e-10
    with pytest.raises(dvm.DvmError) as ei:
        s.param_sensitivity(np.zeros((nw, 2, dvm.MAX_PARAMS + 1)))
    assert ei.value.code == dvm.DVM_EINVAL


def test_c1_circle_full_size():
    """Circle O-grid 64x32, 16x16 velocities on [-5,5], Kn 1, Ma 0.5, FP64:
    the GPU converges the primal and the adjoint to a relative residual of
    1e-8; the oracle then runs the same numbers of sweeps, and drag, C_d and
    the 8 Fourier-mode sensitivities agree to 1e-10."""
    wl = I.c1_circle()
    s = dvm.Solver.from_workload(wl, precision=dvm.FP64)
    s.primal_init()
    itp, rp = s.primal_iterate(20000, tol=1e-8, check_every=100)
    J, Cd = s.objective()
    s.adjoint_init()
    ita, ra = s.adjoint_iterate(20000, tol=1e-8, check_every=100)
    g = s.param_sensitivity(wl.grid.wall_jac)
    _say(f"[c1] primal {itp} sweeps (resid {rp:.2e}), adjoint {ita} sweeps (resid {ra:.2e}), C_d {Cd:.10f}")
    assert rp < 1e-8 and ra < 1e-8
    o = oracle.Problem.from_workload(wl, nthreads=NTHREADS)
    o.primal_init()
    rpo = o.primal_iterate(itp)
    Jo = o.objective()
    o.adjoint_init()
    rao = o.adjoint_iterate(ita)
    go = np.einsum("md,mdp->p", o.wall_sensitivity()["dJ_dnodes"], wl.grid.wall_jac)
    # the stopping test: the oracle's residual after the same sweeps is the
    # GPU's (so both stop at the same sweep)
    check_resid(rp, rpo, "c1 primal")
    check_resid(ra, rao, "c1 adjoint")
    assert rpo < 1e-8 and rao < 1e-8
    assert abs(J - Jo) <= 1e-10 * abs(Jo)
    assert abs(Cd - Jo / o.cd_scale()) <= 1e-10 * abs(Cd)
    assert _rel(g, go) <= 1e-10


EQ_CASES = ["tiny_circle", "tiny_naca", "c_nc24", "c_sinh36", "heat_hotwall", "o12x6_v17", "o70x20_tiles"]


def _run_eq(wl, precision, n_primal, n_adjoint, order=1):
    """Both sides with the discrete-conservative equilibrium."""
    _say(f"[gpu-eq] {wl.name} precision={precision} order={order} primal={n_primal} adjoint={n_adjoint}")
    s = dvm.Solver.from_workload(wl, precision=precision, equilibrium=dvm.EQ_CONSERVATIVE, order=order,
                                 correction_every=5)
    o = oracle.Problem.from_workload(wl, nthreads=NTHREADS)
    o.set_equilibrium(1)
    if order == 2:
        o.set_scheme(2, True, 5)
    s.primal_init()
    o.primal_init()
    _, rps = s.primal_iterate(n_primal)
    rpo = o.primal_iterate(n_primal)
    s.adjoint_init()
    o.adjoint_init()
    _, ras = s.adjoint_iterate(n_adjoint)
    rao = o.adjoint_iterate(n_adjoint)
    return s, o, (rps, rpo), (ras, rao)


@pytest.mark.parametrize("name", EQ_CASES)
def test_fp64_conservative_equilibrium_parity(name):
    wl = _case(name)
    s, o, rp, ra = _run_eq(wl, dvm.FP64, 37, 29)
    check_resid(*rp, label=f"{name} conservative primal")
    check_resid(*ra, label=f"{name} conservative adjoint")
    ef, eW, ep = _rel(s.state_array(dvm.STATE_F), o.f), _rel(s.moments(), o.W), _rel(s.state_array(dvm.STATE_PHI), o.phi)
    J, _ = s.objective()
    Jo = o.objective()
    _say(f"[gpu-eq] {name}: f {ef:.2e} W {eW:.2e} phi {ep:.2e} J {abs(J - Jo) / abs(Jo):.2e}")
    assert ef <= 1e-11 and eW <= 1e-11 and ep <= 1e-11
    assert abs(J - Jo) <= 1e-10 * abs(Jo)
    check_sens(s.wall_sensitivity(), o.wall_sensitivity(), 1e-10, f"{name} conservative")
    assert _rel(s.mesh_sensitivity(), o.mesh_sensitivity()) <= 1e-10


@pytest.mark.parametrize("name", ["tiny_circle", "c_sinh36", "o12x6_v17"])
def test_mixed_conservative_equilibrium_parity(name):
    wl = _case(name)
    s, o, _, _ = _run_eq(wl, dvm.MIXED, 37, 29)
    ef = _rel(s.state_array(dvm.STATE_F), o.f)
    J, _ = s.objective()
    Jo = o.objective()
    eS = check_sens(s.wall_sensitivity(), o.wall_sensitivity(), 1e-3, f"{name} conservative mixed")
    _say(f"[gpu-eq mixed] {name}: f {ef:.2e} J {abs(J - Jo) / abs(Jo):.2e} sens {eS:.2e}")
    assert ef <= 2e-5 and abs(J - Jo) <= 2e-5 * abs(Jo)


def test_second_order_conservative_equilibrium_parity():
    wl = _case("tiny_naca")
    s, o, rp, ra = _run_eq(wl, dvm.FP64, 23, 17, order=2)
    check_resid(*rp, label="order-2 conservative primal")
    check_resid(*ra, label="order-2 conservative adjoint")
    assert _rel(s.state_array(dvm.STATE_F), o.f) <= 1e-11
    assert _rel(s.state_array(dvm.STATE_PHI), o.phi) <= 1e-11
    check_sens(s.wall_sensitivity(), o.wall_sensitivity(), 1e-10, "order 2 conservative")


def test_near_continuum_case_converges_with_the_conservative_equilibrium():
    """128x64 NACA0012 C-grid, 32x32 Newton-Cotes velocities on [-6, 6],
    Kn 0.01, Ma 0.5: the pointwise equilibrium's Jacobi iteration turns
    non-finite within 400 sweeps (DVM_ENAN); the conservative one decreases
    its residual every 50 sweeps and matches the oracle after 100."""
    g = I.naca_cgrid(16, 48, 64, t=0.12, m=0.0)
    wl = I.Workload("naca0012_c128x64_v32nc_kn0.01", g, I.VGridSpec(I.VG_NEWTON_COTES, 32, 32, 6.0),
                    I.FlowSpec(0.01, 0.5), 0)
    _say("[gpu-eq] near-continuum case: pointwise")
    p = dvm.Solver.from_workload(wl)
    p.primal_init()
    with pytest.raises(dvm.DvmError) as ei:
        p.primal_iterate(400, tol=1e-300, check_every=50)
    assert ei.value.code == dvm.DVM_ENAN
    _say("[gpu-eq] near-continuum case: conservative")
    s = dvm.Solver.from_workload(wl, equilibrium=dvm.EQ_CONSERVATIVE)
    s.primal_init()
    rs = [s.primal_iterate(50)[1] for _ in range(8)]
    _say(f"[gpu-eq] residuals every 50 sweeps: {' '.join(f'{r:.2e}' for r in rs)}")
    assert all(b < a for a, b in zip(rs, rs[1:]))
    o = oracle.Problem.from_workload(wl, nthreads=NTHREADS)
    o.set_equilibrium(1)
    o.primal_init()
    o.primal_iterate(100)
    t = dvm.Solver.from_workload(wl, equilibrium=dvm.EQ_CONSERVATIVE)
    t.primal_init()
    t.primal_iterate(100)
    assert _rel(t.state_array(dvm.STATE_F), o.f) <= 1e-11
