"""The allocation-free batch (dvm_batch_create_static) against the batch
with a caller-owned work buffer (dvm_batch_create), through the C ABI.

Two creates in a row on the device's fixed table array, the second with a
smaller batch (fewer, smaller members) after the first is destroyed (the
first with a member that runs the macroscopic prediction): every
member's f / phi, moments and residuals bitwise equal to the same members
run in a dvm_batch_create batch (the same kernels, the same block map).  A
second live static batch on the device and oversized batches are refused.
"""
import numpy as np
import pytest

from paper_2501_00923_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2501_00923_amd import dvm  # noqa: E402
from _parity import _say  # noqa: E402

BIG = [I.tiny_circle(Kn=1.0, Ma=0.5), I.tiny_naca(Kn=0.3, Ma=1.5),
       I.circle_case(24, 12, 20, 5.0, 0.3, 0.9, r_outer=6.0, stretch=1.15),
       I.circle_case(10, 5, 17, 5.0, 0.6, 0.7, r_outer=4.0, stretch=1.2),
       I.circle_case(70, 20, 12, 5.0, 0.5, 0.9, r_outer=6.0, stretch=1.12)]
SMALL = [I.tiny_circle(Kn=2.0, Ma=0.4), I.circle_case(12, 6, 17, 5.0, 0.7, 0.8, r_outer=4.0, stretch=1.2)]


def _members(cases, precision):
    """Fresh solvers: the first in its adjoint phase, the second of the
    second-order scheme, the fourth with the conservative equilibrium and
    the macroscopic prediction, the others primal."""
    out = []
    for i, wl in enumerate(cases):
        extra = dict(equilibrium=1, accelerate=(3, 5)) if i == 3 else {}
        s = dvm.Solver.from_workload(wl, precision=precision, order=2 if i == 1 else 1, correction_every=3, **extra)
        s.primal_init()
        s.primal_sweeps(4)
        if i == 0:
            s.adjoint_init()
            s.adjoint_sweeps(2)
        out.append(s)
    return out


def _state(s):
    which = dvm.STATE_PHI if s.phase == 1 else dvm.STATE_F
    return s.state_save(which), s.moments()


def _compare(cases, precision, sweeps):
    ref = _members(cases, precision)
    b = dvm.Batch(ref)
    b.run(sweeps)
    r_ref = b.residuals()
    b.close()
    got = _members(cases, precision)
    sb = dvm.Batch(got, static=True)
    try:
        sb.run(sweeps)
        r_got = sb.residuals()
    finally:
        sb.close()
    assert np.array_equal(r_ref, r_got)
    for s, t in zip(ref, got):
        (a, wa), (c, wc) = _state(s), _state(t)
        assert np.array_equal(a, c) and np.array_equal(wa, wc)
        assert s.iterations(s.phase) == t.iterations(t.phase)


@pytest.mark.parametrize("precision", [dvm.FP64, dvm.MIXED])
def test_static_batch_equals_batch_twice(precision):
    _say(f"[gpu] allocation-free batch precision={precision}: {len(BIG)} members, then {len(SMALL)}")
    _compare(BIG, precision, 11)
    _compare(SMALL, precision, 6)


def test_static_batch_limits():
    _say("[gpu] allocation-free batch limits")
    a = _members(SMALL, dvm.FP64)
    sb = dvm.Batch(a[:1], static=True)
    try:
        with pytest.raises(dvm.DvmError) as ei:
            dvm.Batch(a[1:], static=True)
        assert ei.value.code == dvm.DVM_ESTATE
    finally:
        sb.close()
    sb = dvm.Batch(a[1:], static=True)        # the slot is free again
    sb.close()
    many = [dvm.Solver.from_workload(I.tiny_circle()) for _ in range(65)]
    for s in many:
        s.primal_init()
    with pytest.raises(dvm.DvmError) as ei:
        dvm.Batch(many, static=True)
    assert ei.value.code == dvm.DVM_EINVAL
