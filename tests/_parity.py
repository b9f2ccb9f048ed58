"""Comparison helpers of the GPU parity tests (HIP path against the oracle)."""
import sys

import numpy as np


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    """max|a - b| / max|b| (max-norm relative error of an array)."""
    scale = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / (scale if scale > 0 else 1.0)


SENS_KEYS = ("S_A", "S_x", "S_n", "dJ_dnodes")
# An output array whose largest entry is below this fraction of the largest
# sensitivity of the case is rounding noise of a quantity that vanishes in
# exact arithmetic (e.g. S_x of a converged free-molecular flow, where the
# wall-cell gradient terms cancel); it is held to the noise floor instead of
# to a relative bar.
SENS_NOISE = 1e-12


def check_sens(gs, go, tol, label=""):
    """Each sensitivity array against the oracle's: max|a - b| <= tol *
    max|b| (relative, per array), or, where max|b| is below SENS_NOISE times
    the case's largest sensitivity, max|a - b| <= SENS_NOISE times it."""
    scale = max(np.max(np.abs(go[k])) for k in SENS_KEYS)
    worst = 0.0
    for key in SENS_KEYS:
        ref = np.max(np.abs(go[key]))
        diff = np.max(np.abs(gs[key] - go[key]))
        if ref > SENS_NOISE * scale:
            err = diff / ref
            _say(f"[sens] {label} {key}: max|ref| {ref:.3e}  rel err {err:.2e}")
            assert err <= tol, (label, key, err, ref)
            worst = max(worst, err)
        else:
            _say(f"[sens] {label} {key}: max|ref| {ref:.3e} (noise floor)  abs err {diff:.2e}")
            assert diff <= SENS_NOISE * scale, (label, key, diff, ref, scale)
    return worst


def check_resid(r_gpu, r_or, label=""):
    """The stopping residual of the last sweep (relative change of W, or the
    weighted relative change of phi) against the oracle's after the same
    sweeps: <= 1e-10 relative, plus an absolute 1e-12 for the cancellation
    in W^{n+1} - W^n (both sides' W agree to ~1e-14 of |W|, which bounds the
    difference of the two residuals to that order)."""
    err = abs(r_gpu - r_or)
    _say(f"[resid] {label} gpu {r_gpu:.15e} oracle {r_or:.15e} diff {err:.2e}")
    assert err <= 1e-10 * abs(r_or) + 1e-12, (label, r_gpu, r_or)
