"""Python binding of libdvm's outer-loop calls (include/dvm.h): the CST
parameterisation (Sec. 3.3), the volume constraint (Sec. 2.4, 3.2) and the
RBF bulk-mesh deformation (Sec. 3.4, Step 2).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import dvm as _dvm
from .dvm import Mesh, _check, alloc_device, current_stream_handle, lib

MAX_NB = 20


def n_params(nb: int) -> int:
    return 2 * nb + 6


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(np.asarray(a).astype(np.int32))


def cst_eval(nb: int, alpha, xi, upper, jacobian: bool = False):
    """eta at the stations (and d eta / d alpha, shape (n, 2 nb + 6))."""
    alpha, xi, up = _f64(alpha), _f64(xi), _i32(upper)
    n = len(xi)
    eta = np.zeros(n)
    jac = np.zeros((n, n_params(nb))) if jacobian else None
    _check(lib().dvm_cst_eval(int(nb), alpha.ctypes.data, n, xi.ctypes.data, up.ctypes.data, eta.ctypes.data,
                              None if jac is None else jac.ctypes.data))
    return (eta, jac) if jacobian else eta


def cst_fit(nb: int, xi, upper, eta, fixed=None, alpha=None):
    """Least-squares initial design (eq. cstini); returns (alpha, rms)."""
    xi, up, eta = _f64(xi), _i32(upper), _f64(eta)
    a = np.zeros(n_params(nb)) if alpha is None else _f64(alpha).copy()
    fx = None if fixed is None else _i32(fixed)
    rms = C.c_double()
    _check(lib().dvm_cst_fit(int(nb), len(xi), xi.ctypes.data, up.ctypes.data, eta.ctypes.data,
                             None if fx is None else fx.ctypes.data, a.ctypes.data, C.byref(rms)))
    return a, rms.value


def volume_constraint(wall_xy, v_min: float):
    """(Q, dQ/dx[nw][2]) of the closed wall loop."""
    w = _f64(wall_xy)
    Q = C.c_double()
    dQ = np.zeros_like(w)
    _check(lib().dvm_volume_constraint(len(w), w.ctypes.data, float(v_min), C.byref(Q), dQ.ctypes.data))
    return Q.value, dQ


class Deformer:
    """Wendland-C0 RBF deformation of a reference mesh, bound to a
    torch-allocated device workspace."""

    def __init__(self, mesh: Mesh, radius: float, buffer=None, stream=None):
        h = C.c_void_p()
        _check(lib().dvm_deform_create(mesh._h, float(radius), C.byref(h)))
        self._h = h
        self.ni, self.nj, self.nw = mesh.ni, mesh.nj, mesh.nw
        self.radius = float(radius)
        self.workspace_bytes = int(lib().dvm_deform_workspace_bytes(h))
        if buffer is None:
            buffer = alloc_device(self.workspace_bytes)
        self.buffer = buffer
        st = current_stream_handle() if stream is None else C.c_void_p(int(stream))
        _check(lib().dvm_deform_bind(h, C.c_void_p(buffer.data_ptr()), C.c_size_t(buffer.numel()), st))

    def apply(self, wall_xy) -> np.ndarray:
        """New wall node positions (nw, 2) -> every node, (nj+1, ni+1, 2)."""
        w = _f64(wall_xy)
        if w.shape != (self.nw, 2):
            raise ValueError(f"wall_xy must have shape ({self.nw}, 2)")
        out = np.zeros((self.nj + 1, self.ni + 1, 2))
        _check(lib().dvm_deform_apply(self._h, w.ctypes.data, out.ctypes.data))
        return out

    def chain(self, dJ_dx) -> np.ndarray:
        """dJ/d(all nodes) (nj+1, ni+1, 2) -> dJ/d(wall nodes) (nw, 2)."""
        g = _f64(dJ_dx)
        if g.size != 2 * (self.nj + 1) * (self.ni + 1):
            raise ValueError("dJ_dx must hold every node coordinate")
        out = np.zeros((self.nw, 2))
        _check(lib().dvm_deform_chain(self._h, g.ctypes.data, out.ctypes.data))
        return out

    def close(self):
        # the library is loaded by then (create needed it); at interpreter
        # shutdown the module globals may already be gone
        if getattr(self, "_h", None) and _dvm._lib is not None:
            _dvm._lib.dvm_deform_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
