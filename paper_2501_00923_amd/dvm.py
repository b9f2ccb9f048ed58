"""Python binding of libdvm (include/dvm.h): argument marshalling only.

Every step of the solver runs in the HIP library; PyTorch provides the device
buffers (one uint8 tensor per solver workspace) and the HIP stream.  If the
built library is missing this module raises instead of falling back to
anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DVM_LIB names another build of the same sources (the host-sanitizer runs)
LIB_PATH = os.environ.get("DVM_LIB") or os.path.join(_HERE, "libdvm.so")

DVM_OK, DVM_EINVAL, DVM_ENOMEM, DVM_EHIP, DVM_ENOTCONV, DVM_ENAN, DVM_ESTATE = 0, -1, -2, -3, -4, -5, -6
TOPO_O, TOPO_C = 0, 1
FP64, MIXED = 0, 1
OBJ_DRAG, OBJ_HEAT = 0, 1
VG_MIDPOINT, VG_NEWTON_COTES, VG_SINH = 0, 1, 2
STATE_F, STATE_PHI, STATE_PHI_ROWS = 0, 1, 2
LIMITER_NONE, LIMITER_VENKAT = 0, 1
EQ_POINTWISE, EQ_CONSERVATIVE = 0, 1
MAX_PARAMS = 64

_ERRNAMES = {DVM_EINVAL: "EINVAL", DVM_ENOMEM: "ENOMEM", DVM_EHIP: "EHIP", DVM_ENOTCONV: "ENOTCONV",
             DVM_ENAN: "ENAN", DVM_ESTATE: "ESTATE"}

EXPORTED = [
    "dvm_mesh_create", "dvm_mesh_info", "dvm_mesh_export", "dvm_mesh_destroy",
    "dvm_vgrid_create", "dvm_vgrid_info", "dvm_vgrid_export", "dvm_vgrid_destroy",
    "dvm_solver_create", "dvm_solver_set_scheme", "dvm_solver_set_equilibrium", "dvm_solver_set_acceleration",
    "dvm_solver_workspace_bytes",
    "dvm_solver_bind",
    "dvm_solver_set_stream",
    "dvm_primal_init", "dvm_primal_iterate", "dvm_primal_sweeps", "dvm_objective", "dvm_read_moments",
    "dvm_adjoint_init", "dvm_adjoint_iterate", "dvm_adjoint_sweeps",
    "dvm_wall_sensitivity", "dvm_param_sensitivity", "dvm_mesh_sensitivity",
    "dvm_state_bytes", "dvm_state_save", "dvm_state_load", "dvm_state_copy",
    "dvm_batch_work_bytes", "dvm_batch_create", "dvm_batch_create_static", "dvm_batch_run", "dvm_batch_residual",
    "dvm_batch_destroy",
    "dvm_solver_iterations", "dvm_solver_phase", "dvm_last_error", "dvm_solver_destroy",
    "dvm_cst_eval", "dvm_cst_fit", "dvm_volume_constraint",
    "dvm_deform_create", "dvm_deform_workspace_bytes", "dvm_deform_bind", "dvm_deform_apply",
    "dvm_deform_chain", "dvm_deform_destroy",
]


class DvmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dvm {_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class NotConverged(DvmError):
    pass


_lib = None


def lib():
    """Load libdvm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built; run paper_2501_00923_amd/build.py (or __graft_entry__.build())")
    # torch carries its own HIP runtime; bring it up before libdvm's so that
    # both see the device whichever the caller touches first
    try:
        import torch
        torch.cuda.is_available()
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, d, sz = C.c_void_p, C.c_int, C.c_int64, C.c_double, C.c_size_t
    pvp, pi, pd = C.POINTER(C.c_void_p), C.POINTER(C.c_int), C.POINTER(C.c_double)
    sig = {
        "dvm_mesh_create": (i32, [i32, i32, i32, i32, vp, pvp]),
        "dvm_mesh_info": (i32, [vp, vp, vp]),
        "dvm_mesh_export": (i32, [vp] + [vp] * 7),
        "dvm_mesh_destroy": (None, [vp]),
        "dvm_vgrid_create": (i32, [i32, i32, i32, d, d, pvp]),
        "dvm_vgrid_info": (i32, [vp, vp]),
        "dvm_vgrid_export": (i32, [vp, vp, vp]),
        "dvm_vgrid_destroy": (None, [vp]),
        "dvm_solver_create": (i32, [vp, vp, vp, i32, i32, pvp]),
        "dvm_solver_set_scheme": (i32, [vp, i32, i32, i32]),
        "dvm_solver_set_equilibrium": (i32, [vp, i32]),
        "dvm_solver_set_acceleration": (i32, [vp, i32, i32]),
        "dvm_solver_workspace_bytes": (sz, [vp]),
        "dvm_solver_bind": (i32, [vp, vp, sz, vp]),
        "dvm_solver_set_stream": (i32, [vp, vp]),
        "dvm_primal_init": (i32, [vp]),
        "dvm_primal_iterate": (i32, [vp, i32, d, i32, pi, pd]),
        "dvm_primal_sweeps": (i32, [vp, i32]),
        "dvm_objective": (i32, [vp, pd, pd]),
        "dvm_read_moments": (i32, [vp, vp]),
        "dvm_adjoint_init": (i32, [vp]),
        "dvm_adjoint_iterate": (i32, [vp, i32, d, i32, pi, pd]),
        "dvm_adjoint_sweeps": (i32, [vp, i32]),
        "dvm_wall_sensitivity": (i32, [vp, vp, vp, vp, vp]),
        "dvm_param_sensitivity": (i32, [vp, i32, vp, vp]),
        "dvm_mesh_sensitivity": (i32, [vp, vp]),
        "dvm_state_bytes": (sz, [vp, i32]),
        "dvm_state_save": (i32, [vp, i32, vp, sz]),
        "dvm_state_load": (i32, [vp, i32, vp, sz]),
        "dvm_state_copy": (i32, [vp, vp, i32]),
        "dvm_batch_work_bytes": (sz, [i32, i64]),
        "dvm_batch_create": (i32, [vp, i32, vp, sz, vp, pvp]),
        "dvm_batch_create_static": (i32, [vp, i32, vp, pvp]),
        "dvm_batch_run": (i32, [vp, i32]),
        "dvm_batch_residual": (i32, [vp, vp]),
        "dvm_batch_destroy": (None, [vp]),
        "dvm_solver_iterations": (i32, [vp, i32]),
        "dvm_solver_phase": (i32, [vp]),
        "dvm_last_error": (C.c_char_p, []),
        "dvm_solver_destroy": (None, [vp]),
        "dvm_cst_eval": (i32, [i32, vp, i32, vp, vp, vp, vp]),
        "dvm_cst_fit": (i32, [i32, i32, vp, vp, vp, vp, vp, pd]),
        "dvm_volume_constraint": (i32, [i32, vp, d, pd, vp]),
        "dvm_deform_create": (i32, [vp, d, pvp]),
        "dvm_deform_workspace_bytes": (sz, [vp]),
        "dvm_deform_bind": (i32, [vp, vp, sz, vp]),
        "dvm_deform_apply": (i32, [vp, vp, vp]),
        "dvm_deform_chain": (i32, [vp, vp, vp]),
        "dvm_deform_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(code: int):
    if code != DVM_OK:
        msg = lib().dvm_last_error().decode(errors="replace")
        if code == DVM_ENOTCONV:
            raise NotConverged(code, msg)
        raise DvmError(code, msg)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class _Flow(C.Structure):
    _fields_ = [("Kn", C.c_double), ("Ma", C.c_double), ("Tw", C.c_double), ("objective", C.c_int)]


class Mesh:
    def __init__(self, topology: int, ni: int, nj: int, n_wake: int, nodes: np.ndarray):
        nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        if nodes.size != 2 * (ni + 1) * (nj + 1):
            raise ValueError("nodes must hold (nj+1)*(ni+1)*2 values")
        h = C.c_void_p()
        _check(lib().dvm_mesh_create(topology, ni, nj, n_wake, nodes.ctypes.data, C.byref(h)))
        self._h = h
        nc, nw = C.c_int32(), C.c_int32()
        _check(lib().dvm_mesh_info(h, C.byref(nc), C.byref(nw)))
        self.nc, self.nw = nc.value, nw.value
        self.topology, self.ni, self.nj, self.n_wake = topology, ni, nj, n_wake

    @classmethod
    def from_grid(cls, g):
        return cls(g.topology, g.ni, g.nj, g.n_wake, g.nodes)

    def export(self):
        nbr = np.zeros((self.nc, 4), np.int32)
        wc = np.zeros(self.nw, np.int32)
        S = np.zeros((self.nc, 4, 2))
        vol = np.zeros(self.nc)
        wA = np.zeros(self.nw)
        wn = np.zeros((self.nw, 2))
        wx = np.zeros((self.nw, 2))
        _check(lib().dvm_mesh_export(self._h, _ptr(nbr), _ptr(wc), _ptr(S), _ptr(vol), _ptr(wA), _ptr(wn), _ptr(wx)))
        return dict(nbr=nbr, wall_cell=wc, S=S, vol=vol, wall_A=wA, wall_n=wn, wall_x=wx)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dvm_mesh_destroy(self._h)
            self._h = None


class VGrid:
    def __init__(self, kind: int, n1: int, n2: int, vmax: float, param: float = 0.0):
        h = C.c_void_p()
        _check(lib().dvm_vgrid_create(kind, n1, n2, float(vmax), float(param), C.byref(h)))
        self._h = h
        self.n1, self.n2, self.nv = n1, n2, n1 * n2

    @classmethod
    def from_spec(cls, vs):
        return cls(vs.kind, vs.n1, vs.n2, vs.vmax, vs.param)

    def export(self):
        v = np.zeros((self.nv, 2))
        w = np.zeros(self.nv)
        _check(lib().dvm_vgrid_export(self._h, _ptr(v), _ptr(w)))
        return v, w

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dvm_vgrid_destroy(self._h)
            self._h = None


def _torch():
    import torch
    return torch


def current_stream_handle():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def alloc_device(nbytes: int):
    """A 256-byte aligned torch uint8 device buffer (the caching allocator
    aligns to 512 bytes)."""
    torch = _torch()
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")
    assert t.data_ptr() % 256 == 0
    return t


class Solver:
    """One primal/adjoint solve bound to a torch-allocated workspace."""

    def __init__(self, mesh: Mesh, vgrid: VGrid, Kn: float, Ma: float, Tw: float = 1.0,
                 objective: int = OBJ_DRAG, precision: int = FP64, want_adjoint: bool = True,
                 buffer=None, stream=None, bind: bool = True, order: int = 1, limiter: int = LIMITER_VENKAT,
                 correction_every: int = 40, equilibrium: int = EQ_POINTWISE, accelerate=None):
        fl = _Flow(float(Kn), float(Ma), float(Tw), int(objective))
        h = C.c_void_p()
        _check(lib().dvm_solver_create(mesh._h, vgrid._h, C.byref(fl), precision, 1 if want_adjoint else 0,
                                       C.byref(h)))
        self._h = h
        if order != 1:
            _check(lib().dvm_solver_set_scheme(h, int(order), int(limiter), int(correction_every)))
        if equilibrium != EQ_POINTWISE:
            _check(lib().dvm_solver_set_equilibrium(h, int(equilibrium)))
        if accelerate:
            # (every, inner): macroscopic prediction every `every` primal sweeps
            _check(lib().dvm_solver_set_acceleration(h, int(accelerate[0]), int(accelerate[1])))
        self.accelerate = tuple(accelerate) if accelerate else None
        self.order = order
        self.equilibrium = equilibrium
        self.nc, self.nw, self.nv = mesh.nc, mesh.nw, vgrid.nv
        self.ni, self.nj = mesh.ni, mesh.nj
        self.precision = precision
        self.workspace_bytes = int(lib().dvm_solver_workspace_bytes(h))
        self.buffer = None
        if bind:
            self.bind(buffer, stream)

    @classmethod
    def from_workload(cls, wl, precision=FP64, want_adjoint=True, **kw):
        return cls(Mesh.from_grid(wl.grid), VGrid.from_spec(wl.vgrid), wl.flow.Kn, wl.flow.Ma, wl.flow.Tw,
                   wl.flow.objective, precision, want_adjoint, **kw)

    def bind(self, buffer=None, stream=None):
        if buffer is None:
            buffer = alloc_device(self.workspace_bytes)
        self.buffer = buffer
        st = current_stream_handle() if stream is None else C.c_void_p(int(stream))
        _check(lib().dvm_solver_bind(self._h, C.c_void_p(buffer.data_ptr()), C.c_size_t(buffer.numel()), st))

    def set_stream(self, stream):
        _check(lib().dvm_solver_set_stream(self._h, C.c_void_p(int(stream))))

    # primal --------------------------------------------------------------
    def primal_init(self):
        _check(lib().dvm_primal_init(self._h))

    def primal_iterate(self, max_iter: int, tol: float = 0.0, check_every: int = 0, raise_notconv=True):
        it, r = C.c_int(), C.c_double()
        code = lib().dvm_primal_iterate(self._h, int(max_iter), float(tol), int(check_every), C.byref(it), C.byref(r))
        if code != DVM_ENOTCONV or raise_notconv:
            _check(code)
        return it.value, r.value

    def primal_sweeps(self, n: int):
        _check(lib().dvm_primal_sweeps(self._h, int(n)))

    def objective(self):
        J, Cd = C.c_double(), C.c_double()
        _check(lib().dvm_objective(self._h, C.byref(J), C.byref(Cd)))
        return J.value, Cd.value

    def moments(self):
        W = np.zeros((self.nc, 4))
        _check(lib().dvm_read_moments(self._h, W.ctypes.data))
        return W

    # adjoint -------------------------------------------------------------
    def adjoint_init(self):
        _check(lib().dvm_adjoint_init(self._h))

    def adjoint_iterate(self, max_iter: int, tol: float = 0.0, check_every: int = 0, raise_notconv=True):
        it, r = C.c_int(), C.c_double()
        code = lib().dvm_adjoint_iterate(self._h, int(max_iter), float(tol), int(check_every), C.byref(it), C.byref(r))
        if code != DVM_ENOTCONV or raise_notconv:
            _check(code)
        return it.value, r.value

    def adjoint_sweeps(self, n: int):
        _check(lib().dvm_adjoint_sweeps(self._h, int(n)))

    def wall_sensitivity(self):
        SA = np.zeros(self.nw)
        Sx = np.zeros((self.nw, 2))
        Sn = np.zeros((self.nw, 2))
        dn = np.zeros((self.nw, 2))
        _check(lib().dvm_wall_sensitivity(self._h, _ptr(SA), _ptr(Sx), _ptr(Sn), _ptr(dn)))
        return dict(S_A=SA, S_x=Sx, S_n=Sn, dJ_dnodes=dn)

    def mesh_sensitivity(self) -> np.ndarray:
        """Exact discrete dJ/d(node coordinates), shape (nj+1, ni+1, 2)."""
        out = np.zeros((self.nj + 1, self.ni + 1, 2))
        _check(lib().dvm_mesh_sensitivity(self._h, _ptr(out)))
        return out

    def param_sensitivity(self, wall_jac: np.ndarray) -> np.ndarray:
        wall_jac = np.ascontiguousarray(wall_jac, dtype=np.float64)
        npar = wall_jac.shape[-1]
        out = np.zeros(npar)
        _check(lib().dvm_param_sensitivity(self._h, npar, wall_jac.ctypes.data, out.ctypes.data))
        return out

    # checkpoint ------------------------------------------------------------
    def state_bytes(self, which: int) -> int:
        return int(lib().dvm_state_bytes(self._h, which))

    def state_save(self, which: int, out: Optional[np.ndarray] = None) -> np.ndarray:
        n = self.state_bytes(which)
        if out is None:
            out = np.empty(n, dtype=np.uint8)
        _check(lib().dvm_state_save(self._h, which, out.ctypes.data, out.nbytes))
        return out

    def state_load(self, which: int, blob: np.ndarray):
        blob = np.ascontiguousarray(blob)
        _check(lib().dvm_state_load(self._h, which, blob.ctypes.data, blob.nbytes))

    def state_copy_from(self, src: "Solver", which: int):
        """Device-to-device copy of src's f or phi into this solver."""
        _check(lib().dvm_state_copy(self._h, src._h, int(which)))

    def iterations(self, phase: int) -> int:
        return int(lib().dvm_solver_iterations(self._h, phase))

    @property
    def phase(self) -> int:
        return int(lib().dvm_solver_phase(self._h))

    def state_array(self, which: int = STATE_F) -> np.ndarray:
        """f or phi as [nc][nv][2] float64 (copy)."""
        raw = self.state_save(which)
        dt = np.float32 if self.precision == MIXED else np.float64
        n = self.nc * self.nv * 2
        rows = np.frombuffer(raw, dtype=dt, count=n).reshape(self.nc, self.nv, 2)
        return rows.astype(np.float64) if dt != np.float64 else rows

    def state_load_array(self, which: int, rows: np.ndarray):
        """Load f (STATE_F) or phi alone (STATE_PHI_ROWS) from a [nc][nv][2]
        array, converted to the storage precision."""
        dt = np.float32 if self.precision == MIXED else np.float64
        self.state_load(which, np.ascontiguousarray(rows, dtype=dt))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dvm_solver_destroy(self._h)
            self._h = None


class Batch:
    """A group of bound solvers advanced together (one launch per sweep).
    static=True: the allocation-free form (dvm_batch_create_static), whose
    launch tables live in the library's fixed per-device array."""

    def __init__(self, solvers: Sequence[Solver], stream=None, work=None, static: bool = False):
        self.solvers = list(solvers)
        n = len(self.solvers)
        arr = (C.c_void_p * n)(*[s._h.value for s in self.solvers])
        self._arr = arr
        st = current_stream_handle() if stream is None else C.c_void_p(int(stream))
        h = C.c_void_p()
        if static:
            self.work = None
            _check(lib().dvm_batch_create_static(arr, n, st, C.byref(h)))
        else:
            total = sum(s.nc for s in self.solvers)
            need = int(lib().dvm_batch_work_bytes(n, total))
            self.work = alloc_device(need) if work is None else work
            _check(lib().dvm_batch_create(arr, n, C.c_void_p(self.work.data_ptr()), self.work.numel(), st,
                                          C.byref(h)))
        self._h = h

    def run(self, iters: int):
        _check(lib().dvm_batch_run(self._h, int(iters)))

    def residuals(self) -> np.ndarray:
        out = np.zeros(len(self.solvers))
        _check(lib().dvm_batch_residual(self._h, out.ctypes.data))
        return out

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dvm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
