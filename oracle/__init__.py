"""ORACLE -- test infrastructure only.

Plain FP64 CPU implementation (``dvm_oracle.c``) of the discrete-velocity
BGK primal/adjoint solver and wall sensitivity, used to check the GPU
library.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dvm_oracle.c")
# ORACLE_LIB names another build of the same source (the sanitizer runs)
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None
FLAGS = ["-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", *FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        D = C.c_double
        I = C.c_int
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        lp = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        L.or_create.restype = P
        L.or_create.argtypes = [I, I, I, I, dp, I, I, I, D, D, D, D, D, I, I]
        L.or_destroy.argtypes = [P]
        L.or_sizes.argtypes = [P, lp]
        L.or_export_mesh.argtypes = [P, ip, ip, dp, dp, dp, dp, dp, dp]
        L.or_export_vgrid.argtypes = [P, dp, dp]
        L.or_export_flow.argtypes = [P, dp]
        L.or_export_wall.argtypes = [P, dp, dp]
        L.or_vgrid_1d.restype = I
        L.or_vgrid_1d.argtypes = [I, I, D, D, dp, dp]
        L.or_maxwell.argtypes = [D, D, D, D, I, dp, dp]
        L.or_moments.argtypes = [I, dp, dp, dp, dp]
        L.or_dg_dW.argtypes = [D, D, D, D, D, D, dp, dp]
        L.or_primal_init.argtypes = [P]
        L.or_primal_iterate.restype = D
        L.or_primal_iterate.argtypes = [P, I]
        L.or_get_f.argtypes = [P, dp]
        L.or_set_f.argtypes = [P, dp]
        L.or_get_W.argtypes = [P, dp]
        L.or_get_phi.argtypes = [P, dp]
        L.or_set_phi.argtypes = [P, dp]
        L.or_objective.restype = D
        L.or_objective.argtypes = [P, C.c_void_p]
        L.or_cd_scale.restype = D
        L.or_cd_scale.argtypes = [P]
        L.or_primal_residual.argtypes = [P, dp, dp]
        L.or_complex_step.argtypes = [P, C.c_void_p, D, I, C.c_void_p, C.POINTER(D)]
        L.or_adjoint_init.argtypes = [P]
        L.or_adjoint_iterate.restype = D
        L.or_adjoint_iterate.argtypes = [P, I]
        L.or_adjoint_operator.argtypes = [P, dp, I, dp]
        L.or_adjoint_dJdp.restype = D
        L.or_adjoint_dJdp.argtypes = [P, I]
        L.or_wall_sensitivity.argtypes = [P, dp, dp, dp, C.c_void_p]
        L.or_mesh_sensitivity.argtypes = [P, D, dp]
        L.or_gauss_grad.argtypes = [P, I, dp]
        L.or_set_equilibrium.restype = I
        L.or_set_equilibrium.argtypes = [P, I]
        L.or_eq_params.argtypes = [P, dp, dp, dp]
        L.or_set_acceleration.restype = I
        L.or_set_acceleration.argtypes = [P, I, I]
        L.or_macro_system.argtypes = [P, dp, dp, dp, dp]
        L.or_macro_gs.restype = I
        L.or_macro_gs.argtypes = [P, dp, dp]
        L.or_macro_gs_adj.restype = I
        L.or_macro_gs_adj.argtypes = [P, dp, dp]
        L.or_wall_JB.restype = D
        L.or_wall_JB.argtypes = [P, I, D, D, D, D, D]
        L.or_set_scheme.restype = I
        L.or_set_scheme.argtypes = [P, I, I, I]
        L.or_so_slopes.argtypes = [P, dp, dp, dp]
        L.or_so_faces.argtypes = [P, dp, dp]
        _lib = L
    return _lib


def vgrid_1d(kind: int, n: int, vmax: float, param: float = 0.0):
    x = np.zeros(n)
    w = np.zeros(n)
    if lib().or_vgrid_1d(kind, n, vmax, param, x, w) != 0:
        raise ValueError("invalid velocity grid")
    return x, w


def maxwell(rho, u1, u2, th, v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    g = np.zeros((len(v), 2))
    lib().or_maxwell(rho, u1, u2, th, len(v), v, g)
    return g


def moments(v, w, f):
    W = np.zeros(4)
    lib().or_moments(len(w), np.ascontiguousarray(v, np.float64), np.ascontiguousarray(w, np.float64),
                     np.ascontiguousarray(f, np.float64), W)
    return W


def dg_dW(rho, u1, u2, th, v1, v2):
    dg = np.zeros((2, 4))
    dt = np.zeros(4)
    lib().or_dg_dW(rho, u1, u2, th, v1, v2, dg, dt)
    return dg, dt


KN, MA, TW = 1, 2, 3


class Problem:
    """One oracle solve: mesh + velocity grid + flow, primal and adjoint state."""

    def __init__(self, topology, ni, nj, n_wake, nodes, vkind, n1, n2, vmax, vparam,
                 Kn, Ma, Tw=1.0, objective=0, nthreads=None):
        if nthreads is None:
            nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        self.nthreads = nthreads
        nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        self._h = lib().or_create(topology, ni, nj, n_wake, nodes, vkind, n1, n2, vmax, vparam,
                                  float(Kn), float(Ma), float(Tw), objective, nthreads)
        if not self._h:
            raise ValueError("oracle: invalid problem")
        s = np.zeros(8, dtype=np.int64)
        lib().or_sizes(self._h, s)
        self.nc, self.nw, self.nv, self.n1, self.n2 = (int(x) for x in s[:5])
        self.ni, self.nj = int(ni), int(nj)
        self.order = 1
        self.equilibrium = 0

    def set_scheme(self, order: int = 2, limiter: bool = True, correction_every: int = 40):
        """Spatial order 1 (first-order upwind) or 2 (Green-Gauss slopes with an
        optional Venkatakrishnan limiter, iterated by defect correction with the
        correction re-evaluated every `correction_every` sweeps)."""
        if lib().or_set_scheme(self._h, int(order), 1 if limiter else 0, int(correction_every)) != 0:
            raise ValueError("oracle: invalid scheme")
        self.order = int(order)

    def set_equilibrium(self, kind: int):
        """0: pointwise Maxwellian of the cell's primitive variables; 1: the
        discrete-conservative equilibrium (moments on the grid equal W)."""
        if lib().or_set_equilibrium(self._h, int(kind)) != 0:
            raise ValueError("oracle: invalid equilibrium")
        self.equilibrium = int(kind)

    def set_acceleration(self, every: int, inner: int):
        """Macroscopic prediction every `every` primal sweeps (0: off) with
        `inner` red-black block Gauss-Seidel steps (first-order scheme); the
        adjoint iteration gets the transposed step every `every` sweeps."""
        if lib().or_set_acceleration(self._h, int(every), int(inner)) != 0:
            raise ValueError("oracle: invalid acceleration")

    def macro_system(self):
        """The macroscopic prediction's system at the current state: r [nc,4],
        D^-1 [nc,4,4] (the pseudo-time term on the diagonal included),
        off-diagonal blocks [nc,4(face),4,4] and the pseudo-time term [nc]."""
        r = np.zeros((self.nc, 4))
        Dinv = np.zeros((self.nc, 4, 4))
        O = np.zeros((self.nc, 4, 4, 4))
        lam = np.zeros(self.nc)
        lib().or_macro_system(self._h, r, Dinv, O, lam)
        return r, Dinv, O, lam

    def macro_gs(self, r):
        """x = L r, the red-black Gauss-Seidel map of the adjoint's frozen
        macroscopic system (after adjoint_init with the prediction on)."""
        r = np.ascontiguousarray(r, dtype=np.float64)
        x = np.zeros((self.nc, 4))
        if lib().or_macro_gs(self._h, r, x) != 0:
            raise ValueError("oracle: no frozen macroscopic system")
        return x

    def macro_gs_adj(self, s):
        """L^T s, the transpose of macro_gs's map."""
        s = np.ascontiguousarray(s, dtype=np.float64)
        out = np.zeros((self.nc, 4))
        if lib().or_macro_gs_adj(self._h, s, out) != 0:
            raise ValueError("oracle: no frozen macroscopic system")
        return out

    def eq_params(self, W):
        """Equilibrium parameters (rho', u1', u2', theta') of a moment vector
        W and their derivative d(.)/dW (4 x 4)."""
        P = np.zeros(4)
        M = np.zeros((4, 4))
        lib().or_eq_params(self._h, np.ascontiguousarray(W, dtype=np.float64), P, M)
        return P, M

    def so_slopes(self, f=None):
        """Limited slopes G[c, k, component, direction] and limiter factors
        psi[c, k, component] of f (default: the current f)."""
        f = self.f if f is None else np.ascontiguousarray(f, dtype=np.float64)
        G = np.zeros((self.nc, self.nv, 2, 2))
        psi = np.zeros((self.nc, self.nv, 2))
        lib().or_so_slopes(self._h, f, G, psi)
        return G, psi

    def so_faces(self, f=None):
        """Second-order face values [c, q, k, component] on each face's upwind side."""
        f = self.f if f is None else np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros((self.nc, 4, self.nv, 2))
        lib().or_so_faces(self._h, f, out)
        return out

    @classmethod
    def from_workload(cls, wl, nthreads=None, Kn=None, Ma=None, Tw=None):
        g, vg, fl = wl.grid, wl.vgrid, wl.flow
        return cls(g.topology, g.ni, g.nj, g.n_wake, g.nodes, vg.kind, vg.n1, vg.n2, vg.vmax,
                   vg.param, fl.Kn if Kn is None else Kn, fl.Ma if Ma is None else Ma,
                   fl.Tw if Tw is None else Tw, fl.objective, nthreads)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_destroy(self._h)
            self._h = None

    # mesh / grid -----------------------------------------------------
    def mesh(self):
        nbr = np.zeros((self.nc, 4), dtype=np.int32)
        wc = np.zeros(self.nw, dtype=np.int32)
        S = np.zeros((self.nc, 4, 2))
        vol = np.zeros(self.nc)
        wA = np.zeros(self.nw)
        wn = np.zeros((self.nw, 2))
        wx = np.zeros((self.nw, 2))
        cen = np.zeros((self.nc, 2))
        lib().or_export_mesh(self._h, nbr, wc, S, vol, wA, wn, wx, cen)
        return dict(nbr=nbr, wall_cell=wc, S=S, vol=vol, wall_A=wA, wall_n=wn, wall_x=wx, cen=cen)

    def vgrid(self):
        v = np.zeros((self.nv, 2))
        w = np.zeros(self.nv)
        lib().or_export_vgrid(self._h, v, w)
        return v, w

    def flow(self):
        o = np.zeros(3)
        lib().or_export_flow(self._h, o)
        return dict(inv_tau_inf=o[0], u_inf=o[1], theta_w=o[2])

    def wall(self):
        D = np.zeros(self.nw)
        F = np.zeros(self.nw)
        lib().or_export_wall(self._h, D, F)
        return D, F

    # primal ----------------------------------------------------------
    def primal_init(self):
        lib().or_primal_init(self._h)

    def primal_iterate(self, n: int) -> float:
        return lib().or_primal_iterate(self._h, int(n))

    def primal_solve(self, tol: float, max_iter: int, check_every: int = 10):
        it = 0
        r = np.inf
        while it < max_iter:
            m = min(check_every, max_iter - it)
            r = self.primal_iterate(m)
            it += m
            if r < tol:
                break
        return it, r

    @property
    def f(self):
        out = np.zeros((self.nc, self.nv, 2))
        lib().or_get_f(self._h, out)
        return out

    @f.setter
    def f(self, val):
        lib().or_set_f(self._h, np.ascontiguousarray(val, dtype=np.float64))

    @property
    def W(self):
        out = np.zeros((self.nc, 4))
        lib().or_get_W(self._h, out)
        return out

    def objective(self, per_element=False):
        Jl = np.zeros(self.nw)
        J = lib().or_objective(self._h, Jl.ctypes.data)
        return (J, Jl) if per_element else J

    def cd_scale(self):
        return lib().or_cd_scale(self._h)

    def primal_residual(self, f=None):
        f = self.f if f is None else np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros_like(f)
        lib().or_primal_residual(self._h, f, out)
        return out

    def complex_step(self, u=None, which=0, h=1e-30, want_R=True):
        dR = np.zeros((self.nc, self.nv, 2)) if want_R else None
        dJ = C.c_double(0.0)
        uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
        lib().or_complex_step(self._h, None if uu is None else uu.ctypes.data, h, which,
                              None if dR is None else dR.ctypes.data, C.byref(dJ))
        return dR, dJ.value

    # adjoint ---------------------------------------------------------
    def adjoint_init(self):
        lib().or_adjoint_init(self._h)

    def adjoint_iterate(self, n: int) -> float:
        return lib().or_adjoint_iterate(self._h, int(n))

    def adjoint_solve(self, tol: float, max_iter: int, check_every: int = 10):
        it = 0
        r = np.inf
        while it < max_iter:
            m = min(check_every, max_iter - it)
            r = self.adjoint_iterate(m)
            it += m
            if r < tol:
                break
        return it, r

    @property
    def phi(self):
        out = np.zeros((self.nc, self.nv, 2))
        lib().or_get_phi(self._h, out)
        return out

    @phi.setter
    def phi(self, val):
        lib().or_set_phi(self._h, np.ascontiguousarray(val, dtype=np.float64))

    def adjoint_operator(self, phi, with_source=True):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        out = np.zeros_like(phi)
        lib().or_adjoint_operator(self._h, phi, 1 if with_source else 0, out)
        return out

    def adjoint_dJdp(self, which: int) -> float:
        return lib().or_adjoint_dJdp(self._h, which)

    def wall_sensitivity(self):
        SA = np.zeros(self.nw)
        Sx = np.zeros((self.nw, 2))
        Sn = np.zeros((self.nw, 2))
        dn = np.zeros((self.nw, 2))
        lib().or_wall_sensitivity(self._h, SA, Sx, Sn, dn.ctypes.data)
        return dict(S_A=SA, S_x=Sx, S_n=Sn, dJ_dnodes=dn)

    def mesh_sensitivity(self, h: float = 1e-30):
        """dL/dx for every mesh node coordinate, shape (nj+1, ni+1, 2): the
        exact discrete shape derivative at converged f and phi (order 2:
        with the limiter factors of f held fixed, exact with the limiter
        off)."""
        out = np.zeros((self.nj + 1, self.ni + 1, 2))
        lib().or_mesh_sensitivity(self._h, float(h), out)
        return out

    def gauss_grad(self, c: int):
        """Green-Gauss gradient of eq. (gaussgrad) at cell c with the current
        f: [velocity, component, direction]."""
        out = np.zeros((self.nv, 2, 2))
        lib().or_gauss_grad(self._h, int(c), out)
        return out

    def wall_JB(self, l, A, x, n):
        return lib().or_wall_JB(self._h, int(l), float(A), float(x[0]), float(x[1]),
                                float(n[0]), float(n[1]))
