"""Seeded synthetic inputs shared by the GPU library and the CPU oracle.

This module holds no arithmetic of the kinetic method (no Maxwellian, no
moments, no fluxes, no adjoint, no sensitivity).  It only manufactures the
*inputs* the method is applied to:

* body-fitted structured grids, as node coordinates of an O-grid around a
  perturbed circle or a C-grid around a (perturbed) NACA 4-digit profile;
* the Jacobian of the wall nodes (and of every mesh node) with respect to the
  shape parameters that perturb the wall, so that a wall-node sensitivity can
  be chained to parameters by either side;
* workload descriptions (flow state, velocity-grid recipe, seeds) for the
  circle / NACA cases and the request stream of the solve server.

The paper (Sec. 4) runs on unstructured body-fitted meshes that are not
published; these structured grids stand in for them with the same features
(body-fitted, wall-refined first layer, far field at about ten chords).

Node array convention (both topologies): ``nodes[j, i] = (x, y)`` for
``j in [0, nj]`` (``j = 0`` on the wall / wake cut, ``j = nj`` far field) and
``i in [0, ni]``.  The wall is walked clockwise around the body as ``i``
grows, so the quadrilateral (i,j),(i+1,j),(i+1,j+1),(i,j+1) is
counter-clockwise.  For the O-grid column ``ni`` repeats column 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

TOPO_O = 0
TOPO_C = 1

VG_MIDPOINT = 0
VG_NEWTON_COTES = 1
VG_SINH = 2


@dataclass
class GridInput:
    """A structured body-fitted grid plus its shape-parameter Jacobians."""

    topology: int
    ni: int
    nj: int
    n_wake: int
    nodes: np.ndarray            # (nj+1, ni+1, 2) float64
    wall_jac: np.ndarray         # (n_wall_nodes, 2, n_params) d(wall node)/d(alpha)
    node_jac: np.ndarray         # (nj+1, ni+1, 2, n_params) d(node)/d(alpha)
    params: np.ndarray           # (n_params,) the alpha the grid was built at
    param_names: list = field(default_factory=list)

    @property
    def n_cells(self) -> int:
        return self.ni * self.nj

    @property
    def n_wall(self) -> int:
        return self.ni - 2 * self.n_wake

    def wall_nodes(self) -> np.ndarray:
        """Wall node coordinates in wall order (closed loop, no repeat)."""
        return self.nodes[0, self.n_wake:self.n_wake + self.n_wall].copy()


@dataclass
class VGridSpec:
    kind: int
    n1: int
    n2: int
    vmax: float
    param: float = 0.0


@dataclass
class FlowSpec:
    Kn: float
    Ma: float
    Tw: float = 1.0
    objective: int = 0  # 0 = drag (m_J = v1), 1 = heat (m_J = |v|^2 / 2)


def _geom_fractions(n: int, first: float) -> np.ndarray:
    """s_0 = 0 < s_1 = first < ... < s_n = 1, geometric spacing."""
    if n == 1:
        return np.array([0.0, 1.0])
    if abs(first * n - 1.0) < 1e-14:
        return np.arange(n + 1, dtype=np.float64) / n
    # find ratio r with first*(r^n - 1)/(r - 1) = 1
    def total(r):
        if abs(r - 1.0) < 1e-14:
            return first * n
        return first * (r ** n - 1.0) / (r - 1.0)
    lo, hi = (1.0 + 1e-15, 10.0) if first * n < 1.0 else (1e-6, 1.0 - 1e-15)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if (total(mid) < 1.0) == (first * n < 1.0):
            lo = mid
        else:
            hi = mid
    r = 0.5 * (lo + hi)
    s = np.empty(n + 1)
    s[0] = 0.0
    acc = 0.0
    step = first
    for j in range(1, n + 1):
        acc += step
        s[j] = acc
        step *= r
    s /= s[-1]
    return s


def _ratio_fractions(n: int, ratio: float) -> np.ndarray:
    if ratio == 1.0:
        return np.arange(n + 1, dtype=np.float64) / n
    j = np.arange(n + 1, dtype=np.float64)
    return (ratio ** j - 1.0) / (ratio ** n - 1.0)


# --------------------------------------------------------------------------
# O-grid around a circle with radial Fourier perturbation
# --------------------------------------------------------------------------

def ogrid(ni: int = 64, nj: int = 32, r_outer: float = 10.0, stretch: float = 1.1,
          a: Optional[np.ndarray] = None, b: Optional[np.ndarray] = None) -> GridInput:
    """O-grid around r(t) = 1 + sum_m a_m cos(m t) + sum_m b_m sin(m t).

    ``a`` has modes m = 0..len(a)-1, ``b`` modes m = 1..len(b).  The wall
    node i sits at angle t_i = -2 pi i / ni (clockwise walk); radial lines
    go straight to radius ``r_outer`` with geometric spacing ratio ``stretch``.
    """
    a = np.zeros(4) if a is None else np.asarray(a, dtype=np.float64)
    b = np.zeros(4) if b is None else np.asarray(b, dtype=np.float64)
    t = -2.0 * math.pi * np.arange(ni) / ni
    e = np.stack([np.cos(t), np.sin(t)], axis=1)              # (ni, 2)
    r = np.ones(ni)
    basis = []
    names = []
    for m in range(len(a)):
        r = r + a[m] * np.cos(m * t)
        basis.append(np.cos(m * t))
        names.append(f"a{m}")
    for m in range(1, len(b) + 1):
        r = r + b[m - 1] * np.sin(m * t)
        basis.append(np.sin(m * t))
        names.append(f"b{m}")
    basis = np.stack(basis, axis=1)                              # (ni, np)
    P = r[:, None] * e
    Q = r_outer * e
    s = _ratio_fractions(nj, stretch)
    nodes = np.empty((nj + 1, ni + 1, 2))
    nodes[:, :ni] = P[None] + s[:, None, None] * (Q - P)[None]
    nodes[:, ni] = nodes[:, 0]
    wall_jac = e[:, :, None] * basis[:, None, :]                 # (ni, 2, np)
    node_jac = np.empty((nj + 1, ni + 1, 2, basis.shape[1]))
    node_jac[:, :ni] = (1.0 - s)[:, None, None, None] * wall_jac[None]
    node_jac[:, ni] = node_jac[:, 0]
    return GridInput(TOPO_O, ni, nj, 0, np.ascontiguousarray(nodes), wall_jac,
                     node_jac, np.concatenate([a, b]), names)


# --------------------------------------------------------------------------
# C-grid around a NACA 4-digit profile
# --------------------------------------------------------------------------

def naca4(xi: np.ndarray, t: float, m: float, p: float, upper: bool):
    """Public NACA 4-digit definition, closed trailing edge (coefficient
    -0.1036 on x^4).  Returns (x, y) of the upper or lower surface at chord
    stations ``xi`` in [0, 1]."""
    xi = np.asarray(xi, dtype=np.float64)
    yt = 5.0 * t * (0.2969 * np.sqrt(np.maximum(xi, 0.0)) - 0.1260 * xi
                    - 0.3516 * xi ** 2 + 0.2843 * xi ** 3 - 0.1036 * xi ** 4)
    if m == 0.0:
        yc = np.zeros_like(xi)
        th = np.zeros_like(xi)
    else:
        fore = xi < p
        yc = np.where(fore, m / p ** 2 * (2 * p * xi - xi ** 2),
                      m / (1 - p) ** 2 * ((1 - 2 * p) + 2 * p * xi - xi ** 2))
        dyc = np.where(fore, 2 * m / p ** 2 * (p - xi), 2 * m / (1 - p) ** 2 * (p - xi))
        th = np.arctan(dyc)
    if upper:
        return xi - yt * np.sin(th), yc + yt * np.cos(th)
    return xi + yt * np.sin(th), yc - yt * np.cos(th)


def hicks_henne(xi: np.ndarray, h: float) -> np.ndarray:
    """Hicks-Henne bump sin^3(pi xi^{ln 0.5 / ln h}), peak at xi = h."""
    e = math.log(0.5) / math.log(h)
    return np.sin(math.pi * np.power(np.clip(xi, 0.0, 1.0), e)) ** 3


def bspline_basis(xi: np.ndarray, n_ctrl: int, degree: int = 3) -> np.ndarray:
    """Clamped uniform B-spline basis N_c(xi), c = 0..n_ctrl-1, on [0, 1]
    (Cox-de Boor recursion).  Returns (len(xi), n_ctrl)."""
    xi = np.clip(np.asarray(xi, dtype=np.float64), 0.0, 1.0)
    n_int = n_ctrl - degree
    knots = np.concatenate([np.zeros(degree), np.linspace(0.0, 1.0, n_int + 1),
                            np.ones(degree)])
    nk = len(knots)
    N = np.zeros((len(xi), nk - 1))
    for c in range(nk - 1):
        lo, hi = knots[c], knots[c + 1]
        if hi > lo:
            last = hi == 1.0
            N[:, c] = ((xi >= lo) & ((xi < hi) | (last & (xi <= hi)))).astype(np.float64)
    for d in range(1, degree + 1):
        M = np.zeros((len(xi), nk - 1 - d))
        for c in range(nk - 1 - d):
            den1 = knots[c + d] - knots[c]
            den2 = knots[c + d + 1] - knots[c + 1]
            if den1 > 0:
                M[:, c] += (xi - knots[c]) / den1 * N[:, c]
            if den2 > 0:
                M[:, c] += (knots[c + d + 1] - xi) / den2 * N[:, c + 1]
        N = M
    return N[:, :n_ctrl]


def naca_cgrid(n_wake: int = 32, n_half: int = 96, nj: int = 128, t: float = 0.12,
               m: float = 0.0, p: float = 0.4, r_outer: float = 10.0, h1: float = 1e-3,
               perturb: Optional[dict] = None) -> GridInput:
    """C-grid around a NACA 4-digit profile (chord 1, leading edge at 0).

    ``ni = 2 n_wake + 2 n_half`` cells along the C: ``n_wake`` lower wake
    cells (downstream end to trailing edge), ``n_half`` lower-surface cells
    (trailing edge to leading edge, cosine clustered), ``n_half`` upper
    surface cells, ``n_wake`` upper wake cells.  Grid lines run straight
    from each inner node to its partner on the outer C (two horizontal lines
    at y = +-r_outer joined by a half circle of radius r_outer about the
    trailing edge); first-layer height ``h1`` (relative spacing h1/r_outer).

    ``perturb``: None, or
      {"kind": "hicks_henne", "h": positions (nb_up + nb_lo), "n_up": nb_up,
       "amp": amplitudes}  -- upper bumps raise y, lower bumps lower y;
      {"kind": "bspline", "n_ctrl": 14, "amp": 2*(n_ctrl-2) free offsets}
       -- clamped cubic B-spline vertical offsets, end control points fixed
       at zero, first half of ``amp`` upper surface, second half lower.
    """
    ni = 2 * n_wake + 2 * n_half
    nw = 2 * n_half                     # wall faces = wall nodes (closed loop)
    q = np.arange(nw)
    lower = q <= n_half
    beta = np.where(lower, math.pi * (1.0 - q / n_half), math.pi * (q - n_half) / n_half)
    xi = 0.5 * (1.0 - np.cos(beta))
    xl, yl = naca4(xi, t, m, p, upper=False)
    xu, yu = naca4(xi, t, m, p, upper=True)
    wx = np.where(lower, xl, xu)
    wy = np.where(lower, yl, yu)
    wx[0], wy[0] = 1.0, 0.0            # trailing edge exactly closed
    # shape-parameter basis (vertical offsets)
    if perturb is None:
        basis = np.zeros((nw, 0))
        amp = np.zeros(0)
        names = []
    elif perturb["kind"] == "hicks_henne":
        hs = np.asarray(perturb["h"], dtype=np.float64)
        n_up = int(perturb["n_up"])
        amp = np.asarray(perturb.get("amp", np.zeros(len(hs))), dtype=np.float64)
        basis = np.zeros((nw, len(hs)))
        upper_mask = ~lower
        upper_mask[n_half] = False
        for k, h in enumerate(hs):
            bk = hicks_henne(xi, h)
            if k < n_up:
                basis[:, k] = np.where(upper_mask, bk, 0.0)
            else:
                basis[:, k] = np.where(lower & (q != n_half) & (q != 0), -bk, 0.0)
        names = [f"hh_up{k}" for k in range(n_up)] + [f"hh_lo{k}" for k in range(len(hs) - n_up)]
    elif perturb["kind"] == "bspline":
        nc = int(perturb.get("n_ctrl", 14))
        nfree = nc - 2
        amp = np.asarray(perturb.get("amp", np.zeros(2 * nfree)), dtype=np.float64)
        Nb = bspline_basis(xi, nc)[:, 1:nc - 1]                  # (nw, nfree)
        basis = np.zeros((nw, 2 * nfree))
        upper_mask = ~lower
        upper_mask[n_half] = False
        lo_mask = lower.copy()
        lo_mask[0] = False
        lo_mask[n_half] = False
        basis[:, :nfree] = np.where(upper_mask[:, None], Nb, 0.0)
        basis[:, nfree:] = np.where(lo_mask[:, None], Nb, 0.0)
        names = [f"bs_up{k}" for k in range(nfree)] + [f"bs_lo{k}" for k in range(nfree)]
    else:
        raise ValueError(f"unknown perturbation {perturb['kind']}")
    wy = wy + basis @ amp if basis.shape[1] else wy
    wall_jac = np.zeros((nw, 2, basis.shape[1]))
    wall_jac[:, 1, :] = basis

    # wake stations: geometric from the trailing-edge panel length to r_outer
    d0 = 0.5 * (1.0 - math.cos(math.pi / n_half))
    sw = _geom_fractions(n_wake, d0 / r_outer)
    xw = 1.0 + r_outer * sw                                        # (n_wake+1,)

    P = np.zeros((ni + 1, 2))
    Q = np.zeros((ni + 1, 2))
    for i in range(n_wake + 1):                                    # lower wake
        P[i] = (xw[n_wake - i], 0.0)
        Q[i] = (xw[n_wake - i], -r_outer)
    for k in range(nw + 1):                                        # surface
        i = n_wake + k
        kk = k % nw
        P[i] = (wx[kk], wy[kk])
        sig = k / nw
        ph = -0.5 * math.pi - math.pi * sig
        Q[i] = (1.0 + r_outer * math.cos(ph), r_outer * math.sin(ph))
    for k in range(n_wake + 1):                                    # upper wake
        i = ni - n_wake + k
        P[i] = (xw[k], 0.0)
        Q[i] = (xw[k], r_outer)
    s = _geom_fractions(nj, h1 / r_outer)
    nodes = P[None] + s[:, None, None] * (Q - P)[None]
    npar = basis.shape[1]
    node_jac = np.zeros((nj + 1, ni + 1, 2, npar))
    for k in range(nw + 1):
        i = n_wake + k
        node_jac[:, i] = (1.0 - s)[:, None, None] * wall_jac[k % nw][None]
    return GridInput(TOPO_C, ni, nj, n_wake, np.ascontiguousarray(nodes), wall_jac,
                     node_jac, amp.copy(), names)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    grid: GridInput
    vgrid: VGridSpec
    flow: FlowSpec
    seed: int
    note: str = ""


def circle_case(ni=64, nj=32, nv=16, vmax=5.0, Kn=1.0, Ma=0.5, Tw=1.0,
                a=None, b=None, r_outer=10.0, stretch=1.1, kind=VG_MIDPOINT) -> Workload:
    """Flow past a (perturbed) unit circle; 8 radial Fourier modes."""
    g = ogrid(ni, nj, r_outer, stretch, a, b)
    return Workload(f"circle_o{ni}x{nj}_v{nv}", g, VGridSpec(kind, nv, nv, vmax),
                    FlowSpec(Kn, Ma, Tw), 0)


def c1_circle(seed: int = 0) -> Workload:
    """Unit circle, O-grid 64x32 (outer radius 10, stretch 1.1), 16x16
    midpoint velocity grid on [-5, 5], Kn 1, Ma 0.5, Tw 1; 8 Fourier modes
    evaluated at zero amplitude."""
    w = circle_case()
    w.name, w.seed = "circle_o64x32_v16_kn1_ma0.5", seed
    return w


def c2_naca(seed: int = 0, n_bumps: int = 16) -> Workload:
    """NACA0012 C-grid 256x128, 48x48 Newton-Cotes grid on [-6, 6], Kn 0.1,
    Ma 0.8, Tw 1; 16 Hicks-Henne bumps at seed-drawn positions in [0.05, 0.95]
    (8 upper, 8 lower), amplitudes zero."""
    rng = np.random.default_rng(seed)
    h = rng.uniform(0.05, 0.95, size=n_bumps)
    g = naca_cgrid(32, 96, 128, t=0.12, m=0.0,
                   perturb={"kind": "hicks_henne", "h": h, "n_up": n_bumps // 2,
                            "amp": np.zeros(n_bumps)})
    return Workload("naca0012_c256x128_v48nc_kn0.1_ma0.8", g,
                    VGridSpec(VG_NEWTON_COTES, 48, 48, 6.0), FlowSpec(0.1, 0.8, 1.0), seed)


def c3_naca_sinh(Kn: float, seed: int = 0) -> Workload:
    """Same 256x128 NACA0012 C-grid, 64x64 sinh-stretched velocity grid on
    [-6, 6] (denser near 0), Ma 0.5, Tw 1, Kn in {1e-3, 1e-2, 0.1, 1, 10}."""
    rng = np.random.default_rng(seed)
    h = rng.uniform(0.05, 0.95, size=16)
    g = naca_cgrid(32, 96, 128, t=0.12, m=0.0,
                   perturb={"kind": "hicks_henne", "h": h, "n_up": 8, "amp": np.zeros(16)})
    return Workload(f"naca0012_c256x128_v64sinh_kn{Kn:g}_ma0.5", g,
                    VGridSpec(VG_SINH, 64, 64, 6.0, 2.0), FlowSpec(Kn, 0.5, 1.0), seed)


def c4_naca_bspline(seed: int = 0) -> Workload:
    """Seed-drawn NACA (thickness U[0.08, 0.16], camber U[0, 0.04] at 0.4
    chord), C-grid 192x96 (24 wake + 72 + 72 surface + 24 wake), 48x48
    Newton-Cotes grid on [-6, 6], Kn 0.5, Ma 2; 24 B-spline control-point
    offsets drawn N(0, 1e-3)."""
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.08, 0.16)
    m = rng.uniform(0.0, 0.04)
    amp = rng.normal(0.0, 1e-3, size=24)
    g = naca_cgrid(24, 72, 96, t=t, m=m, p=0.4,
                   perturb={"kind": "bspline", "n_ctrl": 14, "amp": amp})
    return Workload(f"naca_t{t:.3f}_m{m:.3f}_c192x96_v48nc_kn0.5_ma2", g,
                    VGridSpec(VG_NEWTON_COTES, 48, 48, 6.0), FlowSpec(0.5, 2.0, 1.0), seed)


def tiny_circle(ni=16, nj=8, nv=8, vmax=5.0, Kn=1.0, Ma=0.5, Tw=1.0, a=None, b=None,
                kind=VG_MIDPOINT) -> Workload:
    """Small O-grid case for finite-difference and invariant tests."""
    return circle_case(ni, nj, nv, vmax, Kn, Ma, Tw, a, b, r_outer=5.0, stretch=1.2, kind=kind)


def tiny_naca(n_wake=4, n_half=8, nj=6, nv=8, Kn=1.0, Ma=0.8, perturb=None) -> Workload:
    g = naca_cgrid(n_wake, n_half, nj, t=0.12, m=0.02, p=0.4, r_outer=4.0, h1=0.05,
                   perturb=perturb)
    return Workload("tiny_naca", g, VGridSpec(VG_MIDPOINT, nv, nv, 5.0), FlowSpec(Kn, Ma, 1.0), 0)


# --------------------------------------------------------------------------
# Request stream for the solve server
# --------------------------------------------------------------------------

SERVE_MESHES = [(64, 32), (128, 64), (256, 128)]
SERVE_VGRIDS = [16, 32, 64]


@dataclass
class Request:
    rid: int
    arrival: float           # seconds after stream start
    workload: Workload
    want_adjoint: bool
    order: int = 1           # spatial scheme of the solve: 1, or 2 (second-order reconstruction)


def serve_request(rid: int, rng: np.random.Generator, mesh_choices=None, vgrid_choices=None) -> tuple:
    """One seed-drawn solve request: circle (Fourier amplitudes N(0, 1e-2))
    or NACA (t ~ U[0.08, 0.16], m ~ U[0, 0.04]); mesh and velocity grid from
    the given menus; Kn log-uniform in [1e-3, 10]; Ma ~ U[0.3, 2]."""
    mesh_choices = SERVE_MESHES if mesh_choices is None else mesh_choices
    vgrid_choices = SERVE_VGRIDS if vgrid_choices is None else vgrid_choices
    ni, nj = mesh_choices[rng.integers(len(mesh_choices))]
    nv = int(vgrid_choices[rng.integers(len(vgrid_choices))])
    Kn = float(10.0 ** rng.uniform(-3.0, 1.0))
    Ma = float(rng.uniform(0.3, 2.0))
    want_adj = bool(rng.random() < 0.5)
    if rng.random() < 0.5:
        a = rng.normal(0.0, 1e-2, size=4)
        b = rng.normal(0.0, 1e-2, size=4)
        g = ogrid(ni, nj, 10.0, 1.1 if nj <= 32 else 1.1 ** (32.0 / nj), a, b)
        name = f"circle_o{ni}x{nj}"
    else:
        t = float(rng.uniform(0.08, 0.16))
        m = float(rng.uniform(0.0, 0.04))
        nw = ni // 8
        nh = (ni - 2 * nw) // 2
        g = naca_cgrid(nw, nh, nj, t=t, m=m, p=0.4)
        name = f"naca_c{ni}x{nj}"
    w = Workload(f"{name}_v{nv}_kn{Kn:.3g}_ma{Ma:.2f}", g, VGridSpec(VG_MIDPOINT, nv, nv, 6.0),
                 FlowSpec(Kn, Ma, 1.0), rid)
    return w, want_adj


def poisson_stream(n: int, rate: float, seed: int = 0, mesh_choices=None,
                   vgrid_choices=None) -> list:
    """``n`` requests with exponential inter-arrival times at ``rate`` /s."""
    rng = np.random.default_rng(seed)
    tnow = 0.0
    out = []
    for rid in range(n):
        tnow += float(rng.exponential(1.0 / rate)) if rate > 0 else 0.0
        w, adj = serve_request(rid, rng, mesh_choices, vgrid_choices)
        out.append(Request(rid, tnow, w, adj))
    return out


# --------------------------------------------------------------------------
# Seeded state perturbations (for parity checks from a non-trivial state)
# --------------------------------------------------------------------------

def perturbation(shape, seed: int, amp: float = 0.2) -> np.ndarray:
    """Seeded multiplicative noise 1 + amp * U(-1, 1) of the given shape
    (float64): applied to a positive distribution it stays positive for
    amp < 1."""
    rng = np.random.default_rng(seed)
    out = rng.random(shape)
    out *= 2.0 * amp
    out += 1.0 - amp
    return out


def noise_field(shape, seed: int, amp: float = 1.0) -> np.ndarray:
    """Seeded additive noise amp * U(-1, 1) of the given shape (float64)."""
    rng = np.random.default_rng(seed)
    out = rng.random(shape)
    out *= 2.0 * amp
    out -= amp
    return out
