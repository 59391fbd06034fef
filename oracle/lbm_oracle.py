"""FP64 CPU oracle of the coupled D3Q19 / D3Q7 thermal pseudopotential step.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously-correct
statement of what the GPU library computes.  It may be imported only by the
tests, by ``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of
``bench.py``; the product path (the HIP library and its Python binding) never
imports, links or executes anything under ``oracle/``.

Method: J. Huang, L. Wang, K. He, C. Huang, "An efficient thermal lattice
Boltzmann method for simulating three-dimensional liquid-vapor phase change"
(arXiv 2206.00946).  Every function cites the section / equation it restates.
All arithmetic is float64, vectorised with numpy over the whole grid; the only
library primitives used are matrix products (the moment transforms).  The
inverse transforms are computed exactly in rationals from the printed
integer matrices and rounded once per entry.

Array layout: populations are (Q, nz, ny, nx); fields are (nz, ny, nx);
vectors are (3, nz, ny, nx) with components (x, y, z).  The flat cell index
is x + nx*(y + ny*z).

Faces are ordered (-x, +x, -y, +y, -z, +z).  Kinds: PERIODIC, WALL (no-slip
wall with the geometric wetting ghost layer, only on z faces, with x and y
periodic), PRESSURE (the constant-pressure outlet of Sec. 3.3).  Every
non-periodic face is a Dirichlet temperature face (Sec. 3.1).

Readings taken where the paper is silent or garbled (all documented again in
the design notes of the repository):
  * relaxation sign in eq. (1) is "-" as in eq. (8);
  * eq. (2) uses |u|^2;
  * eq. (10) is applied literally (its rows 16-18 differ from M f^eq);
  * Sec. 4 "relaxation times" are times: s_nu = 1/1.25, s_e = 1/0.8;
  * D3Q7 wbar is a parameter (default 0.75); varsigma_{1,2,3} from lambda;
  * rho*c_v in eq. (13) is taken at the destination node, at time t;
  * grad T by the local moment relation eqs. (27)-(29) with the
    pre-collision first moments; div u by the D3Q19-weighted stencil applied
    to the real velocity of eq. (5);
  * wall nodes: the real velocity is set to 0, so u_eq = -du/2;
  * Zou-He on any face follows Sec. 3.3 mapped by lattice symmetry; nodes on
    two or more pressure faces use non-equilibrium extrapolation of all 19 f;
  * ghost psi / u beyond a pressure face: copy of the face node; beyond a
    wall: eq. (37) for psi, 0 for u;
  * edge nodes of several Dirichlet faces take T_b and rho_out from the first
    face in the priority order (-z, +z, -y, +y, -x, +x).

Every step function is written for real or complex arrays alike (the
complex-step derivative of ``oracle/gradients.py`` runs the same code on
complex inputs); comparisons only ever see the real parts of masks that
do not depend on the state.

Parity status: every function is pinned by tests under ``tests/`` (algebraic
identities, invariants, closed forms, brute force, printed special cases;
the relaxation rates, the viscosity of Sec. 4, the no-slip wall reading and
both terms of the temperature source of eq. (15) by the transport pins),
except the physics-only quantities listed in the design notes (coexistence
densities of the running model, surface tension, evaporation rate), which
are "parity unpinned" beyond loose physical checks.
"""
from __future__ import annotations

import warnings
from dataclasses import dataclass
from fractions import Fraction
from typing import Dict, Optional, Sequence

import numpy as np

PERIODIC, WALL, PRESSURE = 0, 1, 2
FACE_AXIS = (0, 0, 1, 1, 2, 2)          # x, x, y, y, z, z
FACE_SIGN = (-1, +1, -1, +1, -1, +1)     # outward normal sign
FACE_PRIORITY = (4, 5, 2, 3, 0, 1)       # -z, +z, -y, +y, -x, +x

# --------------------------------------------------------------------------
# Lattices (Sec. 2 and Appendix A)
# --------------------------------------------------------------------------

# Appendix A, eq. (A.1): the non-orthogonal D3Q19 transformation, as printed.
MHAT = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1],
    [0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1],
    [0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1],
    [0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2],
    [0, 2, 2, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2],
    [0, 0, 0, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1],
    [0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1],
    [0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1],
    [0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 0, 0, 0, 0, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1],
], dtype=np.int64)

# Appendix A, eq. (A.2): the D3Q7 transformation, as printed.
M7 = np.array([
    [1, 1, 1, 1, 1, 1, 1],
    [0, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 1, -1, 0, 0],
    [0, 0, 0, 0, 0, 1, -1],
    [0, 1, 1, 1, 1, 1, 1],
    [0, 1, 1, -1, -1, 0, 0],
    [0, 1, 1, 0, 0, -1, -1],
], dtype=np.int64)

# The velocity ordering is fixed by rows 1-3 of the transforms (rows x, y, z
# of the moment basis); Fig. 1 itself is not reproduced in the text.
C19 = MHAT[1:4].T.copy()                 # (19, 3)
C7 = M7[1:4].T.copy()                    # (7, 3)

# Sec. 2.1: D3Q19 weights 1/3, 1/18 (axes), 1/36 (diagonals); c_s^2 = 1/3.
W19 = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)
CS2 = 1.0 / 3.0

def exact_inverse(m: np.ndarray) -> np.ndarray:
    """Inverse of an integer matrix by Gauss-Jordan elimination in exact
    rationals, each entry then rounded once to the nearest double.  The
    transforms of Appendix A are integer matrices with rational inverses;
    a floating-point (LAPACK) inverse perturbs their entries by an ulp, which
    breaks exact mass conservation of the collision at the 1e-16 level."""
    n = len(m)
    a = [[Fraction(int(v)) for v in row] + [Fraction(int(i == j)) for j in range(n)]
         for i, row in enumerate(m)]
    for c in range(n):
        piv = next(r for r in range(c, n) if a[r][c] != 0)
        a[c], a[piv] = a[piv], a[c]
        pv = a[c][c]
        a[c] = [v / pv for v in a[c]]
        for r in range(n):
            if r != c and a[r][c] != 0:
                fac = a[r][c]
                a[r] = [x - fac * y for x, y in zip(a[r], a[c])]
    return np.array([[float(v) for v in row[n:]] for row in a])


MHAT_F = MHAT.astype(np.float64)
MHAT_INV = exact_inverse(MHAT)
M7_F = M7.astype(np.float64)
M7_INV = exact_inverse(M7)


def opposite(c: np.ndarray) -> np.ndarray:
    """Index of the velocity -c_i for every i (used by bounce-back, eq. (34))."""
    q = len(c)
    out = np.empty(q, dtype=np.int64)
    for i in range(q):
        out[i] = [j for j in range(q) if np.all(c[j] == -c[i])][0]
    return out


OPP19 = opposite(C19)
OPP7 = opposite(C7)


def w7(wbar: float) -> np.ndarray:
    """Sec. 2.2 after eq. (14): w_0 = 1 - wbar, w_{1..6} = wbar/6."""
    return np.array([1.0 - wbar] + [wbar / 6.0] * 6)


# --------------------------------------------------------------------------
# Parameters
# --------------------------------------------------------------------------

@dataclass
class Params:
    nx: int
    ny: int
    nz: int
    # Peng-Robinson EOS, Sec. 4 eqs. (54)-(55): a = 3/49, b = 2/21, R = 1, omega = 0.344
    a: float = 3.0 / 49.0
    b: float = 2.0 / 21.0
    R: float = 1.0
    omega: float = 0.344
    G: float = -1.0                      # eq. (6): G = -1
    # D3Q19 relaxation rates, eq. (11) with the values of Sec. 4
    s_e: float = 1.25
    s_nu: float = 0.8
    s_q: float = 1.0
    s_pi: float = 1.0
    # D3Q7: wbar (Sec. 2.2), conductivity lambda and c_v (Sec. 4.2)
    wbar: float = 0.75
    lam: float = 1.0 / 3.0
    cv: float = 5.0
    s_T_other: float = 1.0               # varsigma_0, varsigma_4..6 (Sec. 4: "taken as 1")
    faces: Sequence[int] = (PERIODIC,) * 6
    face_T: Sequence[float] = (0.0,) * 6
    face_rho: Sequence[float] = (0.0,) * 6
    kappa_w: float = 0.0                 # tan(pi/2 - theta), eq. (37)
    # Density-dependent conductivity (the Sec. 4.1 benchmark gives liquid and
    # vapour values): lambda(rho) linear in rho between (lam_rho_v, lam_vapour)
    # and (lam_rho_l, lam_liquid), constant beyond; None keeps lam uniform.
    lam_vapour: Optional[float] = None
    lam_liquid: Optional[float] = None
    lam_rho_v: float = 0.0
    lam_rho_l: float = 1.0
    # vartheta of eq. (13): 1 adds the correction S_i of eq. (16)
    theta_corr: int = 0

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def cs2_T(self) -> float:
        return self.wbar / 3.0           # Sec. 2.2: c_s^2 = wbar/3 for D3Q7

    @property
    def varsigma_flux(self) -> float:
        # after eq. (33): lambda = (1/varsigma - 1/2) c_s^2 (dt = 1)
        return 1.0 / (0.5 + self.lam / self.cs2_T)

    def lambda19(self) -> np.ndarray:
        """eq. (11): diag(1,1,1,1,s_e,s_nu x5,s_q x6,s_pi x3)."""
        return np.array([1.0, 1.0, 1.0, 1.0, self.s_e] + [self.s_nu] * 5
                        + [self.s_q] * 6 + [self.s_pi] * 3)

    def lambda7(self) -> np.ndarray:
        s = self.varsigma_flux
        o = self.s_T_other
        return np.array([o, s, s, s, o, o, o])

    def conductivity(self, rho):
        """lambda at density rho (uniform lam unless liquid/vapour values are set)."""
        if self.lam_vapour is None:
            return np.full(np.shape(rho), self.lam)
        frac = np.clip((np.real(rho) - self.lam_rho_v) / (self.lam_rho_l - self.lam_rho_v), 0.0, 1.0)
        return self.lam_vapour + (self.lam_liquid - self.lam_vapour) * frac

    def lambda7_field(self, rho) -> np.ndarray:
        """Relaxation rates of the D3Q7 collision at every node, (7,) + shape:
        varsigma_{1,2,3} = 1 / (1/2 + lambda(rho) / c_s^2), the rest s_T_other."""
        flux = 1.0 / (0.5 + self.conductivity(rho) / self.cs2_T)
        out = np.empty((7,) + np.shape(rho))
        out[:] = self.s_T_other
        out[1:4] = flux
        return out


# --------------------------------------------------------------------------
# Peng-Robinson equation of state (Sec. 4, eqs. (54)-(55)) and psi (eq. (7))
# --------------------------------------------------------------------------

def critical_temperature(p: Params) -> float:
    """eq. (55): a/b = 0.45724 R Tc / 0.0778, hence Tc = 0.0778 a / (0.45724 b R)."""
    return 0.0778 * p.a / (0.45724 * p.b * p.R)


def pr_kappa(p: Params) -> float:
    """The factor multiplying (1 - sqrt(T/Tc)) inside xi(T), Sec. 4."""
    w = p.omega
    return 0.37464 + 1.54226 * w - 0.26992 * w * w


def pr_xi(T, p: Params):
    """xi(T) = [1 + kappa (1 - sqrt(T/Tc))]^2 (Sec. 4)."""
    Tc = critical_temperature(p)
    return (1.0 + pr_kappa(p) * (1.0 - np.sqrt(T / Tc))) ** 2


def pr_dxi_dT(T, p: Params):
    """d xi / dT = -kappa [1 + kappa (1 - sqrt(T/Tc))] / sqrt(T Tc)."""
    Tc = critical_temperature(p)
    k = pr_kappa(p)
    return -k * (1.0 + k * (1.0 - np.sqrt(T / Tc))) / np.sqrt(T * Tc)


def pr_pressure(rho, T, p: Params):
    """eq. (54): p = rho R T/(1 - b rho) - a xi(T) rho^2/(1 + 2 b rho - b^2 rho^2)."""
    b = p.b
    return (rho * p.R * T / (1.0 - b * rho)
            - p.a * pr_xi(T, p) * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho))


def pr_dp_dT(rho, T, p: Params):
    """(dp/dT) at constant rho, the factor of the phase-change term of eq. (12)/(15)."""
    b = p.b
    return (rho * p.R / (1.0 - b * rho)
            - p.a * pr_dxi_dT(T, p) * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho))


def psi_radicand(rho, T, p: Params):
    """The argument of the square root of eq. (7): 2 (p_EOS - rho c_s^2)/G."""
    return 2.0 * (pr_pressure(rho, T, p) - rho * CS2) / p.G


def pseudopotential(rho, T, p: Params):
    """eq. (7) with dx = dt = 1: psi = sqrt(2 (p_EOS - rho c_s^2) / G)."""
    return np.sqrt(psi_radicand(rho, T, p))


def maxwell_coexistence(T: float, p: Params, tol: float = 1e-14):
    """Equal-area (Maxwell) construction at temperature T < Tc (Sec. 4.2).

    Returns (rho_v, rho_l, p_sat): the two densities with equal pressure
    p_sat such that the integral of (p(rho) - p_sat)/rho^2 from rho_v to
    rho_l vanishes.  Plain bracketing on the subcritical isotherm.
    """
    from scipy.optimize import brentq
    from scipy.integrate import quad

    rmax = 1.0 / p.b
    # spinodals: zeros of dp/drho on a fine grid, refined by bisection
    grid = np.linspace(1e-6, rmax * 0.999, 200001)
    h = 1e-7

    def dpdr(r):
        return (pr_pressure(r + h, T, p) - pr_pressure(r - h, T, p)) / (2 * h)

    d = dpdr(grid)
    idx = np.nonzero(np.sign(d[:-1]) != np.sign(d[1:]))[0]
    if len(idx) < 2:
        raise ValueError("temperature is not subcritical")
    r1 = brentq(dpdr, grid[idx[0]], grid[idx[0] + 1], xtol=1e-15)
    r2 = brentq(dpdr, grid[idx[1]], grid[idx[1] + 1], xtol=1e-15)
    p_lo = max(pr_pressure(r2, T, p), 1e-14)
    p_hi = pr_pressure(r1, T, p)

    def branches(ps):
        lo = 0.25 * ps / (p.R * T)          # p(r) < r R T / (1 - b r) on the vapour branch
        rv = brentq(lambda r: pr_pressure(r, T, p) - ps, lo, r1, xtol=1e-16)
        rl = brentq(lambda r: pr_pressure(r, T, p) - ps, r2, rmax * (1 - 1e-12), xtol=1e-16)
        return rv, rl

    def area(ps):
        rv, rl = branches(ps)
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            val, _ = quad(lambda r: (pr_pressure(r, T, p) - ps) / (r * r), rv, rl,
                          epsabs=1e-15, epsrel=1e-13, limit=200)
        return val

    ps = brentq(area, p_lo * (1 + 1e-12), p_hi * (1 - 1e-12), xtol=tol, rtol=1e-15)
    rv, rl = branches(ps)
    return rv, rl, ps


# --------------------------------------------------------------------------
# Equilibria (eqs. (2), (10), (14), (25))
# --------------------------------------------------------------------------

def feq19(rho, u):
    """eq. (2) with |u|^2: w_i rho [1 + 3 c.u + 4.5 (c.u)^2 - 1.5 |u|^2]."""
    cu = np.tensordot(C19.astype(np.float64), u, axes=(1, 0))
    usq = np.sum(u * u, axis=0)
    wshape = (19,) + (1,) * (cu.ndim - 1)
    return W19.reshape(wshape) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq)


def meq19(rho, u):
    """eq. (10) applied literally, with c_s^2 = 1/3 and c_s^4 = 1/9."""
    ux, uy, uz = u[0], u[1], u[2]
    usq = ux * ux + uy * uy + uz * uz
    c2, c4 = CS2, CS2 * CS2
    rest = rho * c4 * (1.0 - 1.5 * usq)
    return np.stack([
        rho, rho * ux, rho * uy, rho * uz,
        rho + rho * usq,
        rho * (2.0 * ux * ux - uy * uy - uz * uz),
        rho * (uy * uy - uz * uz),
        rho * ux * uy, rho * ux * uz, rho * uy * uz,
        rho * c2 * uy, rho * c2 * ux, rho * c2 * uz,
        rho * c2 * ux, rho * c2 * uz, rho * c2 * uy,
        rest + rho * c2 * (ux * ux + uy * uy),
        rest + rho * c2 * (ux * ux + uz * uz),
        rest + rho * c2 * (uy * uy + uz * uz),
    ])


def geq7(T, p: Params):
    """eq. (14): g_i^eq = w_i T."""
    w = w7(p.wbar)
    return w.reshape((7,) + (1,) * np.ndim(T)) * T


# --------------------------------------------------------------------------
# Geometry helpers: face membership, ghost layers, neighbour sampling
# --------------------------------------------------------------------------

def face_masks(p: Params):
    """Boolean mask of the nodes lying on each non-periodic face (None if periodic)."""
    masks = []
    z, y, x = np.meshgrid(np.arange(p.nz), np.arange(p.ny), np.arange(p.nx), indexing="ij")
    coord = (x, y, z)
    n = (p.nx, p.ny, p.nz)
    for k in range(6):
        if p.faces[k] == PERIODIC:
            masks.append(None)
            continue
        a = FACE_AXIS[k]
        masks.append(coord[a] == (0 if FACE_SIGN[k] < 0 else n[a] - 1))
    return masks


def check_params(p: Params):
    for a in range(3):
        lo, hi = p.faces[2 * a], p.faces[2 * a + 1]
        if (lo == PERIODIC) != (hi == PERIODIC):
            raise ValueError("periodic faces must come in pairs")
    if WALL in (p.faces[0], p.faces[1], p.faces[2], p.faces[3]):
        raise ValueError("walls are supported on the z faces only")
    if WALL in (p.faces[4], p.faces[5]) and any(f != PERIODIC for f in p.faces[:4]):
        raise ValueError("a z wall requires periodic x and y")
    for a, n in enumerate((p.nx, p.ny, p.nz)):
        if p.faces[2 * a] != PERIODIC and n < 3:
            raise ValueError("a bounded axis needs at least 3 nodes")


def _wetting_ghost(psi, kappa, plane_wall, plane_inner):
    """eq. (37): psi at the ghost layer beyond a wall.

    plane_wall: psi on the wall layer (ny, nx); plane_inner: psi one layer
    inside.  Tangential differences are periodic (x, y periodic with walls).
    """
    dx = np.roll(plane_wall, -1, axis=1) - np.roll(plane_wall, 1, axis=1)
    dy = np.roll(plane_wall, -1, axis=0) - np.roll(plane_wall, 1, axis=0)
    return plane_inner + np.sqrt(dx * dx + dy * dy) * kappa


def pad_field(phi, p: Params, wall_ghost):
    """Pad a scalar field (nz, ny, nx) by one ghost layer on every side.

    Periodic faces wrap, pressure faces copy the face node, and wall faces
    (z only) use wall_ghost(plane_wall, plane_inner) -> ghost plane.
    The z axis is padded first (ghost planes computed on the unpadded x, y
    extent), then y, then x, so ghost corners follow the same rules.
    """
    out = phi
    # z
    lo_k, hi_k = p.faces[4], p.faces[5]
    if lo_k == PERIODIC:
        lo = out[-1]
    elif lo_k == PRESSURE:
        lo = out[0]
    else:
        lo = wall_ghost(out[0], out[1])
    if hi_k == PERIODIC:
        hi = out[0]
    elif hi_k == PRESSURE:
        hi = out[-1]
    else:
        hi = wall_ghost(out[-1], out[-2])
    out = np.concatenate([lo[None], out, hi[None]], axis=0)
    # y then x
    for axis, (lk, hk) in ((1, (p.faces[2], p.faces[3])), (2, (p.faces[0], p.faces[1]))):
        n = out.shape[axis]
        first = np.take(out, [0], axis=axis)
        last = np.take(out, [n - 1], axis=axis)
        lo = last if lk == PERIODIC else first
        hi = first if hk == PERIODIC else last
        out = np.concatenate([lo, out, hi], axis=axis)
    return out


def pad_psi(psi, p: Params):
    return pad_field(psi, p, lambda w, i: _wetting_ghost(psi, p.kappa_w, w, i))


def pad_velocity_component(uc, p: Params):
    """Ghost velocity: 0 beyond walls, copy beyond pressure faces, wrap if periodic."""
    return pad_field(uc, p, lambda w, i: np.zeros_like(w))


def neighbour(padded, c, shape):
    """Sample a one-cell-padded field at x + c for every interior x."""
    nz, ny, nx = shape
    cx, cy, cz = int(c[0]), int(c[1]), int(c[2])
    return padded[1 + cz:1 + cz + nz, 1 + cy:1 + cy + ny, 1 + cx:1 + cx + nx]


# --------------------------------------------------------------------------
# Stencils: interaction force (eq. (6)) and isotropic divergence (Sec. 2.2)
# --------------------------------------------------------------------------

def interaction_force(psi, p: Params):
    """eq. (6): F = -G psi(x) sum_{i=1..18} varpi(|c_i|^2) psi(x + c_i) c_i,
    varpi(1) = 1/6, varpi(2) = 1/12.  F_ext = 0 (gravity neglected, Sec. 4.3)."""
    P = pad_psi(psi, p)
    acc = np.zeros((3,) + psi.shape, dtype=np.result_type(P, np.float64))
    for i in range(1, 19):
        c = C19[i]
        varpi = 1.0 / 6.0 if int(np.dot(c, c)) == 1 else 1.0 / 12.0
        nb = neighbour(P, c, psi.shape)
        for a in range(3):
            if c[a] != 0:
                acc[a] += varpi * c[a] * nb
    return -p.G * psi * acc


def divergence(u, p: Params):
    """Isotropic central divergence on the D3Q19 stencil (Sec. 2.2, end):
    div u = (1/c_s^2) sum_i w_i c_i . u(x + c_i)."""
    pads = [pad_velocity_component(u[a], p) for a in range(3)]
    div = np.zeros(u.shape[1:], dtype=np.result_type(u, np.float64))
    for i in range(1, 19):
        c = C19[i]
        for a in range(3):
            if c[a] != 0:
                div += (W19[i] / CS2) * c[a] * neighbour(pads[a], c, u.shape[1:])
    return div


# --------------------------------------------------------------------------
# Boundary conditions (Sec. 3)
# --------------------------------------------------------------------------

def _boundary_nodes(p: Params):
    """Per node: number of non-periodic faces it lies on, the inward offset
    (sum of inward normals of those faces) and the priority face index."""
    masks = face_masks(p)
    count = np.zeros(p.shape, dtype=np.int64)
    inward = np.zeros((3,) + p.shape, dtype=np.int64)
    prio = np.full(p.shape, -1, dtype=np.int64)
    for k in range(6):
        if masks[k] is None:
            continue
        count += masks[k]
        inward[FACE_AXIS[k]] -= FACE_SIGN[k] * masks[k]
    for k in reversed(FACE_PRIORITY):
        if masks[k] is not None:
            prio[masks[k]] = k
    return masks, count, inward, prio


def thermal_dirichlet(g, p: Params, Tw: Optional[Dict[int, np.ndarray]] = None):
    """Sec. 3.1, eqs. (35)-(36): non-equilibrium extrapolation at every node of
    a non-periodic face: g_i(x_b) = w_i T_b + g_i(x_f) - w_i T(x_f) for all i,
    with x_f the inward (diagonal at edges) neighbour.  Returns a new array."""
    _, count, inward, prio = _boundary_nodes(p)
    g = g.copy()
    bz, by, bx = np.nonzero(count > 0)
    if len(bz) == 0:
        return g
    w = w7(p.wbar)
    fx = bx + inward[0, bz, by, bx]
    fy = by + inward[1, bz, by, bx]
    fzz = bz + inward[2, bz, by, bx]
    gf = g[:, fzz, fy, fx]
    Tf = gf.sum(axis=0)
    k = prio[bz, by, bx]
    Tb = np.array(p.face_T, dtype=np.float64)[k]
    if Tw:
        Tb = Tb.astype(np.result_type(Tb, *[np.asarray(v) for v in Tw.values()]))
        for face, field2d in Tw.items():
            sel = k == face
            Tb[sel] = field2d[by[sel], bx[sel]]
    g = g.astype(np.result_type(g, Tb), copy=False)
    g[:, bz, by, bx] = w[:, None] * Tb[None, :] + gf - w[:, None] * Tf[None, :]
    return g


def pressure_nodes(p: Params):
    """(face_node_mask_per_face, edge_mask, rho_out field or None)."""
    masks, count, inward, prio = _boundary_nodes(p)
    face_only = []
    for k in range(6):
        if masks[k] is None or p.faces[k] != PRESSURE:
            face_only.append(None)
        else:
            face_only.append(masks[k] & (count == 1))
    edge = np.zeros(p.shape, dtype=bool)
    any_p = np.zeros(p.shape, dtype=bool)
    for k in range(6):
        if masks[k] is not None and p.faces[k] == PRESSURE:
            any_p |= masks[k]
    edge = any_p & (count >= 2)
    rho_out = np.zeros(p.shape)
    rho_out[any_p] = np.array(p.face_rho, dtype=np.float64)[prio[any_p]]
    return face_only, edge, any_p, rho_out, inward


def zou_he_face(f, F, rho_out, k):
    """Sec. 3.3, eqs. (38)-(53), for the face k at nodes given as columns.

    f: (19, m) populations of the face nodes (unknowns are overwritten),
    F: (3, m) total force, rho_out: (m,).  The +z derivation of the paper is
    applied to face k through the symmetry that maps its outward normal n to
    +z: u_n from mass and normal momentum (eq. (41)), the normal unknown by
    normal non-equilibrium bounce-back (eq. (42)), the four diagonal unknowns
    by eqs. (43)-(49) with delta_t from the tangential momenta and
    delta_n = -F.n/8."""
    a = FACE_AXIS[k]
    n = np.zeros(3, dtype=np.int64)
    n[a] = FACE_SIGN[k]
    tangents = [t for t in range(3) if t != a]
    cn = C19 @ n
    sig0 = f[cn == 0].sum(axis=0)
    sig1 = f[cn == 1].sum(axis=0)
    Fn = F[a] * FACE_SIGN[k]
    un = (sig0 + 2.0 * sig1 + 0.5 * Fn) / rho_out - 1.0
    delta_t = {}
    for t in tangents:
        delta_t[t] = -0.5 * (f[cn == 0] * C19[cn == 0, t][:, None]).sum(axis=0) - 0.25 * F[t]
    delta_n = -Fn / 8.0
    out = f.astype(np.result_type(f, F))
    for i in np.nonzero(cn == -1)[0]:
        j = OPP19[i]
        if np.all(C19[i] == -n):
            out[i] = f[j] - rho_out * un / 3.0
        else:
            v = f[j] - rho_out * un / 6.0 + C19[i] @ n * delta_n
            for t in tangents:
                v = v + C19[i, t] * delta_t[t]
            out[i] = v
    return out


def zou_he(f, F, p: Params):
    """Fill the unknown populations at pressure-face nodes (Sec. 3.3).  Nodes on
    two or more pressure faces (edges, corners) take every population by
    non-equilibrium extrapolation from the inward diagonal neighbour x_f:
    f_i = f_i^eq(rho_out, u_eq(x_f)) + f_i(x_f) - f_i^eq(rho(x_f), u_eq(x_f))."""
    face_only, edge, any_p, rho_out, inward = pressure_nodes(p)
    if not any_p.any():
        return f
    f = f.astype(np.result_type(f, F))
    for k in range(6):
        m = face_only[k]
        if m is None or not m.any():
            continue
        z, y, x = np.nonzero(m)
        f[:, z, y, x] = zou_he_face(f[:, z, y, x], F[:, z, y, x], rho_out[z, y, x], k)
    if edge.any():
        z, y, x = np.nonzero(edge)
        fz = z + inward[2, z, y, x]
        fy = y + inward[1, z, y, x]
        fx = x + inward[0, z, y, x]
        ff = f[:, fz, fy, fx]
        rf = ff.sum(axis=0)
        ueq = (C19.T.astype(np.float64) @ ff) / rf
        f[:, z, y, x] = feq19(rho_out[z, y, x], ueq) + ff - feq19(rf, ueq)
    return f


def wall_node_mask(p: Params):
    m = np.zeros(p.shape, dtype=bool)
    masks = face_masks(p)
    for k in (4, 5):
        if p.faces[k] == WALL:
            m |= masks[k]
    return m


# --------------------------------------------------------------------------
# One time step (Sec. 2 + Sec. 3), in the order S0 .. S10
# --------------------------------------------------------------------------

def init_populations(rho0, T0, p: Params):
    """f = f^eq(rho0, u = 0) (eq. (2)), g = w_i T0 (eq. (14))."""
    zero = np.zeros((3,) + rho0.shape)
    return feq19(rho0, zero), geq7(T0, p)


def macroscopic(f, g, p: Params, Tw=None):
    """Complete the boundary nodes of the state at t and evaluate every
    macroscopic quantity the update needs (S0-S6).  Returns a dict."""
    check_params(p)
    g = thermal_dirichlet(g, p, Tw)                             # S0, eqs. (35)-(36)
    _, _, any_p, rho_out, _ = pressure_nodes(p)
    rho = f.sum(axis=0)                                         # S1, eq. (3)
    rho = np.where(any_p, rho_out, rho)
    T = g.sum(axis=0)                                           # T = sum g (eq. (25), m_0 = T)
    rad = psi_radicand(rho, T, p)                               # S2, eq. (7)
    bad = (~np.isfinite(rho)) | (~np.isfinite(T)) | (rho <= 0) | (rho * p.b >= 1.0) \
        | (T <= 0) | (~np.isfinite(rad)) | (rad < 0)
    with np.errstate(invalid="ignore"):
        psi = np.sqrt(rad)
    F = interaction_force(psi, p)                               # S3, eq. (6)
    f = zou_he(f, F, p)                                         # S4, Sec. 3.3
    j = np.tensordot(C19.T.astype(np.float64), f, axes=(1, 0))  # eq. (3)
    ueq = j / rho
    du = F / rho                                                # eq. (4): du = F dt / rho
    u = ueq + 0.5 * du                                          # eq. (5)
    wall = wall_node_mask(p)
    if wall.any():                                              # Sec. 3.1: u specified = 0
        u = np.where(wall, 0.0, u)
        ueq = np.where(wall, -0.5 * du, ueq)
    div_u = divergence(u, p)                                    # S6, isotropic stencil
    mg = np.tensordot(C7.T.astype(np.float64), g, axes=(1, 0))  # first moments of g
    lam7 = p.lambda7_field(rho)
    gradT = -(lam7[1:4] * mg) / p.cs2_T                         # eqs. (27)-(29)
    dpdT = pr_dp_dT(rho, T, p)
    Fbar = rho * p.cv * np.sum(u * gradT, axis=0) + T * dpdT * div_u   # eq. (15)
    return dict(f=f, g=g, rho=rho, T=T, psi=psi, F=F, j=j, ueq=ueq, du=du, u=u,
                div_u=div_u, gradT=gradT, dpdT=dpdT, Fbar=Fbar, bad=bad)


def collide19(f, rho, ueq, du, p: Params):
    """eq. (8): m* = m - L(m - m_eq(u_eq)) + [m_eq(u_eq + du) - m_eq(u_eq)],
    f* = M^-1 m*, with m = M f and m_eq from eq. (10)."""
    shp = f.shape
    m = MHAT_F @ f.reshape(19, -1)
    me0 = meq19(rho, ueq).reshape(19, -1)
    me1 = meq19(rho, ueq + du).reshape(19, -1)
    lam = p.lambda19()[:, None]
    mstar = m - lam * (m - me0) + (me1 - me0)
    return (MHAT_INV @ mstar).reshape(shp)


def collide7(g, T, Fbar, p: Params, rho):
    """eq. (13) collision part with theta = 0: g* = g - M^-1 L M (g - g_eq) + dt Fbar_i,
    Fbar_i = -w_i Fbar (eq. (15)); the D3Q7 equilibrium moments are
    (T, 0, 0, 0, wbar T, 0, 0) (eq. (25)); L from the conductivity at rho."""
    shp = g.shape
    n = M7_F @ g.reshape(7, -1)
    Tf = T.reshape(-1)
    neq = np.zeros_like(n)
    neq[0] = Tf
    neq[4] = p.wbar * Tf
    nstar = n - p.lambda7_field(rho).reshape(7, -1) * (n - neq)
    gstar = M7_INV @ nstar - w7(p.wbar)[:, None] * Fbar.reshape(-1)[None, :]
    return gstar.reshape(shp)


def _source_index(p: Params, c):
    """For every destination y: the source y - c and whether it lies in the domain."""
    z, y, x = np.meshgrid(np.arange(p.nz), np.arange(p.ny), np.arange(p.nx), indexing="ij")
    src = []
    valid = np.ones(p.shape, dtype=bool)
    for a, (coord, n) in enumerate(((x, p.nx), (y, p.ny), (z, p.nz))):
        s = coord - int(c[a])
        if p.faces[2 * a] == PERIODIC:
            s = np.mod(s, n)
        else:
            valid &= (s >= 0) & (s < n)
            s = np.clip(s, 0, n - 1)
        src.append(s)
    return src[2], src[1], src[0], valid


def stream19(fstar, p: Params):
    """eq. (9) push streaming; links that leave the domain through a wall are
    bounced back onto the opposite velocity at the same node (eq. (34)); links
    leaving through a pressure face are discarded.  Slots without a source
    (unknowns at pressure faces) are NaN until the next Zou-He fill."""
    out = np.full_like(fstar, np.nan)
    for i in range(19):
        sz, sy, sx, valid = _source_index(p, C19[i])
        v = fstar[i][sz, sy, sx]
        out[i][valid] = v[valid]
    # bounce-back at wall nodes: the unknown slot i at x_b comes from the
    # link opp(i) that would have left through the wall (eq. (34))
    for k in (4, 5):
        if p.faces[k] != WALL:
            continue
        zb = 0 if k == 4 else p.nz - 1
        for i in range(19):
            if C19[i, 2] * FACE_SIGN[k] == -1:         # slot fed from outside
                out[i, zb] = fstar[OPP19[i], zb]
    return out


def stream7_blend(gstar, g, rho, p: Params):
    """eq. (13) streaming with the rho c_v blend (destination y = x + c_i):
    g_i(y, t+1) = g_i(y, t) + [g*_i(y - c_i) - g_i(y, t)] / (rho(y, t) c_v).
    Slots whose source lies outside the domain keep g_i(y, t)."""
    out = g.copy()
    inv = 1.0 / (rho * p.cv)
    for i in range(7):
        sz, sy, sx, valid = _source_index(p, C7[i])
        src = gstar[i][sz, sy, sx]
        blended = g[i] + (src - g[i]) * inv
        out[i] = np.where(valid, blended, g[i])
    return out


def correction_source(mac, p: Params, T_hist):
    """eq. (16) with vartheta = 1: S_i = w_i rho c_v (dt/2) d^2T/dt^2 enters
    the collision like the source of eq. (15), so it is applied as Fbar ->
    Fbar - (1/2) rho c_v d^2T/dt^2.  d^2T/dt^2 is the backward difference
    T(t) - 2 T(t-1) + T(t-2) of the S1 temperatures (the paper asks for a
    finite difference without fixing it); zero until two past values exist."""
    if not p.theta_corr or T_hist is None or len(T_hist) < 2:
        return mac["Fbar"]
    d2T = mac["T"] - 2.0 * T_hist[0] + T_hist[1]
    return mac["Fbar"] - 0.5 * mac["rho"] * p.cv * d2T


def step(f, g, p: Params, Tw=None, T_hist=None):
    """One full time step S0..S10.  T_hist: the S1 temperatures of the two
    previous steps, most recent first (used with vartheta = 1 only).
    Returns (f_next, g_next, macroscopic dict at t)."""
    mac = macroscopic(f, g, p, Tw)
    Fbar = correction_source(mac, p, T_hist)
    fstar = collide19(mac["f"], mac["rho"], mac["ueq"], mac["du"], p)   # S7
    gstar = collide7(mac["g"], mac["T"], Fbar, p, mac["rho"])           # S8
    f_next = stream19(fstar, p)                                         # S9
    g_next = stream7_blend(gstar, mac["g"], mac["rho"], p)              # S10
    return f_next, g_next, mac


def run(f, g, p: Params, nsteps: int, Tw=None, T_hist=None):
    """nsteps steps; T_hist (a list, most recent first) carries the
    temperature history between calls when vartheta = 1."""
    hist = T_hist if T_hist is not None else []
    for _ in range(nsteps):
        f, g, mac = step(f, g, p, Tw, hist)
        if mac["bad"].any():
            raise FloatingPointError("non-physical state")
        hist[:] = [mac["T"]] + hist[:1]
    return f, g


def fields(f, g, p: Params, Tw=None):
    """rho, real velocity u (eq. (5)) and T of the current state, with the
    boundary nodes completed (S0-S5)."""
    mac = macroscopic(f, g, p, Tw)
    return mac["rho"], mac["u"], mac["T"]


def diagnostics(rho, T, p: Params, rho_v: float, rho_l: float):
    """Mass sum(rho), energy sum(rho c_v T), liquid volume (hard threshold at
    the mid density and smooth clipped fraction), all in float64."""
    mass = float(np.sum(rho))
    energy = float(np.sum(rho * p.cv * T))
    mid = 0.5 * (rho_l + rho_v)
    vol_hard = float(np.count_nonzero(rho > mid))
    vol_smooth = float(np.sum(np.clip((rho - rho_v) / (rho_l - rho_v), 0.0, 1.0)))
    return dict(mass=mass, energy=energy, vol_hard=vol_hard, vol_smooth=vol_smooth)
