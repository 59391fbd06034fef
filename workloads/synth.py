"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no arithmetic of the lattice Boltzmann method: it draws
random numbers (SplitMix64), lays out geometry (droplets, hemispheres, blobs
with the tanh profile of the initial condition, eq. (57)) and looks up
coexistence densities in a stored table.  The table
(``coexistence_pr.json``) is written by ``make_coexistence_table.py``, which
calls only the oracle's Maxwell construction.

Every workload returns a plain dict:
  name, nx, ny, nz, faces (-x,+x,-y,+y,-z,+z; 0 periodic, 1 wall, 2 pressure),
  face_T, face_rho, kappa_w, rho0 / T0 (float64, shape (nz, ny, nx)),
  Tw ({face: (ny, nx) float64} or {}), steps, rho_v, rho_l (diagnostic
  references), rho_ref / T_ref (deviation-storage references), Tc.
"""
from __future__ import annotations

import json
import os
from typing import Dict

import numpy as np

PERIODIC, WALL, PRESSURE = 0, 1, 2
_HERE = os.path.dirname(os.path.abspath(__file__))
_TABLE = None

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int) -> np.ndarray:
    """n successive outputs of SplitMix64 (Steele, Lea & Flood, OOPSLA 2014)."""
    with np.errstate(over="ignore"):
        k = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_pm1(seed: int, n: int) -> np.ndarray:
    """Uniform doubles in [-1, 1)."""
    return 2.0 * uniform01(seed, n) - 1.0


def coexistence_table() -> dict:
    global _TABLE
    if _TABLE is None:
        with open(os.path.join(_HERE, "coexistence_pr.json")) as fh:
            _TABLE = json.load(fh)
    return _TABLE


def critical_temperature() -> float:
    return coexistence_table()["Tc"]


def coexistence(T_over_Tc):
    """(rho_v, rho_l) at T/Tc by linear interpolation of the stored table."""
    tab = coexistence_table()
    t = np.array([e[0] for e in tab["rows"]])
    rv = np.array([e[1] for e in tab["rows"]])
    rl = np.array([e[2] for e in tab["rows"]])
    x = np.asarray(T_over_Tc, dtype=np.float64)
    if np.any(x < t[0]) or np.any(x > t[-1]):
        raise ValueError("temperature outside the stored coexistence table")
    return np.interp(x, t, rv), np.interp(x, t, rl)


def _grid(nx, ny, nz):
    return np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                       np.arange(nx, dtype=np.float64), indexing="ij")


def tanh_profile(dist, R0, W, inside, outside):
    """eq. (57): (in+out)/2 - (in-out)/2 tanh(2 (|x - x0| - R0)/W)."""
    return 0.5 * (inside + outside) - 0.5 * (inside - outside) * np.tanh(2.0 * (dist - R0) / W)


def _base(name, nx, ny, nz, faces, steps, Tsat_over_Tc):
    Tc = critical_temperature()
    rv, rl = coexistence(Tsat_over_Tc)
    return dict(name=name, nx=nx, ny=ny, nz=nz, faces=list(faces),
                face_T=[0.0] * 6, face_rho=[0.0] * 6, kappa_w=0.0, Tw={},
                steps=steps, rho_v=float(rv), rho_l=float(rl),
                rho_ref=float(rv), T_ref=Tsat_over_Tc * Tc, Tc=Tc)


def droplet_periodic(n=32, R0=8.0, W=5.0, Tsat=0.86, noise=1e-6, seed=1, steps=500,
                     center=None, nx=None, ny=None, nz=None):
    """Periodic box with a centred droplet at uniform T = Tsat*Tc, zero
    velocity and additive uniform density noise of amplitude `noise`."""
    nx = nx or n
    ny = ny or n
    nz = nz or n
    w = _base("droplet_periodic", nx, ny, nz, [PERIODIC] * 6, steps, Tsat)
    z, y, x = _grid(nx, ny, nz)
    cx, cy, cz = center if center is not None else (nx / 2, ny / 2, nz / 2)
    d = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2)
    rho = tanh_profile(d, R0, W, w["rho_l"], w["rho_v"])
    if noise:
        rho = rho + noise * uniform_pm1(seed, rho.size).reshape(rho.shape)
    w["rho0"] = rho
    w["T0"] = np.full(rho.shape, Tsat * w["Tc"])
    return w


def droplet_open(n=128, R0=25.0, W=5.0, Tsat=0.86, Tg_factor=1.1, steps=20000,
                 nx=None, ny=None, nz=None):
    """Droplet evaporation in an open box (Sec. 4.2 set-up): constant-pressure
    faces on all six sides at rho_v(Tsat), faces held at Tg = Tg_factor*Tsat;
    the droplet starts at Tsat, the vapour at Tg with the same tanh profile."""
    nx = nx or n
    ny = ny or n
    nz = nz or n
    w = _base("droplet_open", nx, ny, nz, [PRESSURE] * 6, steps, Tsat)
    Tc = w["Tc"]
    Tg = Tg_factor * Tsat * Tc
    w["face_T"] = [Tg] * 6
    w["face_rho"] = [w["rho_v"]] * 6
    z, y, x = _grid(nx, ny, nz)
    d = np.sqrt((x - nx / 2) ** 2 + (y - ny / 2) ** 2 + (z - nz / 2) ** 2)
    w["rho0"] = tanh_profile(d, R0, W, w["rho_l"], w["rho_v"])
    w["T0"] = tanh_profile(d, R0, W, Tsat * Tc, Tg)
    return w


def heated_wall(n=256, R0=40.0, W=5.0, Tsat=0.86, Tw_factor=1.15, steps=10000,
                Tw_jitter=0.0, seed=5, kappa_w=0.0, nx=None, ny=None, nz=None):
    """Hemispherical droplet on a heated no-slip wall at z = 0 (Sec. 4.3
    set-up): periodic x, y; constant-pressure top face at rho_v(Tsat) held
    at Tsat; wall temperature Tw_factor*Tsat, optionally jittered per wall
    cell by a relative uniform +-Tw_jitter (seeded)."""
    nx = nx or n
    ny = ny or n
    nz = nz or n
    faces = [PERIODIC, PERIODIC, PERIODIC, PERIODIC, WALL, PRESSURE]
    w = _base("heated_wall", nx, ny, nz, faces, steps, Tsat)
    Tc = w["Tc"]
    Tw = Tw_factor * Tsat * Tc
    w["face_T"] = [0.0, 0.0, 0.0, 0.0, Tw, Tsat * Tc]
    w["face_rho"] = [0.0, 0.0, 0.0, 0.0, 0.0, w["rho_v"]]
    w["kappa_w"] = kappa_w
    z, y, x = _grid(nx, ny, nz)
    d = np.sqrt((x - nx / 2) ** 2 + (y - ny / 2) ** 2 + z ** 2)
    w["rho0"] = tanh_profile(d, R0, W, w["rho_l"], w["rho_v"])
    w["T0"] = np.full(w["rho0"].shape, Tsat * Tc)
    field = np.full((ny, nx), Tw)
    if Tw_jitter:
        field = field * (1.0 + Tw_jitter * uniform_pm1(seed, nx * ny).reshape(ny, nx))
    w["Tw"] = {4: field}
    return w


def slab(nx=128, ny=8, nz=8, width=64.0, W=5.0, Tsat=0.86, steps=20000):
    """Flat liquid slab across x in a periodic box at uniform T = Tsat*Tc:
    liquid for |x - nx/2| < width/2, tanh interfaces of width W."""
    w = _base("slab", nx, ny, nz, [PERIODIC] * 6, steps, Tsat)
    z, y, x = _grid(nx, ny, nz)
    d = np.abs(x - nx / 2) + 0.0 * (y + z)
    w["rho0"] = tanh_profile(d, width / 2, W, w["rho_l"], w["rho_v"])
    w["T0"] = np.full(w["rho0"].shape, Tsat * w["Tc"])
    return w


def saturated_heat_transfer(nx=10, ny=10, nz=200, W=5.0, Tsat=0.86, Th=1.0, lam_v=0.2, lam_l=0.4, cv=5.0,
                            steps=200000):
    """Heat transfer through a flat liquid-vapour interface (Sec. 4.1 set-up,
    turned so that the walls are the z faces): vapour for z < nz/2, liquid
    above, both at Tsat*Tc; the z = 0 wall is held at Th*Tc, the z = nz-1
    wall at Tsat*Tc; conductivities lam_v (vapour) and lam_l (liquid)."""
    w = _base("saturated_heat_transfer", nx, ny, nz, [PERIODIC] * 4 + [WALL] * 2, steps, Tsat)
    Tc = w["Tc"]
    w["face_T"] = [0.0] * 4 + [Th * Tc, Tsat * Tc]
    z, y, x = _grid(nx, ny, nz)
    s = z - (nz / 2 - 0.5) + 0.0 * (x + y)       # > 0 in the liquid half
    w["rho0"] = tanh_profile(s, 0.0, W, w["rho_v"], w["rho_l"])
    w["T0"] = np.full(w["rho0"].shape, Tsat * Tc)
    w.update(lambda_vapour=lam_v, lambda_liquid=lam_l, lambda_rho_v=w["rho_v"], lambda_rho_l=w["rho_l"], cv=cv)
    return w


def heated_surface(nx=160, ny=160, nz=100, diameter=70.0, W=5.0, Tsat=0.86, Tw=0.8931, theta_deg=120.0,
                   steps=20000):
    """Droplet on a heated surface (Sec. 4.3 set-up): a hemisphere of the given
    diameter centred on the z = 0 wall, droplet and vapour at Tsat*Tc, wall
    at Tw*Tc, outlet on top held at Tsat*Tc, periodic sides, wetting ghost
    layer with kappa_w = tan(pi/2 - theta)."""
    w = heated_wall(nx=nx, ny=ny, nz=nz, R0=diameter / 2.0, W=W, Tsat=Tsat, Tw_factor=Tw / Tsat, steps=steps,
                    kappa_w=float(np.tan(np.pi / 2.0 - np.radians(theta_deg))))
    w["name"] = "heated_surface"
    w["T0"] = np.full(w["rho0"].shape, Tsat * w["Tc"])
    return w


def _poisson(lam: float, u: float) -> int:
    """Inverse-CDF Poisson draw from one uniform number."""
    k = 0
    pk = np.exp(-lam)
    cdf = pk
    while u > cdf and k < 10 * lam + 100:
        k += 1
        pk *= lam / k
        cdf += pk
    return k


def blobs_closed(nx=512, ny=512, nz=384, T_bottom=0.85, T_top=0.95, mean_blobs=256,
                 rmin=8.0, rmax=30.0, W=5.0, seed=4, steps=1000, cutoff=15.0, gap=10.0,
                 max_attempts=64):
    """Closed box between two no-slip walls (z = 0 at T_bottom*Tc, z = nz-1 at
    T_top*Tc), periodic x, y, linear initial T(z); a Poisson(mean_blobs)
    number of liquid blobs with radii U[rmin, rmax], centres uniform in x, y
    and in z within [r + 3, nz - 4 - r].  Blobs do not overlap: a candidate
    closer than r_i + r_j + gap (periodic in x, y) to an accepted blob is
    redrawn (up to max_attempts draws per blob), so no vapour pocket is
    trapped between merging liquid bodies.
    rho = rho_v(T(z)) + (rho_l - rho_v)(T(z)) max_k 1/2[1 - tanh(2 (d_k - r_k)/W)],
    each blob profile truncated to 0 beyond d_k - r_k > cutoff.
    The cold wall defaults to 0.85 Tc: at 0.80 Tc the liquid of the larger
    blobs (r > 15) is compressed past the psi^2 > 0 limit (rho ~ 9.1) within
    a few tens of steps, in the oracle as on the GPU."""
    faces = [PERIODIC, PERIODIC, PERIODIC, PERIODIC, WALL, WALL]
    Tmid = 0.5 * (T_bottom + T_top)
    w = _base("blobs_closed", nx, ny, nz, faces, steps, Tmid)
    Tc = w["Tc"]
    w["face_T"] = [0.0, 0.0, 0.0, 0.0, T_bottom * Tc, T_top * Tc]
    zc = np.arange(nz, dtype=np.float64)
    t_over = T_bottom + (T_top - T_bottom) * zc / (nz - 1)
    rv, rl = coexistence(t_over)
    u0 = uniform01(seed, 1)[0]
    nb = _poisson(mean_blobs, u0)
    draws = uniform01(seed + 1000, 4 * max(nb, 1) * max_attempts).reshape(-1, 4)
    blobs = []
    cursor = 0
    for _ in range(nb):
        for _attempt in range(max_attempts):
            d = draws[cursor]
            cursor += 1
            r = rmin + (rmax - rmin) * d[3]
            zlo, zhi = r + 3.0, (nz - 4.0) - r
            if zhi < zlo:
                continue
            c = (d[0] * nx, d[1] * ny, zlo + (zhi - zlo) * d[2])
            ok = True
            for (bx, by, bz, br) in blobs:
                dx = abs(c[0] - bx)
                dx = min(dx, nx - dx)
                dy = abs(c[1] - by)
                dy = min(dy, ny - dy)
                if dx * dx + dy * dy + (c[2] - bz) ** 2 < (r + br + gap) ** 2:
                    ok = False
                    break
            if ok:
                blobs.append((c[0], c[1], c[2], r))
                break
    frac = np.zeros((nz, ny, nx), dtype=np.float64)
    for (cx, cy, cz, r) in blobs:
        ext = r + cutoff
        z0 = max(int(np.floor(cz - ext)), 0)
        z1 = min(int(np.ceil(cz + ext)) + 1, nz)
        ys = np.arange(int(np.floor(cy - ext)), int(np.ceil(cy + ext)) + 1)
        xs = np.arange(int(np.floor(cx - ext)), int(np.ceil(cx + ext)) + 1)
        zs = np.arange(z0, z1)
        dz = (zs - cz)[:, None, None]
        dy = (ys - cy)[None, :, None]
        dx = (xs - cx)[None, None, :]
        dist = np.sqrt(dx * dx + dy * dy + dz * dz)
        prof = np.where(dist - r > cutoff, 0.0, 0.5 * (1.0 - np.tanh(2.0 * (dist - r) / W)))
        sel = np.ix_(zs, np.mod(ys, ny), np.mod(xs, nx))
        frac[sel] = np.maximum(frac[sel], prof)
    rho = rv[:, None, None] + (rl - rv)[:, None, None] * frac
    w["rho0"] = rho
    w["T0"] = np.broadcast_to((t_over * Tc)[:, None, None], rho.shape).copy()
    w["n_blobs"] = len(blobs)
    w["blobs"] = blobs
    w["rho_v"] = float(coexistence(Tmid)[0])
    w["rho_l"] = float(coexistence(Tmid)[1])
    return w


def named(name: str, **kw) -> Dict:
    """The five standard workloads by name, full size unless overridden."""
    table = {
        "droplet_periodic_32": lambda: droplet_periodic(**kw),
        "droplet_open_128": lambda: droplet_open(**kw),
        "heated_wall_256": lambda: heated_wall(**kw),
        "blobs_closed_512x512x384": lambda: blobs_closed(**kw),
        "heated_wall_adjoint_96": lambda: heated_wall(**dict(dict(n=96, R0=15.0, steps=2000,
                                                                  Tw_jitter=0.02, seed=5), **kw)),
    }
    return table[name]()
