"""Physics checks of the method, run through the GPU library in FP64 (which
agrees with the oracle to 1e-12 per step) or FP32:

* flat interface: the converged bulk densities of a liquid slab equal the
  oracle's (a stored value) and lie near the Maxwell equal-area coexistence
  densities of the Peng-Robinson EOS (eqs. (54)-(55));
* Laplace law: the pressure jump across a droplet is linear in 1/R with a
  small intercept;
* d^2 law (Sec. 4.2, eq. (56)): after the initial transient the squared
  diameter of an evaporating droplet falls linearly in time;
* heat transfer through a flat interface between two conductivities
  (Sec. 4.1): at steady state the temperature slopes in the two phases are
  in the inverse ratio of the conductivities (2; the paper reports 1.9507).

The two equilibrium checks hold T fixed by taking c_v very large (the rho c_v
blend of eq. (13) then leaves g unchanged to 1e-6 per step), which isolates
the flow lattice.  Pseudopotential models are not exactly Maxwell-consistent
and the paper prints no numbers for these cases, so the bounds are loose and
the measured values are printed.
"""
import sys

import numpy as np
import pytest

from oracle import lbm_oracle as O
from workloads import synth

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_2206_00946_amd as P
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    P.load_library()
    return P


def _isothermal(P, w, prec="fp64"):
    prm = P.params_from_workload(w, prec)
    prm.cv = 1e6
    sim = P.Lbm3D(prm)
    sim.init(w["rho0"], w["T0"])
    return sim


def test_flat_interface_coexistence(P):
    """Converged slab: equal to the oracle's converged 1-D column
    (tests/golden/slab_coexistence.json) and near the Maxwell construction
    (the model's vapour density sits 16 % below it: pseudopotential
    coexistence is not Maxwell-consistent)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "slab_coexistence.json")))
    w = synth.slab(nx=128, ny=8, nz=8, width=64.0)
    _log("flat interface 128x8x8 FP64, 20000 steps")
    sim = _isothermal(P, w)
    sim.step(20000)
    rho, u, T = sim.fields()
    sim.close()
    prof = rho.mean(axis=(0, 1))
    rl, rv = prof[w["nx"] // 2], prof[0]
    el, ev = rl / w["rho_l"] - 1, rv / w["rho_v"] - 1
    _log(f"  rho_l {rl:.8f} (oracle {gold['rho_liquid']:.8f}, Maxwell {el:+.2e})  "
         f"rho_v {rv:.8f} (oracle {gold['rho_vapour']:.8f}, Maxwell {ev:+.2e})")
    assert abs(rl / gold["rho_liquid"] - 1) < 1e-6 and abs(rv / gold["rho_vapour"] - 1) < 1e-6
    assert abs(el) < 0.01 and abs(ev) < 0.2
    assert np.max(np.abs(rho - prof[None, None, :])) < 1e-9 * rl  # stays one-dimensional


def test_laplace_law(P):
    p = O.Params(64, 64, 64)
    pts = []
    for R in (12, 14, 16, 20):
        w = synth.droplet_periodic(n=64, R0=float(R), noise=0.0)
        sim = _isothermal(P, w)
        sim.step(10000)
        rho, u, T = sim.fields()
        sim.close()
        c = 32
        dp = O.pr_pressure(rho[c, c, c], T[c, c, c], p) - O.pr_pressure(rho[0, 0, 0], T[0, 0, 0], p)
        vol = float(np.sum(np.clip((rho - w["rho_v"]) / (w["rho_l"] - w["rho_v"]), 0.0, 1.0)))
        Reff = (3.0 * vol / (4.0 * np.pi)) ** (1.0 / 3.0)
        pts.append((1.0 / Reff, dp))
        _log(f"  R0 {R}: R {Reff:.3f} rho_in {rho[c, c, c]:.5f} rho_out {rho[0, 0, 0]:.5f} dp {dp:.5e}")
    x, y = np.array(pts).T
    A = np.vstack([x, np.ones_like(x)]).T
    (slope, icpt), *_ = np.linalg.lstsq(A, y, rcond=None)
    r2 = 1.0 - np.sum((y - (slope * x + icpt)) ** 2) / np.sum((y - y.mean()) ** 2)
    _log(f"  Laplace fit: 2 sigma = {slope:.5f}, intercept {icpt:.3e}, r^2 {r2:.5f}")
    assert r2 > 0.99 and slope > 0
    assert abs(icpt) < 0.1 * y.min()


def _d2_rate(P, w):
    """Evaporation rate K of the d^2 law over t in [4000, 20000] and r^2."""
    import torch
    sim = P.from_workload(w, "fp32")
    t, vol = [], []
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(sim.stream)
    for k in range(201):
        d = sim.reduce()
        t.append(100 * k)
        vol.append(d["vol_smooth"])
        if k < 200:
            sim.step(100)
    end.record(sim.stream)
    torch.cuda.synchronize()
    sim.close()
    t, vol = np.array(t, dtype=float), np.array(vol)
    D2 = (6.0 * vol / np.pi) ** (2.0 / 3.0)
    sel = t >= 4000
    A = np.vstack([t[sel], np.ones(sel.sum())]).T
    (m, c), *_ = np.linalg.lstsq(A, D2[sel], rcond=None)
    r2 = 1.0 - np.sum((D2[sel] - (m * t[sel] + c)) ** 2) / np.sum((D2[sel] - D2[sel].mean()) ** 2)
    return -m, r2, D2, start.elapsed_time(end) / 20000.0


def test_d2_law_with_and_without_correction(P):
    """vartheta = 0 and 1 give almost the same evaporation rate (Sec. 4.1
    and Table 1 of the paper report the two as almost the same)."""
    w = synth.named("droplet_open_128")
    K0, r0, _, ms0 = _d2_rate(P, w)
    w1 = dict(w)
    w1["theta_corr"] = 1
    K1, r1, _, ms1 = _d2_rate(P, w1)
    _log(f"  K(theta=0) {K0:.5e} ({ms0:.4f} ms/step)  K(theta=1) {K1:.5e} ({ms1:.4f} ms/step)  "
         f"relative difference {K1 / K0 - 1:+.2e}, time {ms1 / ms0 - 1:+.1%}")
    assert r1 > 0.99 and abs(K1 / K0 - 1) < 0.05


def _d2_series(P, w, prec):
    sim = P.from_workload(w, prec)
    t, vol = [], []
    for k in range(201):
        d = sim.reduce()
        t.append(100 * k)
        vol.append(d["vol_smooth"])
        if k < 200:
            sim.step(100)
    rho, _, T = sim.fields()
    sim.close()
    t, vol = np.array(t, dtype=float), np.array(vol)
    return t, (6.0 * vol / np.pi) ** (2.0 / 3.0), rho, T


def test_d2_law(P):
    """The 128^3 evaporating droplet (Zou-He outlets on all six faces, faces
    at 1.1 T_sat) in FP64 and in FP32 deviation storage: (D/D0)^2 is linear
    in t after the initial transient in both, and FP32 follows FP64."""
    w = synth.named("droplet_open_128")
    out = {}
    for prec in ("fp64", "fp32"):
        _log(f"d^2 law: droplet_open_128 {prec}, 20000 steps, volume every 100")
        t, D2, rho, T = _d2_series(P, w, prec)
        sel = t >= 4000
        A = np.vstack([t[sel], np.ones(sel.sum())]).T
        (m, c), *_ = np.linalg.lstsq(A, D2[sel], rcond=None)
        r2 = 1.0 - np.sum((D2[sel] - (m * t[sel] + c)) ** 2) / np.sum((D2[sel] - D2[sel].mean()) ** 2)
        _log(f"  {prec}: D0^2 {D2[0]:.1f}, K = {-m:.5e} per step, r^2 {r2:.5f}, "
             f"final (D/D0)^2 {D2[-1] / D2[0]:.4f}")
        assert m < 0 and r2 > 0.99
        out[prec] = (D2 / D2[0], rho, T, -m)
    d_curve = float(np.max(np.abs(out["fp32"][0] - out["fp64"][0])))
    rel_rho = np.abs(out["fp32"][1] - out["fp64"][1]) / out["fp64"][1]
    e_rho = float(rel_rho.max())
    at = np.unravel_index(int(np.argmax(rel_rho)), rel_rho.shape)
    c = np.array(rel_rho.shape) // 2
    _log(f"  largest rho difference at (z, y, x) = {tuple(int(v) for v in at)}, "
         f"{float(np.linalg.norm(np.array(at) - c)):.1f} cells from the centre, rho64 {float(out['fp64'][1][at]):.4f}; "
         f"99.9th percentile {float(np.quantile(rel_rho, 0.999)):.2e}, median {float(np.median(rel_rho)):.2e}")
    e_T = float(np.max(np.abs(out["fp32"][2] - out["fp64"][2]) / out["fp64"][2]))
    e_K = abs(out["fp32"][3] / out["fp64"][3] - 1)
    _log(f"  FP32 vs FP64 after 20000 steps: rho {e_rho:.2e}, T {e_T:.2e} (max relative), "
         f"(D/D0)^2 curve {d_curve:.2e} (max absolute), K {e_K:.2e} (relative)")
    # integral measures and T to 1e-4 / 1e-3; pointwise rho after 20000 steps
    # to 1e-2 (the largest differences sit in the interface, see the log)
    assert e_T < 1e-4 and d_curve < 1e-4 and e_K < 1e-3 and e_rho < 1e-2


def test_saturated_heat_transfer_slope_ratio(P):
    """Sec. 4.1 set-up turned to z walls (10 x 10 x 100 here, half the
    paper's length so that the liquid reaches steady state in 1.5e6 steps):
    vapour (lambda 0.2) below liquid (lambda 0.4), hot wall at T_c, cold wall
    at T_sat.  Fourier's law with a continuous heat flux gives a slope ratio
    of 2; the model converges to about 1.90 (the paper reports 1.9507)."""
    w = synth.saturated_heat_transfer(nz=100)
    _log("saturated heat transfer 10x10x100 FP64, 1.5e6 steps")
    sim = P.from_workload(w, "fp64")
    sim.step(1500000)
    rho, u, T = sim.fields()
    sim.close()
    Tz = T.mean(axis=(1, 2)) / w["Tc"]
    rz = rho.mean(axis=(1, 2))
    mid = 0.5 * (w["rho_v"] + w["rho_l"])
    iface = int(np.argmax((rz[:-1] - mid) * (rz[1:] - mid) < 0))
    zv, zl = np.arange(5, iface - 5), np.arange(iface + 5, 95)
    sv, sl = np.polyfit(zv, Tz[zv], 1)[0], np.polyfit(zl, Tz[zl], 1)[0]
    lin_v = np.max(np.abs(Tz[zv] - np.polyval(np.polyfit(zv, Tz[zv], 1), zv)))
    _log(f"  interface at z = {iface}, slopes {sv:.5e} (vapour) {sl:.5e} (liquid), ratio {sv / sl:.4f}, "
         f"vapour profile linear to {lin_v:.1e}")
    assert abs(sv / sl - 2.0) < 0.12
    assert lin_v < 1e-3


def _cap_angle(w, rho, zwall=-0.5):
    """Contact angle of a sessile droplet from a spherical-cap fit of the
    liquid area of each z layer (away from the wall and the apex); the wall
    lies half a cell below the first fluid layer (the ghost layer of eq. (37)
    mirrors layer 1 about layer 0)."""
    frac = np.clip((rho - w["rho_v"]) / (w["rho_l"] - w["rho_v"]), 0.0, 1.0)
    area = frac.sum(axis=(1, 2))
    top = int(np.max(np.nonzero(area > 50)[0]))
    zs = np.arange(3, top - 3)
    A = np.vstack([2.0 * zs, np.ones_like(zs)]).T.astype(float)
    (zc, c), *_ = np.linalg.lstsq(A, area[zs] / np.pi + zs ** 2, rcond=None)
    R = np.sqrt(c + zc ** 2)
    return float(np.degrees(np.arccos(np.clip(-(zc - zwall) / R, -1.0, 1.0))))


@pytest.mark.parametrize("theta", [60.0, 90.0, 120.0])
def test_contact_angle_of_the_wetting_layer(P, theta):
    """eq. (37) with kappa_w = tan(pi/2 - theta): a hemispherical droplet of
    diameter 70 on a 160 x 160 x 100 wall (the Sec. 4.3 geometry) relaxes to
    the prescribed angle; T held fixed (wall at T_sat, very large c_v) so that
    only wetting acts; FP32, 2000 steps."""
    w = synth.heated_surface(theta_deg=theta, Tw=0.86)
    w["cv"] = 1e6
    sim = P.from_workload(w, "fp32")
    sim.step(2000)
    rho, _, _ = sim.fields()
    sim.close()
    got = _cap_angle(w, rho)
    _log(f"  prescribed {theta:.0f} deg, fitted {got:.1f} deg")
    assert abs(got - theta) < 6.0


def test_droplet_on_heated_surface_evaporates(P):
    """Sec. 4.3 set-up (160 x 160 x 100, diameter 70, theta = 120 deg, wall at
    0.8931 T_c, outlet on top): the droplet loses mass at a steady rate."""
    w = synth.heated_surface()
    sim = P.from_workload(w, "fp32")
    mass, vol = [], []
    for _ in range(5):
        d = sim.reduce()
        mass.append(d["mass"])
        vol.append(d["vol_smooth"])
        sim.step(2000)
    sim.close()
    _log(f"  liquid volume {vol[0]:.0f} -> {vol[-1]:.0f} over 8000 steps")
    assert all(b < a for a, b in zip(vol[1:], vol[2:]))
    assert vol[-1] < 0.97 * vol[0]
