"""Pins of the oracle's transport physics: relaxation rates, viscosity, the
no-slip wall and the temperature source.

Each test fixes a part of the oracle against what the paper states and what
the mathematics gives for a special input: the relaxation values of Sec. 4
(shear viscosity 0.25), the temperature equation eq. (12) that the D3Q7
scheme recovers (eq. (33)), the continuity equation, and the statement of
Sec. 3.1 that the velocity of a wall node is prescribed.  None of them
re-evaluates an oracle formula; the inputs are built from the printed
definitions (moment monomials of (A.1), the equilibrium eq. (2)) and the
expected values are closed forms or invariants.
"""
import numpy as np
import pytest

from oracle import lbm_oracle as O

TC = O.critical_temperature(O.Params(1, 1, 1))
T_SAT = 0.86 * TC


def _moment_basis():
    """The rows of (A.1) as the monomials 1, x, y, z, |c|^2, 2x^2-y^2-z^2,
    y^2-z^2, xy, xz, yz, x^2y, xy^2, x^2z, xz^2, y^2z, yz^2, x^2y^2, x^2z^2,
    y^2z^2 of the velocities (built here, not taken from the oracle's table)."""
    c = O.C19.astype(float)
    x, y, z = c[:, 0], c[:, 1], c[:, 2]
    return np.array([np.ones(19), x, y, z, x * x + y * y + z * z, 2 * x * x - y * y - z * z, y * y - z * z,
                     x * y, x * z, y * z, x * x * y, x * y * y, x * x * z, x * z * z, y * y * z, y * z * z,
                     x * x * y * y, x * x * z * z, y * y * z * z])


def _complex_step(fun, x, h=1e-30):
    return np.imag(fun(x + 1j * h)) / h


def _dp_dT(rho, T, p):
    """Partial derivative of the Peng-Robinson pressure eq. (54) in T at fixed
    rho, by complex step (exact to rounding, independent of the oracle's
    closed-form derivative)."""
    return _complex_step(lambda t: O.pr_pressure(rho + 0j, t, p), T)


# ---------------------------------------------------------------- D3Q19 relaxation

# Sec. 4: the shear relaxation time 1.25 (shear viscosity 0.25) and the bulk
# relaxation time 0.8, all other rates 1; read as rates s = 1/time
PAPER_RATES = {4: 1 / 0.8, 5: 1 / 1.25, 6: 1 / 1.25, 7: 1 / 1.25, 8: 1 / 1.25, 9: 1 / 1.25,
               10: 1.0, 11: 1.0, 12: 1.0, 13: 1.0, 14: 1.0, 15: 1.0, 16: 1.0, 17: 1.0, 18: 1.0}


@pytest.mark.parametrize("k", sorted(PAPER_RATES))
def test_moment_relaxation_rates_of_a_uniform_state(k):
    """eq. (8) on a uniform state at rest: F = 0 and streaming moves nothing, so
    one step multiplies the departure of each non-conserved moment from its
    equilibrium by exactly (1 - s_k) and leaves every other moment alone.
    Pins the relaxation matrix of eq. (11) with the Sec. 4 values, moment by
    moment (a swapped or repeated rate fails here)."""
    M = _moment_basis()
    Minv = np.linalg.inv(M)
    p = O.Params(3, 3, 3)
    rho0, d = 0.9, 1e-4
    f = O.feq19(np.full(p.shape, rho0), np.zeros((3,) + p.shape))
    f = f + (Minv[:, k] * d)[:, None, None, None]
    g = O.geq7(np.full(p.shape, T_SAT), p)
    f1, _, _ = O.step(f, g, p)
    m1 = np.einsum("ki,izyx->kzyx", M, f1)
    meq = M @ O.feq19(np.array(rho0), np.zeros(3))
    dep = m1 - meq[:, None, None, None]
    assert np.allclose(dep[k], (1.0 - PAPER_RATES[k]) * d, rtol=1e-9, atol=1e-15)
    others = np.delete(dep, k, axis=0)
    assert np.abs(others).max() < 1e-14


def _shear_rate(n, walls):
    """Decay factor per step of the fundamental shear mode u_x(z) of small
    amplitude on a 1 x 1 x n column, measured after the non-hydrodynamic
    transient.  Periodic: sin(2 pi z / n).  Walls at z = 0 and n-1:
    sin(pi z / (n - 1)), zero on the wall nodes."""
    if walls:
        p = O.Params(1, 1, n, faces=(0, 0, 0, 0, O.WALL, O.WALL), face_T=(0, 0, 0, 0, T_SAT, T_SAT))
        prof = np.sin(np.pi * np.arange(n) / (n - 1))
    else:
        p = O.Params(1, 1, n)
        prof = np.sin(2 * np.pi * np.arange(n) / n)
    u = np.zeros((3,) + p.shape)
    u[0] = 1e-6 * prof[:, None, None]
    f = O.feq19(np.full(p.shape, 0.9), u)
    g = O.geq7(np.full(p.shape, T_SAT), p)

    def amp(f, g):
        _, uu, _ = O.fields(f, g, p)
        return np.sum(uu[0][:, 0, 0] * prof) / np.sum(prof * prof)

    f, g = O.run(f, g, p, 50)
    a0 = amp(f, g)
    f, g = O.run(f, g, p, 200)
    return (amp(f, g) / a0) ** (1.0 / 200)


def test_shear_wave_decay_gives_the_paper_viscosity():
    """A periodic shear wave decays as exp(-nu k^2 t) with nu = 0.25 (Sec. 4:
    'shear viscosity 0.25'; nu = c_s^2 (1/s_nu - 1/2)).  The measured nu(k)
    converges at second order in k: the Richardson extrapolation of the
    16- and 32-cell columns must give 0.25."""
    nus = {}
    for n in (16, 32):
        k = 2 * np.pi / n
        nus[n] = -np.log(_shear_rate(n, walls=False)) / k ** 2
    assert abs(nus[32] - 0.25) < 5e-4 and abs(nus[16] - 0.25) < 2e-3
    assert abs(nus[32] - 0.25) < 0.35 * abs(nus[16] - 0.25)       # second order
    assert abs((4 * nus[32] - nus[16]) / 3 - 0.25) < 2e-5


def test_shear_flow_between_no_slip_walls():
    """Sec. 3.1, eq. (34) with the wall-node velocity prescribed 0: a shear
    mode between walls at z = 0 and z = n-1 decays as exp(-nu (pi/L)^2 t)
    with L = n - 1 - delta.  Two column heights give nu and delta: nu must be
    the viscosity 0.25 and the no-slip surface must lie within a fifth of a
    cell of the wall nodes (|delta| < 0.4; measured: a tenth of a cell beyond
    each wall node.  A wall node that relaxes to its own momentum instead of
    the prescribed rest moves it about half a cell beyond, delta ~ -1)."""
    L1, L2 = 32, 64
    r1, r2 = -np.log(_shear_rate(L1 + 1, True)), -np.log(_shear_rate(L2 + 1, True))
    # sqrt(r) = pi sqrt(nu) / (L - delta)
    sq_nu = (L2 - L1) / (np.pi * (1 / np.sqrt(r2) - 1 / np.sqrt(r1)))
    nu = sq_nu ** 2
    delta = L1 - np.pi * sq_nu / np.sqrt(r1)
    assert abs(nu - 0.25) < 2e-4, nu
    assert abs(delta) < 0.4, delta


def test_wall_node_at_rest_collides_like_an_interior_node():
    """Sec. 3.1: the velocity of a wall node is prescribed (zero).  A fluid
    already at rest (real velocity of eq. (5) zero everywhere) is unchanged by
    that prescription, so one step of a z-uniform state at rest in a box with
    no-slip z walls (kappa_w = 0, whose ghost layer mirrors the wall layer)
    gives the wall layer the same populations as the z-periodic box, for
    every direction that does not arrive through the wall (c_z <= 0 at z = 0,
    c_z >= 0 at z = nz-1).  The state has a liquid/vapour density profile
    along x, so the interaction force and u_eq = -F/(2 rho) of the wall nodes
    do not vanish."""
    nx, ny, nz = 24, 2, 5
    x = np.arange(nx)
    rho_x = 0.38 + 3.0 * np.exp(-((x - nx / 2) / 4.0) ** 2)
    rho = np.broadcast_to(rho_x[None, None, :], (nz, ny, nx)).copy()
    T = np.full((nz, ny, nx), T_SAT)
    per = O.Params(nx, ny, nz)
    wal = O.Params(nx, ny, nz, faces=(0, 0, 0, 0, O.WALL, O.WALL), face_T=(0, 0, 0, 0, T_SAT, T_SAT))
    F = O.interaction_force(O.pseudopotential(rho, T, per), per)
    assert np.abs(F[0]).max() > 1e-3
    f = O.feq19(rho, -F / (2 * rho))                     # real velocity zero
    g = O.geq7(T, per)
    fp, _, _ = O.step(f, g, per)
    fw, _, mac = O.step(f, g, wal)
    assert np.abs(mac["ueq"][0]).max() > 1e-4
    cz = O.C19[:, 2]
    lo, hi = cz <= 0, cz >= 0
    assert np.abs(fw[lo, 0] - fp[lo, 0]).max() < 1e-15
    assert np.abs(fw[hi, -1] - fp[hi, -1]).max() < 1e-15


# ---------------------------------------------------------------- temperature source

def test_compression_heating_one_step_closed_form():
    """eq. (15) compression term on a uniform fluid (F = 0) with the velocity
    u = A (sin kx, sin ky, sin kz) and uniform T at equilibrium (no local
    temperature gradient): after one step
        T - T0 = -(T0 dp/dT / (rho c_v)) A sin(k) [1 - (wbar/3)(1 - cos k)]
                 (cos kx + cos ky + cos kz),
    the factor sin(k)/k being the isotropic divergence stencil on a sine and
    the bracket the spread of -w_i Fbar over the D3Q7 links (eq. (13)).  As
    k -> 0 this is -T dp/dT div u / (rho c_v) of eq. (12)."""
    errs = []
    for n in (8, 16, 32):
        p = O.Params(n, n, n)
        k = 2 * np.pi / n
        A, rho0 = 1e-5, 0.9
        s = np.sin(k * np.arange(n))
        u = np.zeros((3,) + p.shape)
        u[0] = A * s[None, None, :]
        u[1] = A * s[None, :, None]
        u[2] = A * s[:, None, None]
        f = O.feq19(np.full(p.shape, rho0), u)
        g = O.geq7(np.full(p.shape, T_SAT), p)
        _, g1, _ = O.step(f, g, p)
        c = np.cos(k * np.arange(n))
        S = c[None, None, :] + c[None, :, None] + c[:, None, None]
        coef = -T_SAT * _dp_dT(rho0, T_SAT, p) / (rho0 * p.cv)
        exact = coef * A * np.sin(k) * (1 - (p.wbar / 3) * (1 - np.cos(k))) * S
        dT = g1.sum(0) - T_SAT
        assert np.abs(dT - exact).max() < 1e-8 * np.abs(exact).max()
        errs.append(np.abs(dT - coef * A * k * S).max() / np.abs(coef * A * k * S).max())
    assert errs[1] < 0.3 * errs[0] and errs[2] < 0.3 * errs[1] and errs[2] < 0.015


def _one_step_T_change(n, rho0, u0, eps=1e-6):
    """uniform rho0, uniform velocity u0 along x, T = T_sat + eps sin(kx) with
    the first moments of g set to the local gradient of eqs. (27)-(29),
    m_x = -(c_s^2 / varsigma) dT/dx.  Returns (one-step T change, T', T'')."""
    p = O.Params(n, 1, 1)
    k = 2 * np.pi / n
    x = np.arange(n)
    T = T_SAT + eps * np.sin(k * x)
    dT = eps * k * np.cos(k * x)
    d2T = -eps * k * k * np.sin(k * x)
    u = np.zeros((3,) + p.shape)
    u[0] = u0
    f = O.feq19(np.full(p.shape, rho0), u)
    Tf = np.broadcast_to(T[None, None, :], p.shape).copy()
    g = O.geq7(Tf, p)
    m = -(p.cs2_T / p.varsigma_flux) * dT[None, None, :]
    g[1] += m / 2
    g[2] -= m / 2
    _, g1, _ = O.step(f, g, p)
    return (g1.sum(0) - Tf)[0, 0], dT, d2T, p


@pytest.mark.parametrize("rho0,u0", [(0.38, 0.02), (6.5, 0.0), (6.5, 0.01)])
def test_temperature_equation_recovered_in_one_step(rho0, u0):
    """eq. (12) is what eqs. (13)-(15) recover (eq. (33)):
        rho c_v (dT/dt + u.grad T) = div(lambda grad T) - T dp/dT div u,
    with u the real velocity of eq. (5).  For a uniform density and a small
    temperature sine, u = u0 + F/(2 rho) with F = grad(rho c_s^2 - p) =
    -dp/dT grad T (eq. (6) with G = -1 at long wavelength), so at first order
        dT/dt = -u0 T' + [lambda + T (dp/dT)^2 / (2 rho)] T'' / (rho c_v):
    the half-force part of the real velocity compresses the fluid where it is
    hot.  The one-step change must match this to O(k^2) (second-order
    convergence over 32, 64, 128 cells), which fixes the sign and size of
    both source terms, the conductivity map of eq. (33) and the use of the
    real velocity in the divergence."""
    errs = []
    for n in (32, 64, 128):
        dTs, dT, d2T, p = _one_step_T_change(n, rho0, u0)
        pT = _dp_dT(rho0, T_SAT, p)
        rhs = -u0 * dT + (p.lam + T_SAT * pT * pT / (2 * rho0)) * d2T / (rho0 * p.cv)
        errs.append(np.abs(dTs - rhs).max() / np.abs(rhs).max())
    assert errs[2] < 2e-3, errs
    assert errs[1] < 0.35 * errs[0] and errs[2] < 0.35 * errs[1], errs


def test_source_vanishes_at_zero_real_velocity():
    """eq. (15) is written with the velocity u of eq. (5), not u_eq of eq. (3):
    a non-uniform fluid whose real velocity is zero everywhere (populations at
    equilibrium with u_eq = -F/(2 rho)) has no convective and no compression
    source, however large u_eq and the local temperature gradient are."""
    n = 16
    p = O.Params(n, n, n)
    i = np.arange(n)
    zz, yy, xx = np.meshgrid(i, i, i, indexing="ij")
    k = 2 * np.pi / n
    rho = 2.0 + (np.sin(k * xx) * np.cos(k * yy) + 0.5 * np.sin(k * zz)) / 1.5
    T = T_SAT * (1 + 0.02 * np.cos(k * xx + 0.3) * np.sin(k * zz))
    F = O.interaction_force(O.pseudopotential(rho, T, p), p)
    f = O.feq19(rho, -F / (2 * rho))
    g = O.geq7(T, p)
    g[1] += 1e-3 * np.sin(k * yy)
    g[2] -= 1e-3 * np.sin(k * yy)
    g[5] += 1e-3 * np.cos(k * xx)
    g[6] -= 1e-3 * np.cos(k * xx)
    mac = O.macroscopic(f, g, p)
    conv = rho * p.cv * np.sum(mac["ueq"] * mac["gradT"], axis=0)
    assert np.abs(conv).max() > 1e-4
    assert np.abs(mac["Fbar"]).max() < 1e-12 * np.abs(conv).max()


def test_wall_node_divergence_matches_its_mass_balance():
    """At a no-slip wall node the fluid does not move (Sec. 3.1), so the
    continuity equation reads d rho/dt = -rho div u there: the divergence that
    enters the compression term of eq. (15) at the wall node must equal the
    node's relative mass loss over the step.  A flow u_z = A sin(pi z/(n-1))
    towards and away from the walls, uniform rho and T."""
    n = 24
    p = O.Params(1, 1, n, faces=(0, 0, 0, 0, O.WALL, O.WALL), face_T=(0, 0, 0, 0, T_SAT, T_SAT))
    u = np.zeros((3,) + p.shape)
    u[2] = 1e-6 * np.sin(np.pi * np.arange(n) / (n - 1))[:, None, None]
    f = O.feq19(np.full(p.shape, 0.9), u)
    g = O.geq7(np.full(p.shape, T_SAT), p)
    mac = O.macroscopic(f, g, p)
    f1, _, _ = O.step(f, g, p)
    r0, r1 = f.sum(0)[:, 0, 0], f1.sum(0)[:, 0, 0]
    loss = -(r1 - r0) / r0
    div = mac["div_u"][:, 0, 0]
    for z in (0, n - 1):
        assert abs(div[z]) > 1e-8
        assert abs(div[z] - loss[z]) < 1e-5 * abs(loss[z])
