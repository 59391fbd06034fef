"""The oracle's pins against plausible mistakes, each planted in a temporary
copy of the oracle (CPU only; the repository's oracle is not touched).  A
planted mistake must make the pins named beside it fail.

Misreadings of the paper's transport terms (the transport pins):
  the bulk and shear rates of eq. (11) swapped, s_q set to s_nu, s_pi halved
  (the Sec. 4 relaxation values); the convective term of eq. (15) or the
  divergence built from u_eq instead of the real velocity of eq. (5); the
  sign of either source term flipped; the wall-node velocity of Sec. 3.1
  read as u_eq = 0, or not prescribed at all; the ghost velocity beyond a
  wall copied from the first interior layer instead of 0.
Slips elsewhere (the other pins): the force weights of eq. (6) swapped; the
factor 2 of eq. (7) dropped; a sign in the denominator of eq. (54); the
forcing term of eq. (8) with the wrong sign or half the velocity shift;
bounce-back (eq. (34)) onto the same slot; streaming without the rho c_v
blend of eq. (13); the source of eq. (15) added instead of subtracted; a
sign in eq. (36); a sign in the outlet fill (Sec. 3.3); the divergence
without its 1/c_s^2; the D3Q7 equilibrium moment w_bar T of eq. (25) set
to 0.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join("oracle", "lbm_oracle.py")
TRANSPORT = "tests/test_oracle_pins_transport.py"
PINS = "tests/test_oracle_pins.py"

# name: (text in the oracle, mistake written in its place, pins that must fail)
MISTAKES = {
    "bulk_and_shear_rates_swapped": ("[1.0, 1.0, 1.0, 1.0, self.s_e] + [self.s_nu] * 5",
                                     "[1.0, 1.0, 1.0, 1.0, self.s_nu] + [self.s_e] * 5", [TRANSPORT]),
    "s_q_equal_to_s_nu": ("[self.s_q] * 6", "[self.s_nu] * 6", [TRANSPORT]),
    "s_pi_halved": ("[self.s_pi] * 3", "[0.5 * self.s_pi] * 3", [TRANSPORT]),
    "convection_with_u_eq": ("np.sum(u * gradT, axis=0)", "np.sum(ueq * gradT, axis=0)", [TRANSPORT]),
    "divergence_of_u_eq": ("div_u = divergence(u, p)", "div_u = divergence(ueq, p)", [TRANSPORT]),
    "compression_sign": ("+ T * dpdT * div_u", "- T * dpdT * div_u", [TRANSPORT]),
    "convection_sign": ("Fbar = rho * p.cv * np.sum", "Fbar = -rho * p.cv * np.sum", [TRANSPORT]),
    "wall_node_u_eq_zero": ("ueq = np.where(wall, -0.5 * du, ueq)", "ueq = np.where(wall, 0.0, ueq)",
                            [TRANSPORT]),
    "wall_node_not_prescribed": ("    if wall.any():", "    if False:", [TRANSPORT]),
    "ghost_u_copied_inward": ("lambda w, i: np.zeros_like(w))", "lambda w, i: i)", [TRANSPORT]),
    "force_weights_swapped": ("varpi = 1.0 / 6.0 if int(np.dot(c, c)) == 1 else 1.0 / 12.0",
                              "varpi = 1.0 / 12.0 if int(np.dot(c, c)) == 1 else 1.0 / 6.0",
                              [PINS + "::test_force_stencil_is_exact_gradient"]),
    "psi_without_factor_2": ("return 2.0 * (pr_pressure(rho, T, p) - rho * CS2) / p.G",
                             "return (pr_pressure(rho, T, p) - rho * CS2) / p.G",
                             [TRANSPORT + "::test_temperature_equation_recovered_in_one_step"]),
    "pr_denominator_sign": ("- p.a * pr_xi(T, p) * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho))",
                            "- p.a * pr_xi(T, p) * rho * rho / (1.0 + 2.0 * b * rho + b * b * rho * rho))",
                            [PINS + "::test_pr_critical_point"]),
    "forcing_sign": ("mstar = m - lam * (m - me0) + (me1 - me0)", "mstar = m - lam * (m - me0) - (me1 - me0)",
                     [PINS + "::test_collision_conserves_mass_and_adds_force"]),
    "forcing_half_shift": ("me1 = meq19(rho, ueq + du)", "me1 = meq19(rho, ueq + 0.5 * du)",
                           [PINS + "::test_collision_conserves_mass_and_adds_force"]),
    "bounce_back_same_slot": ("out[i, zb] = fstar[OPP19[i], zb]", "out[i, zb] = fstar[i, zb]",
                              [PINS + "::test_bounce_back_brute_force"]),
    "streaming_without_blend": ("blended = g[i] + (src - g[i]) * inv", "blended = src",
                                [PINS + "::test_energy_identity_periodic"]),
    "source_added": ("gstar = M7_INV @ nstar - w7(p.wbar)[:, None]", "gstar = M7_INV @ nstar + w7(p.wbar)[:, None]",
                     [PINS + "::test_energy_identity_periodic"]),
    "dirichlet_sign": ("g[:, bz, by, bx] = w[:, None] * Tb[None, :] + gf - w[:, None] * Tf[None, :]",
                       "g[:, bz, by, bx] = w[:, None] * Tb[None, :] + gf + w[:, None] * Tf[None, :]",
                       [PINS + "::test_thermal_dirichlet_identity"]),
    "outlet_fill_sign": ("v = f[j] - rho_out * un / 6.0 + C19[i] @ n * delta_n",
                         "v = f[j] + rho_out * un / 6.0 + C19[i] @ n * delta_n",
                         [PINS + "::test_zou_he_plus_z_matches_printed_formulas"]),
    "divergence_without_1_over_cs2": ("div += (W19[i] / CS2) * c[a]", "div += W19[i] * c[a]",
                                      [PINS + "::test_divergence_stencil_is_exact"]),
    "d3q7_equilibrium_moment_dropped": ("neq[4] = p.wbar * Tf", "neq[4] = 0.0 * Tf",
                                        [PINS + "::test_uniform_rest_state_is_a_fixed_point"]),
}


@pytest.fixture(scope="module")
def pristine(tmp_path_factory):
    d = tmp_path_factory.mktemp("oracle_copy")
    for sub in ("tests", "oracle", "workloads"):
        shutil.copytree(os.path.join(ROOT, sub), d / sub,
                        ignore=shutil.ignore_patterns("__pycache__", "*.pyc"))
    return d


@pytest.mark.parametrize("name", list(MISTAKES))
def test_planted_mistake_fails_a_pin(pristine, tmp_path, name):
    before, after, pins = MISTAKES[name]
    d = tmp_path / "repo"
    shutil.copytree(pristine, d)
    path = d / ORACLE
    text = path.read_text()
    assert text.count(before) == 1, f"the oracle text for {name} is not unique"
    path.write_text(text.replace(before, after))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *pins],
                       cwd=d, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"{name}: the pins passed\n{r.stdout[-2000:]}"
    assert "FAILED" in r.stdout
