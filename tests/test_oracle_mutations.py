"""The transport pins against plausible misreadings of the paper, planted in
a temporary copy of the oracle (CPU only; the repository's oracle is not
touched).  Each misreading must make at least one pin of
tests/test_oracle_pins_transport.py fail:

  the bulk and shear rates of eq. (11) swapped, s_q set to s_nu, s_pi halved
  (the Sec. 4 relaxation values); the convective term of eq. (15) or the
  divergence built from u_eq instead of the real velocity of eq. (5); the
  sign of either source term flipped; the wall-node velocity of Sec. 3.1
  read as u_eq = 0, or not prescribed at all; the ghost velocity beyond a
  wall copied from the first interior layer instead of 0.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join("oracle", "lbm_oracle.py")

# name: (text in the oracle, misreading written in its place)
MISREADINGS = {
    "bulk_and_shear_rates_swapped": ("[1.0, 1.0, 1.0, 1.0, self.s_e] + [self.s_nu] * 5",
                                     "[1.0, 1.0, 1.0, 1.0, self.s_nu] + [self.s_e] * 5"),
    "s_q_equal_to_s_nu": ("[self.s_q] * 6", "[self.s_nu] * 6"),
    "s_pi_halved": ("[self.s_pi] * 3", "[0.5 * self.s_pi] * 3"),
    "convection_with_u_eq": ("np.sum(u * gradT, axis=0)", "np.sum(ueq * gradT, axis=0)"),
    "divergence_of_u_eq": ("div_u = divergence(u, p)", "div_u = divergence(ueq, p)"),
    "compression_sign": ("+ T * dpdT * div_u", "- T * dpdT * div_u"),
    "convection_sign": ("Fbar = rho * p.cv * np.sum", "Fbar = -rho * p.cv * np.sum"),
    "wall_node_u_eq_zero": ("ueq = np.where(wall, -0.5 * du, ueq)", "ueq = np.where(wall, 0.0, ueq)"),
    "wall_node_not_prescribed": ("    if wall.any():", "    if False:"),
    "ghost_u_copied_inward": ("lambda w, i: np.zeros_like(w))", "lambda w, i: i)"),
}


@pytest.fixture(scope="module")
def pristine(tmp_path_factory):
    d = tmp_path_factory.mktemp("oracle_copy")
    for sub in ("tests", "oracle", "workloads"):
        shutil.copytree(os.path.join(ROOT, sub), d / sub,
                        ignore=shutil.ignore_patterns("__pycache__", "*.pyc"))
    return d


@pytest.mark.parametrize("name", list(MISREADINGS))
def test_misreading_fails_a_transport_pin(pristine, tmp_path, name):
    before, after = MISREADINGS[name]
    d = tmp_path / "repo"
    shutil.copytree(pristine, d)
    path = d / ORACLE
    text = path.read_text()
    assert text.count(before) == 1, f"the oracle text for {name} is not unique"
    path.write_text(text.replace(before, after))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join("tests", "test_oracle_pins_transport.py")],
                       cwd=d, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"{name}: every transport pin passed\n{r.stdout[-2000:]}"
    assert "FAILED" in r.stdout
