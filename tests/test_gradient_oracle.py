"""Pins of the gradient oracle (oracle/gradients.py) against the plain
definition of the derivative and against facts of the method.

* The complex-step derivative agrees with central differences of the real
  oracle, and the difference falls as h^2 (the truncation order of central
  differences), so both compute the same derivative.
* Derivatives are linear in the direction.
* In a box closed by two walls the mass is conserved exactly (bounce-back,
  eq. (34)), so the evaporated mass is 0 for every wall temperature and its
  derivative vanishes.
"""
import numpy as np
import pytest

from oracle import gradients as Gr
from oracle import lbm_oracle as O
from tests.helpers import oracle_params
from workloads import synth


def _case(kappa=0.2, top=O.PRESSURE):
    w = synth.heated_wall(nx=10, ny=8, nz=9, R0=3.5, Tw_jitter=0.02, seed=5, kappa_w=kappa)
    faces = list(w["faces"])
    faces[5] = top
    w["faces"] = faces
    return w, oracle_params(w)


def test_complex_step_matches_central_differences():
    w, p = _case()
    Tw = w["Tw"][4]
    v = np.random.default_rng(3).uniform(-1, 1, Tw.shape)
    exact = Gr.directional_derivative(w["rho0"], w["T0"], p, 5, 4, Tw, v, 0.0)
    errs = []
    for h in (1e-3, 1e-4):
        fd = Gr.central_difference(w["rho0"], w["T0"], p, 5, 4, Tw, v, 0.0, h)
        errs.append(abs(fd - exact) / abs(exact))
    assert errs[1] < 1e-5
    # O(h^2): ten times smaller h, a hundred times smaller error
    assert 30 < errs[0] / errs[1] < 300, errs


def test_complex_step_kappa_matches_central_differences():
    w, p = _case()
    Tw = w["Tw"][4]
    z = np.zeros_like(Tw)
    exact = Gr.directional_derivative(w["rho0"], w["T0"], p, 5, 4, Tw, z, 1.0)
    fd = Gr.central_difference(w["rho0"], w["T0"], p, 5, 4, Tw, z, 1.0, 1e-4)
    assert exact != 0.0
    assert abs(fd - exact) < 1e-6 * abs(exact)


def test_directional_derivative_is_linear():
    w, p = _case()
    Tw = w["Tw"][4]
    rng = np.random.default_rng(4)
    v1, v2 = rng.uniform(-1, 1, Tw.shape), rng.uniform(-1, 1, Tw.shape)
    d = lambda v, k: Gr.directional_derivative(w["rho0"], w["T0"], p, 4, 4, Tw, v, k)
    a, b, ab = d(v1, 0.3), d(v2, -0.7), d(v1 + v2, -0.4)
    assert abs(ab - (a + b)) < 1e-10 * (abs(a) + abs(b))


def test_closed_box_evaporates_nothing():
    w, p = _case(top=O.WALL)
    w["face_T"] = list(w["face_T"])
    w["face_T"][5] = w["face_T"][4]
    p = oracle_params(w)
    Tw = w["Tw"][4]
    v = np.random.default_rng(5).uniform(-1, 1, Tw.shape)
    J = Gr.evaporated_mass(w["rho0"], w["T0"], p, 5, w["Tw"])
    M = float(np.sum(w["rho0"]))
    assert abs(J) < 1e-13 * M
    d = Gr.directional_derivative(w["rho0"], w["T0"], p, 5, 4, Tw, v, 1.0)
    assert abs(d) < 1e-13 * M
