"""FP64 CPU oracle of the evaporated-mass objective and its derivatives.

TEST INFRASTRUCTURE ONLY (same rules as ``oracle/lbm_oracle.py``: imported by
the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` only).

Objective: the evaporated mass J = M(0) - M(N), M(t) = sum over all cells of
rho at time t (rho_out on outlet nodes, Sec. 3.3), the quantity behind the
d^2 law of Sec. 4.2, eq. (56).  Parameters: the wall temperature field T_w of
one bounded z face (eqs. (35)-(36)) and the wetting parameter kappa_w of
eq. (37).

Derivatives are taken by their definitions, with no adjoint code:
  * ``directional_derivative``: complex-step differentiation (Squire and
    Trapp, SIAM Review 40, 1998; Martins, Sturdza and Alonso, ACM TOMS 29,
    2003): for an analytic J, dJ/dtheta . v = Im J(theta + i h v) / h + O(h^2)
    with no subtractive cancellation, so h = 1e-30 gives the derivative to
    rounding.  The forward oracle runs unchanged on complex arrays.
  * ``central_difference``: (J(theta + h v) - J(theta - h v)) / (2 h), the
    plain definition, with truncation error O(h^2).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Optional

import numpy as np

from . import lbm_oracle as O


def total_mass(f, g, p: O.Params, Tw=None):
    """M = sum of rho after S0-S1 (eq. (3); rho_out on outlet nodes)."""
    return np.sum(O.macroscopic(f, g, p, Tw)["rho"])


def evaporated_mass(rho0, T0, p: O.Params, nsteps: int, Tw: Optional[Dict[int, np.ndarray]] = None):
    """J = M(0) - M(N) from the initial state f = f^eq(rho0, 0), g = w T0."""
    f, g = O.init_populations(rho0, T0, p)
    m0 = total_mass(f, g, p, Tw)
    f, g = O.run(f, g, p, nsteps, Tw)
    return m0 - total_mass(f, g, p, Tw)


def _perturbed(p: O.Params, face: int, Tw_field, dTw, dkappa, h):
    q = dataclasses.replace(p, kappa_w=p.kappa_w + h * dkappa)
    field = np.asarray(Tw_field) + h * np.asarray(dTw)
    return q, {face: field}


def directional_derivative(rho0, T0, p: O.Params, nsteps: int, face: int, Tw_field, dTw, dkappa: float,
                           h: float = 1e-30) -> float:
    """dJ/dT_w . dTw + dJ/dkappa_w * dkappa by the complex step."""
    q, Tw = _perturbed(p, face, np.asarray(Tw_field, dtype=np.complex128), dTw, dkappa, 1j * h)
    return float(np.imag(evaporated_mass(rho0, T0, q, nsteps, Tw)) / h)


def central_difference(rho0, T0, p: O.Params, nsteps: int, face: int, Tw_field, dTw, dkappa: float,
                       h: float) -> float:
    """The same directional derivative by central differences with step h."""
    qp, Twp = _perturbed(p, face, Tw_field, dTw, dkappa, h)
    qm, Twm = _perturbed(p, face, Tw_field, dTw, dkappa, -h)
    return float((evaporated_mass(rho0, T0, qp, nsteps, Twp) - evaporated_mass(rho0, T0, qm, nsteps, Twm))
                 / (2.0 * h))
