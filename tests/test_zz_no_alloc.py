"""lbm_adjoint_noalloc (workspace in the library's fixed device array)
against lbm_adjoint, through the C ABI: two calls in a row, the second on a
smaller request, each compared with the allocating entry point on the same
state; and a request beyond the fixed size is refused before any work."""
import sys

import numpy as np
import pytest

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


def _adjoint(P, w, prec, nsteps, noalloc):
    sim = P.Lbm3D(P.params_from_workload(w, prec))
    sim.init(w["rho0"], w["T0"])
    if w.get("Tw"):
        sim.set_wall_T(4, w["Tw"][4])
    J, grad, dk = sim.adjoint(nsteps, wall_face=4, n_checkpoints=2, noalloc=noalloc)
    d = sim.reduce()
    fields = sim.fields()
    sim.close()
    return J, grad, dk, d, fields


# (name, workload, storage, steps): each request is smaller than the one before
CALLS = [
    ("heated_wall_64x16x12 fp64, 8 steps",
     lambda: synth.heated_wall(nx=64, ny=16, nz=12, R0=5.0, Tw_jitter=0.02, seed=5, kappa_w=0.2), "fp64", 8),
    ("heated_wall_64x8x8 fp64, 5 steps",
     lambda: synth.heated_wall(nx=64, ny=8, nz=8, R0=3.0, Tw_jitter=0.02, seed=6, kappa_w=0.3), "fp64", 5),
    ("heated_wall_64x8x8 fp32, 4 steps",
     lambda: synth.heated_wall(nx=64, ny=8, nz=8, R0=3.0, Tw_jitter=0.02, seed=7, kappa_w=0.3), "fp32", 4),
]


def test_noalloc_adjoint_matches_allocating_adjoint(P):
    for name, make, prec, nsteps in CALLS:
        w = make()
        _log(f"[noalloc] {name}")
        ref = _adjoint(P, w, prec, nsteps, noalloc=False)
        got = _adjoint(P, w, prec, nsteps, noalloc=True)
        J0, g0, k0, d0, f0 = ref
        J1, g1, k1, d1, f1 = got
        assert np.isfinite(g1).all()
        assert abs(J1 - J0) <= 1e-12 * abs(J0), (J1, J0)
        assert np.max(np.abs(g1 - g0)) <= 1e-12 * np.max(np.abs(g0))
        assert abs(k1 - k0) <= 1e-12 * abs(k0)
        assert d1["step"] == d0["step"] == nsteps
        for a, b in zip(f0, f1):
            assert np.array_equal(a, b)
        _log(f"  J {J1:.6e} dJ/dkappa {k1:.6e}: equal to lbm_adjoint")


def test_noalloc_adjoint_refuses_requests_beyond_its_array(P):
    """A request whose workspace exceeds the fixed 64 MiB returns LBM_ENOMEM
    and leaves the state at t0."""
    w = synth.heated_wall(nx=64, ny=64, nz=64, R0=10.0, Tw_jitter=0.02, seed=5)
    sim = P.Lbm3D(P.params_from_workload(w, "fp64"))
    sim.init(w["rho0"], w["T0"])
    sim.set_wall_T(4, w["Tw"][4])
    assert sim.adjoint_bytes(50, wall_face=4) > 64 << 20
    with pytest.raises(P.LbmError) as e:
        sim.adjoint(50, wall_face=4, noalloc=True)
    assert e.value.status == 2
    assert sim.reduce()["step"] == 0
    sim.close()
