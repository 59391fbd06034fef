"""GPU discrete adjoint (lbm_adjoint, through the C ABI) against the oracle's
complex-step derivatives of the evaporated mass (oracle/gradients.py).

Each case runs a few steps on a small ragged grid with two checkpoint
segments, and compares J, directional derivatives along random wall
temperature directions, single wall cells, and the wetting parameter.
"""
import sys

import numpy as np
import pytest

from oracle import gradients as Gr
from oracle import lbm_oracle as O
from tests.helpers import oracle_params
from workloads import synth

pytestmark = pytest.mark.gpu

NSTEPS = 6


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


def _case(name):
    """Small adjoint cases.  The 12 x 10 x 9 and 37 x 34 x 29 grids run the
    general kernels; the fused_* cases (64 x 16 x 12) satisfy the
    single-pass kernel's conditions (64 x 16 x 16 for the droplet between
    two outlets), so their forward steps and segment recomputations run on it and the reverse sweep derives the fields of
    every state again."""
    kappa = 0.2 if "kappa" in name else 0.0
    if name.startswith("fused_"):
        base = name[len("fused_"):]
        if base.startswith("two_outlets"):
            w = synth.droplet_open(nx=64, ny=16, nz=16, R0=4.0)
            w["faces"] = [O.PERIODIC] * 4 + [O.PRESSURE] * 2
            w["Tw"] = None
            return w
        w = synth.heated_wall(nx=64, ny=16, nz=12, R0=5.0, Tw_jitter=0.02, seed=5, kappa_w=kappa)
        if base.startswith("closed"):
            w["faces"] = list(w["faces"][:5]) + [O.WALL]
            w["face_T"] = list(w["face_T"][:5]) + [w["face_T"][4]]
        return w
    w = synth.heated_wall(nx=12, ny=10, nz=9, R0=3.5, Tw_jitter=0.02, seed=5, kappa_w=kappa)
    faces = list(w["faces"])
    face_T = list(w["face_T"])
    face_rho = list(w["face_rho"])
    if ("closed" in name):
        faces[5] = O.WALL
        face_T[5] = face_T[4]
    if name.startswith("two_outlets"):
        # a droplet between outlets at z = 0 and z = nz - 1, periodic in x and y
        w = synth.droplet_open(nx=37, ny=34, nz=29, R0=9.0)
        faces, face_T, face_rho = [O.PERIODIC] * 4 + [O.PRESSURE] * 2, list(w["face_T"]), list(w["face_rho"])
        w["Tw"] = None
    w["faces"], w["face_T"], w["face_rho"] = faces, face_T, face_rho
    return w


CASES = ["heated_wall_kappa", "heated_wall", "two_outlets", "closed_kappa",
         "fused_heated_wall_kappa", "fused_closed_kappa", "fused_two_outlets"]


def _gpu_adjoint(P, w, prec="fp64", n_checkpoints=2, nsteps=NSTEPS):
    sim = P.Lbm3D(P.params_from_workload(w, prec))
    sim.init(w["rho0"], w["T0"])
    if w.get("Tw"):
        sim.set_wall_T(4, w["Tw"][4])
    J, grad, dk = sim.adjoint(nsteps, wall_face=4, n_checkpoints=n_checkpoints)
    d = sim.reduce()
    sim.close()
    return J, grad, dk, d


def _wall_field(w):
    if w.get("Tw"):
        return w["Tw"][4]
    return np.full((w["ny"], w["nx"]), w["face_T"][4])


@pytest.mark.parametrize("name", CASES)
def test_adjoint_matches_complex_step_fp64(P, name):
    w = _case(name)
    p = oracle_params(w)
    Tw = _wall_field(w)
    _log(f"adjoint {name}: grid {w['nx']}x{w['ny']}x{w['nz']} faces {w['faces']} steps {NSTEPS}")
    J, grad, dk, d = _gpu_adjoint(P, w)
    assert d["step"] == NSTEPS
    M0 = float(np.sum(w["rho0"]))
    J_ref = Gr.evaporated_mass(w["rho0"], w["T0"], p, NSTEPS, {4: Tw})
    assert abs(J - J_ref) < 1e-12 * M0, (J, J_ref)
    rng = np.random.default_rng(105)
    dirs = [rng.uniform(-1, 1, Tw.shape) for _ in range(3)]
    for (y, x) in ((0, 0), (w["ny"] // 2, w["nx"] // 2), (w["ny"] - 1, 3)):
        e = np.zeros_like(Tw)
        e[y, x] = 1.0
        dirs.append(e)
    worst = 0.0
    for v in dirs:
        ref = Gr.directional_derivative(w["rho0"], w["T0"], p, NSTEPS, 4, Tw, v, 0.0)
        got = float(np.sum(grad * v))
        # closed box: the exact derivative is 0 and both sides give rounding
        # noise, judged against the size of an open case's derivative (~1e-2)
        scale = 1e-2 if ("closed" in name) else float(np.sum(np.abs(grad * v)))
        err = abs(got - ref) / scale
        worst = max(worst, err)
        assert err < 1e-9, (got, ref)
    ref_k = Gr.directional_derivative(w["rho0"], w["T0"], p, NSTEPS, 4, Tw, np.zeros_like(Tw), 1.0)
    if O.WALL not in w["faces"]:
        assert dk == 0.0 and ref_k == 0.0  # kappa_w acts on wall faces only
        err_k = 0.0
    else:
        err_k = abs(dk - ref_k) / (1e-2 if ("closed" in name) else abs(ref_k))
    _log(f"  J {J:.6e} (oracle {J_ref:.6e})  dJ/dTw worst {worst:.2e}  dJ/dkappa {dk:.6e} vs {ref_k:.6e} ({err_k:.2e})")
    assert err_k < 1e-9
    if ("closed" in name):
        assert abs(J) < 1e-12 * M0
        assert np.max(np.abs(grad)) < 1e-12 * M0


@pytest.mark.parametrize("name", ["heated_wall_kappa", "fused_heated_wall_kappa"])
def test_checkpoint_count_does_not_change_the_gradient(P, name):
    """On the general kernels every state of the reverse sweep is produced and
    evaluated by the same kernels whatever the segmentation: the gradient is
    bitwise independent of the checkpoint count.  On the single-pass kernel
    the recomputed states come from its field-writing instantiation and the
    checkpoints from the plain one, which agree to rounding: 1e-13."""
    w = _case(name)
    out = [_gpu_adjoint(P, w, n_checkpoints=k) for k in (1, 2, 0, NSTEPS)]
    # the same request twice: bitwise the same (deterministic)
    again = _gpu_adjoint(P, w, n_checkpoints=2)
    assert np.array_equal(again[1], out[1][1]) and again[2] == out[1][2]
    for J, grad, dk, _ in out[1:]:
        assert J == out[0][0]
        if name.startswith("fused_"):
            eg = float(np.max(np.abs(grad - out[0][1])) / np.max(np.abs(out[0][1])))
            _log(f"{name}: checkpoint counts differ by {eg:.2e} (dJ/dTw), {abs(dk - out[0][2]) / abs(dk):.2e} (kappa)")
            assert eg < 1e-13 and abs(dk - out[0][2]) < 1e-13 * abs(dk)
        else:
            assert np.array_equal(grad, out[0][1])
            assert dk == out[0][2]


# bounds on the normwise dJ/dT_w and the dJ/dkappa_w differences to FP64
# (measured on the single-pass grid: FP32 1.6e-3 and 4.9e-3)
NARROW_BOUNDS = {"fp32": 1e-2, "fp16": 2e-2, "bf16": 5e-2}


@pytest.mark.parametrize("name", ["heated_wall_kappa", "fused_heated_wall_kappa"])
@pytest.mark.parametrize("prec", list(NARROW_BOUNDS))
def test_adjoint_narrow_storage_against_fp64(P, prec, name):
    """The adjoint with FP32 (and, measured, FP16 / BF16) storage of the
    forward states against the FP64 adjoint."""
    w = _case(name)
    J64, g64, k64, _ = _gpu_adjoint(P, w, "fp64")
    J32, g32, k32, _ = _gpu_adjoint(P, w, prec)
    if name.startswith("fused_"):
        # the same storage on the general kernels, for scale
        import os
        os.environ["LBM_FUSED"] = "0"
        try:
            _, gu, ku, _ = _gpu_adjoint(P, w, prec)
        finally:
            del os.environ["LBM_FUSED"]
        _log(f"{name} {prec} adjoint on the general kernels vs fp64: dJ/dTw normwise "
             f"{float(np.max(np.abs(gu - g64)) / np.max(np.abs(g64))):.2e}, dJ/dkappa {abs(ku - k64) / abs(k64):.2e}")
    assert np.isfinite(g32).all() and np.isfinite(k32)
    eg = float(np.max(np.abs(g32 - g64)) / np.max(np.abs(g64)))
    ek = abs(k32 - k64) / abs(k64)
    _log(f"{name} {prec} adjoint vs fp64: dJ/dTw normwise {eg:.2e}, dJ/dkappa {ek:.2e}, J {abs(J32 - J64):.2e}")
    bound = NARROW_BOUNDS[prec]
    assert eg < bound and ek < bound


def test_autograd_function(P):
    import torch
    w = _case("heated_wall_kappa")
    sim = P.Lbm3D(P.params_from_workload(w, "fp64"))
    EM = P.evaporated_mass_function()
    Tw = torch.tensor(w["Tw"][4], dtype=torch.float64, requires_grad=True)
    kappa = torch.tensor(0.2, dtype=torch.float64, requires_grad=True)
    J = EM.apply(sim, w["rho0"], w["T0"], NSTEPS, 4, Tw, kappa)
    (2.0 * J).backward()
    J0, g0, k0, _ = _gpu_adjoint(P, w)
    assert float(J.detach()) == J0
    assert np.array_equal(Tw.grad.numpy(), 2.0 * g0)
    assert float(kappa.grad) == 2.0 * k0
    sim.close()


def test_adjoint_errors(P):
    w = _case("heated_wall")
    sim = P.Lbm3D(P.params_from_workload(w, "fp64"))
    with pytest.raises(P.LbmError) as e:
        sim.adjoint(3)
    assert e.value.status == 5  # before lbm_init
    sim.init(w["rho0"], w["T0"])
    with pytest.raises(P.LbmError) as e:
        sim.adjoint(0)
    assert e.value.status == 1
    sim.close()
    wp = dict(w)
    wp["faces"] = [O.PERIODIC] * 6
    sim = P.Lbm3D(P.params_from_workload(wp, "fp64"))
    sim.init(w["rho0"], w["T0"])
    with pytest.raises(P.LbmError) as e:
        sim.adjoint(3, wall_face=4)
    assert e.value.status == 1  # periodic face
    sim.close()
    wo = synth.droplet_open(nx=10, ny=9, nz=8, R0=3.0)
    sim = P.Lbm3D(P.params_from_workload(wo, "fp64"))
    sim.init(wo["rho0"], wo["T0"])
    with pytest.raises(P.LbmError) as e:
        sim.adjoint(3, wall_face=4)
    assert e.value.status == 6  # x and y must be periodic
    sim.close()


def test_full_size_adjoint_against_central_differences(P):
    """The 96^3 heated-wall case over its 2000 steps: the FP64 adjoint
    gradient against FP64 central differences of the GPU forward run, along
    4 random wall-temperature directions (seed 105), 4 single wall cells and
    kappa_w, at 1e-5 relative.  Central differences converge as h^2; the
    steps below keep the truncation error near 1e-7."""
    w = synth.named("heated_wall_adjoint_96")
    Tw0 = w["Tw"][4]
    _log("adjoint 96^3 heated wall, 2000 steps, FP64 vs central differences")
    sim = P.Lbm3D(P.params_from_workload(w, "fp64"))
    sim.init(w["rho0"], w["T0"])
    sim.set_wall_T(4, Tw0)
    J, grad, dk = sim.adjoint(w["steps"], wall_face=4)

    def J_of(Tw, kappa):
        sim.init(w["rho0"], w["T0"])
        sim.set_wall_T(4, Tw)
        sim.set_kappa(kappa)
        m0 = sim.reduce()["mass"]
        sim.step(w["steps"])
        return m0 - sim.reduce()["mass"]

    assert abs(J_of(Tw0, 0.0) - J) < 1e-12 * abs(J)
    rng = np.random.default_rng(105)
    cases = [(rng.uniform(-1, 1, Tw0.shape), 0.0, 1e-5) for _ in range(4)]
    for (y, x) in ((48, 48), (10, 70), (90, 5), (0, 0)):
        e = np.zeros_like(Tw0)
        e[y, x] = 1.0
        cases.append((e, 0.0, 2e-5))
    cases.append((np.zeros_like(Tw0), 1.0, 1e-4))
    worst = 0.0
    for v, kdir, h in cases:
        fd = (J_of(Tw0 + h * v, h * kdir) - J_of(Tw0 - h * v, -h * kdir)) / (2 * h)
        ad = float(np.sum(grad * v)) + dk * kdir
        err = abs(fd - ad) / abs(ad)
        worst = max(worst, err)
        assert err < 1e-5, (fd, ad)
    sim.close()
    _log(f"  J = {J:.6e}, dJ/dkappa = {dk:.6e}, worst relative difference to central differences {worst:.2e}")


def test_fused_forward_adjoint_equals_general_kernels(P, monkeypatch):
    """The adjoint of a case that the single-pass kernel runs, against the
    same case forced onto the general kernels (which keep the fields of each
    recomputed state): the same discrete adjoint to rounding."""
    w = _case("fused_heated_wall_kappa")
    out = []
    for flag in ("1", "0"):
        monkeypatch.setenv("LBM_FUSED", flag)
        out.append(_gpu_adjoint(P, w))
    (J1, g1, k1, _), (J0, g0, k0, _) = out
    assert abs(J1 - J0) < 1e-13 * abs(J0)
    assert np.max(np.abs(g1 - g0)) < 1e-12 * np.max(np.abs(g0))
    assert abs(k1 - k0) < 1e-12 * abs(k0)
