"""Edge cases through the C ABI against the oracle (FP64, 1e-12): smallest
grids of every boundary kind (single-cell periodic axes, bounded axes of 3
cells, the fused kernel's smallest z extent), plus context handling: two
interleaved contexts, a library-allocated context and a non-default stream
give bitwise the same results as one context on the default stream."""
import sys

import numpy as np
import pytest

from tests.helpers import oracle_run, rel_err_scalar
from workloads import synth

pytestmark = pytest.mark.gpu

P_, W_, O_ = 0, 1, 2   # periodic, wall, pressure


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


def noisy_uniform(nx, ny, nz, faces, seed=11, kappa_w=0.0):
    """Vapour at T_sat with +-1e-3 relative noise on rho and T (stays physical)."""
    w = synth._base("noisy_uniform", nx, ny, nz, faces, 8, 0.86)
    n = nx * ny * nz
    w["rho0"] = (w["rho_v"] * (1 + 1e-3 * synth.uniform_pm1(seed, n))).reshape(nz, ny, nx)
    w["T0"] = (w["T_ref"] * (1 + 1e-3 * synth.uniform_pm1(seed + 1, n))).reshape(nz, ny, nx)
    w["face_T"] = [w["T_ref"] * 1.02 if f != P_ else 0.0 for f in faces]
    w["face_rho"] = [w["rho_v"] if f == O_ else 0.0 for f in faces]
    w["kappa_w"] = kappa_w
    return w


EDGE = {
    "column_1x1x16_periodic": (1, 1, 16, [P_] * 6),
    "cube_3x3x3_all_outlets": (3, 3, 3, [O_] * 6),
    "box_4x5x3_z_walls": (4, 5, 3, [P_] * 4 + [W_] * 2),
    "box_5x3x7_xy_outlets": (5, 3, 7, [O_] * 4 + [P_] * 2),
    "box_3x4x5_x_outlets": (3, 4, 5, [O_] * 2 + [P_] * 4),
    "fused_64x8x4_z_walls": (64, 8, 4, [P_] * 4 + [W_] * 2),
    "fused_64x8x4_periodic": (64, 8, 4, [P_] * 6),
    "wall_outlet_7x6x3": (7, 6, 3, [P_] * 4 + [W_, O_]),
}


@pytest.mark.parametrize("name", list(EDGE))
def test_edge_shapes_fp64(P, name):
    nx, ny, nz, faces = EDGE[name]
    w = noisy_uniform(nx, ny, nz, faces, kappa_w=0.2 if W_ in faces else 0.0)
    steps = 8
    ref = oracle_run(w, steps, record=(1, steps))
    sim = P.from_workload(w, precision="fp64")
    for s in (1, steps):
        sim.step(s - (1 if s == steps else 0))
        rho, u, T = sim.fields()
        er, eT = rel_err_scalar(rho, ref[s][0]), rel_err_scalar(T, ref[s][2])
        # velocities here are noise-driven (|u| ~ 1e-6 .. 1e-4), so u is
        # judged in absolute terms: rounding of j = sum c_i f_i is ~1e-16
        du = float(np.max(np.abs(u - ref[s][1])))
        umax = float(np.max(np.abs(ref[s][1])))
        _log(f"{name} step {s}: rho {er:.2e} T {eT:.2e} |du| {du:.2e} (max |u| {umax:.1e})")
        assert er < 1e-12 and eT < 1e-12 and du < 2e-15 + 1e-11 * umax
    sim.close()


def _run(P, w, steps=12, **kw):
    sim = P.Lbm3D(P.params_from_workload(w, "fp32"), **kw)
    sim.init(w["rho0"], w["T0"])
    sim.step(steps)
    out = sim.fields()
    sim.close()
    return out


def test_contexts_are_independent(P):
    wa = synth.droplet_periodic(n=24, R0=6.0, noise=1e-6, seed=3)
    wb = synth.blobs_closed(nx=64, ny=16, nz=20, mean_blobs=2, rmin=4.0, rmax=6.0, seed=7)
    ra, rb = _run(P, wa), _run(P, wb)
    # interleaved
    sa = P.Lbm3D(P.params_from_workload(wa, "fp32"))
    sb = P.Lbm3D(P.params_from_workload(wb, "fp32"))
    sa.init(wa["rho0"], wa["T0"])
    sb.init(wb["rho0"], wb["T0"])
    for _ in range(4):
        sa.step(3)
        sb.step(3)
    ia, ib = sa.fields(), sb.fields()
    sa.close()
    sb.close()
    for x, y in zip(ra + rb, ia + ib):
        assert np.array_equal(x, y)


def test_library_allocated_context_and_side_stream(P):
    import torch
    w = synth.droplet_periodic(n=24, R0=6.0, noise=1e-6, seed=3)
    ref = _run(P, w)
    own = _run(P, w, torch_buffer=False)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        on_side = _run(P, w)
    for x, y, z in zip(ref, own, on_side):
        assert np.array_equal(x, y) and np.array_equal(x, z)
