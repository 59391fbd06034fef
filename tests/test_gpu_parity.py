"""GPU (HIP library, through the C ABI) against the FP64 oracle.

FP64 storage must agree with the oracle to 1e-12 (max relative error for rho
and T, normwise for u).  FP32 deviation storage must keep density within
1e-4.  FP16/BF16 storage errors are measured and bounded loosely.
"""
import functools
import sys

import numpy as np
import pytest

from oracle import lbm_oracle as O
from tests.helpers import oracle_params, oracle_run, rel_err_scalar, rel_err_vector, sub_block
from workloads import synth

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


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


def _small_workloads():
    return {
        "droplet_periodic_32": synth.droplet_periodic(n=32, R0=8.0, W=5.0, noise=1e-6, seed=1),
        "droplet_open_37x34x29": synth.droplet_open(nx=37, ny=34, nz=29, R0=9.0),
        "heated_wall_35x31x27": synth.heated_wall(nx=35, ny=31, nz=27, R0=10.0, Tw_jitter=0.02, seed=5,
                                                  kappa_w=0.3),
        "blobs_closed_40x36x30": synth.blobs_closed(nx=40, ny=36, nz=30, mean_blobs=3, rmin=5.0, rmax=9.0),
        # conductivity linear in rho between the phases (Sec. 4.1 values)
        "heat_transfer_6x5x40": synth.saturated_heat_transfer(nx=6, ny=5, nz=40),
    }


SMALL = _small_workloads()


def _compare(name, got, ref, tol_r, tol_u, tol_T):
    er = rel_err_scalar(got[0], ref[0])
    eu = rel_err_vector(got[1], ref[1])
    eT = rel_err_scalar(got[2], ref[2])
    _log(f"{name}: rho {er:.3e}  u {eu:.3e}  T {eT:.3e}")
    assert er < tol_r and eu < tol_u and eT < tol_T, (er, eu, eT)


@pytest.mark.parametrize("name", list(SMALL))
def test_fp64_parity_small(P, name):
    w = SMALL[name]
    steps = 500 if name.startswith("droplet_periodic") else 60
    record = (0, 1, 10, steps) if steps > 10 else (0, 1, steps)
    _log(f"[fp64 parity] {name} steps={steps}")
    ref = oracle_run(w, steps, record=record)
    sim = P.from_workload(w, precision="fp64")
    done = 0
    for s in sorted(ref):
        sim.step(s - done)
        done = s
        _compare(f"{name} step {s}", sim.fields(), ref[s], TOL64, TOL64, TOL64)
    sim.close()


@pytest.mark.parametrize("name", list(SMALL))
def test_fp32_deviation_parity_small(P, name):
    w = SMALL[name]
    steps = 200 if name.startswith("droplet_periodic") else 60
    _log(f"[fp32 parity] {name} steps={steps}")
    ref = oracle_run(w, steps, record=(1, steps))
    sim = P.from_workload(w, precision="fp32")
    sim.step(1)
    _compare(f"{name} fp32 step 1", sim.fields(), ref[1], 1e-5, 1e-5, 1e-5)
    sim.step(steps - 1)
    _compare(f"{name} fp32 step {steps}", sim.fields(), ref[steps], 1e-4, 2e-4, 1e-4)
    sim.close()


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_half_storage_measured(P, prec):
    """Narrow storage: finite and within a loose bound after 20 steps; the
    measured errors are printed."""
    w = SMALL["droplet_periodic_32"]
    ref = oracle_run(w, 20, record=(20,))
    sim = P.from_workload(w, precision=prec)
    sim.step(20)
    rho, u, T = sim.fields()
    assert np.isfinite(rho).all() and np.isfinite(T).all()
    er = rel_err_scalar(rho, ref[20][0])
    eT = rel_err_scalar(T, ref[20][2])
    _log(f"{prec}: rho {er:.3e} T {eT:.3e}")
    assert er < (0.02 if prec == "fp16" else 0.1) and eT < (0.02 if prec == "fp16" else 0.1)
    sim.close()


def test_zero_steps_and_initial_fields(P):
    w = SMALL["droplet_open_37x34x29"]
    ref = oracle_run(w, 0, record=(0,))
    sim = P.from_workload(w, precision="fp64")
    sim.step(0)
    _compare("step 0", sim.fields(), ref[0], TOL64, TOL64, TOL64)
    rho_d, u_d, T_d = sim.fields_device()
    assert np.array_equal(rho_d.cpu().numpy(), sim.fields()[0])
    sim.close()


def test_reductions_fp64(P):
    """FP64 mass, energy and liquid-volume reductions against the oracle."""
    w = SMALL["heated_wall_35x31x27"]
    ref = oracle_run(w, 30, record=(0, 30))
    p = oracle_params(w)
    sim = P.from_workload(w, precision="fp64")
    d0 = sim.reduce()
    sim.step(30)
    d = sim.reduce()
    r0 = O.diagnostics(ref[0][0], ref[0][2], p, w["rho_v"], w["rho_l"])
    r = O.diagnostics(ref[30][0], ref[30][2], p, w["rho_v"], w["rho_l"])
    for k in ("mass", "energy", "vol_smooth"):
        assert abs(d0[k] - r0[k]) <= 1e-12 * abs(r0[k]), k
        assert abs(d[k] - r[k]) <= 1e-12 * abs(r[k]), k
    assert d["vol_hard"] == r["vol_hard"]
    assert abs(d["evap_mass"] - (r0["mass"] - r["mass"])) < 1e-9 * r0["mass"]
    assert d["step"] == 30
    sim.close()


def test_determinism_bitwise(P):
    w = SMALL["blobs_closed_40x36x30"]
    outs = []
    for _ in range(2):
        sim = P.from_workload(w, precision="fp32")
        sim.step(25)
        outs.append(sim.fields())
        outs[-1] = outs[-1] + (sim.reduce()["mass"],)
        sim.close()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(np.asarray(a), np.asarray(b))


def test_closed_box_mass_conservation_fp64(P):
    """No-slip walls on both z faces conserve mass (bounce-back)."""
    w = SMALL["blobs_closed_40x36x30"]
    sim = P.from_workload(w, precision="fp64")
    m0 = sim.reduce()["mass"]
    sim.step(50)
    m1 = sim.reduce()["mass"]
    assert abs(m1 - m0) / m0 < 1e-13


def test_error_paths(P):
    import ctypes
    p = P.make_params(8, 8, 8, precision="fp64")
    sim = P.Lbm3D(p)
    with pytest.raises(P.LbmError) as e:
        sim.step(1)
    assert e.value.status == 5            # LBM_ESTATE
    bad = P.make_params(8, 8, 8, faces=(0, 2, 0, 0, 0, 0))
    with pytest.raises(P.LbmError) as e:
        P.Lbm3D(bad)
    assert e.value.status == 1            # LBM_EINVAL
    unsup = P.make_params(8, 8, 8, faces=(1, 1, 0, 0, 0, 0), face_T=(0.1,) * 6)
    with pytest.raises(P.LbmError) as e:
        P.Lbm3D(unsup)
    assert e.value.status == 6            # LBM_EUNSUPPORTED
    # a density beyond the psi^2 > 0 range at 0.86 Tc (both sides flag it)
    w = synth.droplet_periodic(n=8, R0=2.0, noise=0.0)
    w["rho0"][4, 4, 4] = 9.5
    po = oracle_params(w)
    f, g = O.init_populations(w["rho0"], w["T0"], po)
    assert O.macroscopic(f, g, po)["bad"].any()
    sim = P.from_workload(w, precision="fp64")
    with pytest.raises(P.LbmError) as e:
        sim.step(1)
    assert e.value.status == 4            # LBM_ENONPHYS
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("setup", ["periodic", "wall_outlet"])
def test_nonphysical_state_on_the_single_pass_kernel(P, prec, setup):
    """A density beyond the psi^2 > 0 range is reported (LBM_ENONPHYS) by the
    single-pass kernel too, for closed and outlet z faces."""
    if setup == "periodic":
        w = synth.droplet_periodic(nx=64, ny=8, nz=8, R0=2.0, noise=0.0)
    else:
        w = synth.heated_wall(nx=64, ny=8, nz=8, R0=3.0)
    w["rho0"][4, 4, 30] = 9.5
    po = oracle_params(w)
    f, g = O.init_populations(w["rho0"], w["T0"], po)
    assert O.macroscopic(f, g, po)["bad"].any()
    sim = P.from_workload(w, precision=prec)
    with pytest.raises(P.LbmError) as e:
        sim.step(1)
    assert e.value.status == 4            # LBM_ENONPHYS
    sim.close()


# ---------------------------------------------------------------- full sizes

FULL = ["droplet_open_128", "heated_wall_256", "heated_wall_adjoint_96", "blobs_closed_512x512x384"]


@functools.lru_cache(maxsize=1)
def _full_workload(name):
    return synth.named(name)


def _sample_points(w, rng, n_random=6):
    nx, ny, nz = w["nx"], w["ny"], w["nz"]
    pts = [(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))) for _ in range(n_random)]
    pts += [(0, 0, 0), (nx - 1, ny // 2, nz - 1), (nx // 2, ny - 1, 0), (nx // 3, 1, nz // 2),
            (nx // 2, ny // 2, 1), (nx - 2, ny - 2, nz - 2)]
    # a few cells on the liquid-vapour interface
    rho = w["rho0"]
    mid = 0.5 * (w["rho_v"] + w["rho_l"])
    zz, yy, xx = np.nonzero(np.abs(rho - mid) < 0.25 * (w["rho_l"] - w["rho_v"]))
    if len(zz):
        for k in rng.choice(len(zz), size=min(4, len(zz)), replace=False):
            pts.append((int(xx[k]), int(yy[k]), int(zz[k])))
    return pts


@pytest.mark.parametrize("name", FULL)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_size_multi_step(P, name, prec):
    """Full-size workloads in the launch configuration the bench times, 5
    steps on the GPU, compared at sampled cells with the oracle run for 5
    steps on the surrounding 65^3 block: a cell 31 or more cells from every
    cut side of the block evolves exactly as in the full domain (one step
    reaches 6 cells, the wetting ghost one more).  The block's cut sides are
    artificial and may leave the physical range; the compared cells never
    see them within the 5 steps."""
    k = 5
    _log(f"[full size x{k}] {name} {prec}: generating")
    w = _full_workload(name)
    rng = np.random.default_rng(11)
    pts = _sample_points(w, rng, n_random=3)[:10]
    _log(f"[full size x{k}] {name} {prec}: GPU steps")
    sim = P.from_workload(w, precision=prec)
    sim.step(k)
    rho, u, T = sim.fields()
    sim.close()
    del sim
    tol_r, tol_u, tol_T = (TOL64, 1e-13, TOL64) if prec == "fp64" else (2e-5, 1e-5, 2e-5)
    worst = np.zeros(3)
    for (x, y, z) in pts:
        b = sub_block(w, (x, y, z), half=6 * k + 2, margin=6 * k + 1)
        with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
            ref = oracle_run(b, k, record=(k,), check=False)[k]
        lx, ly, lz = b["local"]
        for a in range(3):
            assert b["valid"][a][0] <= b["local"][a] < b["valid"][a][1]
        er = abs(rho[z, y, x] - ref[0][lz, ly, lx]) / abs(ref[0][lz, ly, lx])
        eT = abs(T[z, y, x] - ref[2][lz, ly, lx]) / abs(ref[2][lz, ly, lx])
        eu = np.abs(u[:, z, y, x] - ref[1][:, lz, ly, lx]).max()
        worst = np.maximum(worst, (er, eu, eT))
        assert er < tol_r and eT < tol_T and eu < tol_u, ((x, y, z), er, eu, eT)
    _log(f"[full size x{k}] {name} {prec}: {len(pts)} cells ok; worst rho {worst[0]:.2e} u {worst[1]:.2e} "
         f"T {worst[2]:.2e}")


@pytest.mark.parametrize("name", FULL)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_size_sampled(P, name, prec):
    """Full-size workloads, the launch configuration the bench times: one step
    on the GPU, compared at sampled cells with the oracle run on the
    surrounding block (exact for cells far enough from the block's cut
    sides)."""
    _log(f"[full size] {name} {prec}: generating")
    w = _full_workload(name)
    rng = np.random.default_rng(7)
    pts = _sample_points(w, rng)
    _log(f"[full size] {name} {prec}: GPU step")
    sim = P.from_workload(w, precision=prec)
    sim.step(1)
    rho, u, T = sim.fields()
    sim.close()
    del sim
    # u is compared in absolute terms: |u| <= 0.1 everywhere, and a block far
    # from any interface has no meaningful local scale
    tol_r, tol_u, tol_T = (TOL64, 1e-13, TOL64) if prec == "fp64" else (1e-5, 2e-6, 1e-5)
    for (x, y, z) in pts:
        b = sub_block(w, (x, y, z), half=9, margin=7)
        ref = oracle_run(b, 1, record=(1,))[1]
        lx, ly, lz = b["local"]
        for a in range(3):
            assert b["valid"][a][0] <= b["local"][a] < b["valid"][a][1]
        er = abs(rho[z, y, x] - ref[0][lz, ly, lx]) / abs(ref[0][lz, ly, lx])
        eT = abs(T[z, y, x] - ref[2][lz, ly, lx]) / abs(ref[2][lz, ly, lx])
        eu = np.abs(u[:, z, y, x] - ref[1][:, lz, ly, lx]).max()
        assert er < tol_r and eT < tol_T and eu < tol_u, ((x, y, z), er, eu, eT)
    _log(f"[full size] {name} {prec}: {len(pts)} cells ok")


# the largest direction planes the single-pass kernel takes (its buffer
# offsets are 32-bit: 19 planes of one level below 0xF0000000 bytes)
LIMIT = {"fp64": (5184, 5104), "fp32": (7296, 7256)}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_largest_single_pass_planes(P, prec):
    """A periodic 4-plane grid whose 19 direction planes of one level span
    just under the single-pass kernel's 32-bit offset limit (4.02 of 4.03 GB;
    one row more runs the general kernels, `test_fused_support.py`): two
    steps in one call (FP64: x-deferred between them), compared at sampled
    cells with the oracle run on the surrounding blocks."""
    nx, ny = LIMIT[prec]
    es = 8 if prec == "fp64" else 4
    assert 19 * (nx * ny + 64) * es < 0xF0000000 <= 19 * (nx * (ny + 8) + 64) * es
    k = 2
    _log(f"[offset limit] {nx}x{ny}x4 {prec}: generating")
    w = synth.droplet_periodic(nx=nx, ny=ny, nz=4, R0=300.0, W=5.0, noise=0.0,
                               center=(nx / 2, ny / 2, 2.0))
    rng = np.random.default_rng(13)
    pts = [(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(4))) for _ in range(4)]
    pts += [(0, 0, 0), (nx - 1, ny - 1, 3), (nx - 1, 0, 1), (0, ny - 1, 2)]
    pts += [(nx // 2 + 300, ny // 2, 1), (nx // 2, ny // 2 - 300, 2)]  # on the interface
    _log(f"[offset limit] {nx}x{ny}x4 {prec}: GPU steps")
    sim = P.from_workload(w, precision=prec)
    sim.step(k)
    rho, u, T = sim.fields()
    sim.close()
    del sim
    tol_r, tol_u, tol_T = (TOL64, 1e-13, TOL64) if prec == "fp64" else (1e-5, 2e-6, 1e-5)
    for (x, y, z) in pts:
        b = sub_block(w, (x, y, z), half=6 * k + 4, margin=6 * k + 1)
        ref = oracle_run(b, k, record=(k,))[k]
        lx, ly, lz = b["local"]
        er = abs(rho[z, y, x] - ref[0][lz, ly, lx]) / abs(ref[0][lz, ly, lx])
        eT = abs(T[z, y, x] - ref[2][lz, ly, lx]) / abs(ref[2][lz, ly, lx])
        eu = np.abs(u[:, z, y, x] - ref[1][:, lz, ly, lx]).max()
        assert er < tol_r and eT < tol_T and eu < tol_u, ((x, y, z), er, eu, eT)
    _log(f"[offset limit] {nx}x{ny}x4 {prec}: {len(pts)} cells ok")


# ---------------------------------------------------------------- fused single-pass kernel

def _closed(w):
    """A heated-wall workload with its outlet replaced by a second wall."""
    w = dict(w)
    w["faces"] = list(w["faces"][:5]) + [1]
    w["face_T"] = list(w["face_T"][:5]) + [w["face_T"][4]]
    return w


def _flip_z(w):
    """The same set-up mirrored in z (faces, face values, wall field, fields)."""
    w = dict(w)
    w["faces"] = list(w["faces"][:4]) + [w["faces"][5], w["faces"][4]]
    w["face_T"] = list(w["face_T"][:4]) + [w["face_T"][5], w["face_T"][4]]
    w["face_rho"] = list(w["face_rho"][:4]) + [w["face_rho"][5], w["face_rho"][4]]
    w["Tw"] = {9 - k: v for k, v in (w.get("Tw") or {}).items()}
    w["rho0"] = np.ascontiguousarray(w["rho0"][::-1])
    w["T0"] = np.ascontiguousarray(w["T0"][::-1])
    return w


def _open_z(w):
    """An open-box workload with its x and y faces made periodic."""
    w = dict(w)
    w["faces"] = [synth.PERIODIC] * 4 + list(w["faces"][4:])
    return w


FUSED = {
    "droplet_periodic_128x16x24": lambda: synth.droplet_periodic(nx=128, ny=16, nz=24, R0=6.0, W=5.0,
                                                                 noise=1e-6, seed=2, center=(70, 8, 12)),
    "blobs_closed_64x32x40": lambda: synth.blobs_closed(nx=64, ny=32, nz=40, mean_blobs=3, rmin=5.0,
                                                        rmax=8.0, seed=9),
    "heat_transfer_64x16x40": lambda: synth.saturated_heat_transfer(nx=64, ny=16, nz=40),
    # wetting ghost layer with kappa_w != 0 on both walls
    "wetting_64x16x24": lambda: _closed(synth.heated_wall(nx=64, ny=16, nz=24, R0=6.0, Tw_jitter=0.02, seed=5,
                                                          kappa_w=0.3)),
    # constant-pressure outlets (Sec. 3.3) on z faces: wall below / outlet
    # above with wetting and a wall temperature field, the mirror image, and
    # outlets on both z faces
    "heated_wall_64x16x24": lambda: synth.heated_wall(nx=64, ny=16, nz=24, R0=6.0, Tw_jitter=0.02, seed=5,
                                                      kappa_w=0.2),
    "outlet_below_64x16x24": lambda: _flip_z(synth.heated_wall(nx=64, ny=16, nz=24, R0=6.0, Tw_jitter=0.02,
                                                               seed=6, kappa_w=0.2)),
    "open_z_64x16x32": lambda: _open_z(synth.droplet_open(nx=64, ny=16, nz=32, R0=6.0)),
    # ragged nx: a last tile column with 32, 36 and 40 active cells (and one
    # below the tile width), idle lanes holding the periodic continuation
    "droplet_periodic_96x16x24": lambda: synth.droplet_periodic(nx=96, ny=16, nz=24, R0=6.0, W=5.0, noise=1e-6,
                                                                seed=3, center=(80, 8, 12)),
    "heated_wall_100x16x20": lambda: synth.heated_wall(nx=100, ny=16, nz=20, R0=6.0, Tw_jitter=0.02, seed=7,
                                                       kappa_w=0.2),
    "blobs_closed_40x16x24": lambda: synth.blobs_closed(nx=40, ny=16, nz=24, mean_blobs=2, rmin=4.0, rmax=6.0,
                                                        seed=9),
    "heated_wall_8x8x12": lambda: synth.heated_wall(nx=8, ny=8, nz=12, R0=2.5, Tw_jitter=0.02, seed=8,
                                                    kappa_w=0.3),
}


@pytest.mark.parametrize("chunk", ["", "5"])
@pytest.mark.parametrize("name", list(FUSED))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fused_parity(P, name, prec, chunk, monkeypatch):
    """The single-pass kernel (default for these shapes) against the oracle,
    with the z range in one piece and cut into 5-plane chunks."""
    monkeypatch.setenv("LBM_FUSED_CHUNK", chunk or "0")
    if not chunk:
        monkeypatch.delenv("LBM_FUSED_CHUNK")
    w = FUSED[name]()
    steps = 40
    _log(f"[fused] {name} {prec} chunk={chunk or 'all'}")
    ref = oracle_run(w, steps, record=(1, steps))
    sim = P.from_workload(w, precision=prec)
    tol = (TOL64, TOL64, TOL64) if prec == "fp64" else (1e-5, 1e-5, 1e-5)
    sim.step(1)
    _compare(f"{name} {prec} step 1", sim.fields(), ref[1], *tol)
    sim.step(steps - 1)
    tol = (TOL64, TOL64, TOL64) if prec == "fp64" else (1e-4, 2e-4, 1e-4)
    _compare(f"{name} {prec} step {steps}", sim.fields(), ref[steps], *tol)
    sim.close()


@pytest.mark.parametrize("name", list(FUSED))
def test_fused_fp32_tile_height_16(P, name, monkeypatch):
    """32-bit storage with the optional 16-row tile (the 8-row tile is the default)."""
    monkeypatch.setenv("LBM_FUSED_TY", "16")
    w = FUSED[name]()
    ref = oracle_run(w, 20, record=(20,))
    sim = P.from_workload(w, precision="fp32")
    sim.step(20)
    _compare(f"{name} fp32 ty=16 step 20", sim.fields(), ref[20], 1e-4, 2e-4, 1e-4)
    sim.close()


@pytest.mark.parametrize("ty", ["8", "16"])
@pytest.mark.parametrize("name", list(FUSED))
def test_fused_half_storage(P, name, ty, monkeypatch):
    """FP16 and BF16 deviation storage on the single-pass kernel (both tile
    heights, every z face kind): finite and within a loose bound of the
    oracle after 20 steps; the measured errors are printed."""
    monkeypatch.setenv("LBM_FUSED_TY", ty)
    w = FUSED[name]()
    ref = oracle_run(w, 20, record=(20,))
    for prec, bound in (("fp16", 5e-3), ("bf16", 2e-2)):
        sim = P.from_workload(w, precision=prec)
        sim.step(20)
        rho, u, T = sim.fields()
        sim.close()
        assert np.isfinite(rho).all() and np.isfinite(T).all()
        er = rel_err_scalar(rho, ref[20][0])
        eT = rel_err_scalar(T, ref[20][2])
        _log(f"{name} {prec} ty={ty} step 20: rho {er:.3e} T {eT:.3e}")
        assert er < bound and eT < bound


@pytest.mark.parametrize("name", list(FUSED))
def test_fused_matches_unfused_fp64(P, name, monkeypatch):
    w = FUSED[name]()
    out = []
    for flag in ("1", "0"):
        monkeypatch.setenv("LBM_FUSED", flag)
        sim = P.from_workload(w, precision="fp64")
        sim.step(15)
        out.append(sim.fields())
        sim.close()
    _compare(f"{name} fused vs unfused", out[0], out[1], 1e-13, 1e-13, 1e-13)


def _storage_ulp(dev, prec):
    """Spacing of the storage format at |dev| (normal range)."""
    import torch
    dt = {"fp32": torch.float32, "fp16": torch.float16, "bf16": torch.bfloat16}[prec]
    t = torch.from_numpy(np.abs(dev)).to(dt)
    e = torch.frexp(t.float())[1].numpy().astype(np.float64)
    mant = {"fp32": 23, "fp16": 10, "bf16": 7}[prec]
    tiny = {"fp32": 2.0 ** -126, "fp16": 2.0 ** -14, "bf16": 2.0 ** -126}[prec]
    return np.maximum(np.ldexp(1.0, (e - 1 - mant).astype(np.int64)), tiny * 2.0 ** -mant)


def _defined_slots(w):
    """Population slots a step defines, (19 + 7, nz) booleans: every slot
    except, on a pressure face plane, the f slots fed from beyond the face
    (unknowns until the next step's outlet fill), and every g of a bounded z
    face plane (all seven are replaced by the Dirichlet completion of the
    next step, so a step leaves the slots fed from outside as they were)."""
    nz = w["nz"]
    mf = np.ones((19, nz), dtype=bool)
    mg = np.ones((7, nz), dtype=bool)
    cz = O.C19[:, 2]
    if w["faces"][4] == O.PRESSURE:
        mf[cz > 0, 0] = False
    if w["faces"][5] == O.PRESSURE:
        mf[cz < 0, nz - 1] = False
    if w["faces"][4] != O.PERIODIC:
        mg[:, 0] = False
    if w["faces"][5] != O.PERIODIC:
        mg[:, nz - 1] = False
    return mf, mg


@pytest.mark.parametrize("prec,ty", [("fp32", "16"), ("fp16", "8"), ("fp16", "16"), ("bf16", "8"),
                                     ("bf16", "16")])
@pytest.mark.parametrize("name", list(FUSED))
def test_fused_matches_unfused_narrow_storage(P, name, prec, ty, monkeypatch):
    """The single-pass kernel (8- or 16-row tiles; 16-bit storage with its
    shifted tiles) against the general kernels after one step, population by
    population: the stored deviations differ by at most one storage ulp plus
    the rounding of float arithmetic on values of the size w_i rho (w_i rho
    c_v T for g): the two paths evaluate the same formulas in different
    orders.  Slots
    the step leaves undefined (see _defined_slots) are not compared."""
    monkeypatch.setenv("LBM_FUSED_TY", ty)
    w = FUSED[name]()
    pops = []
    for flag in ("1", "0"):
        monkeypatch.setenv("LBM_FUSED", flag)
        sim = P.from_workload(w, precision=prec)
        sim.step(1)
        pops.append(sim.populations())
        sim.close()
    wf = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)[:, None, None, None]
    w7 = np.array([0.25] + [0.125] * 6)[:, None, None, None]
    mf, mg = _defined_slots(w)
    worst = 0.0
    for lat, (fa, fb), wt, ref, mask, scale in (
            ("f", (pops[0][0], pops[1][0]), wf, w["rho_ref"], mf, float(np.max(w["rho0"]))),
            ("g", (pops[0][1], pops[1][1]), w7, w["T_ref"], mg,
             float(np.max(w["rho0"]) * (w.get("cv") or 5.0) * np.max(w["T0"])))):
        keep = np.broadcast_to(mask[:, :, None, None], fa.shape)
        da = np.where(keep, fa - wt * ref, 0.0)
        db = np.where(keep, fb - wt * ref, 0.0)
        ulp = _storage_ulp(np.maximum(np.abs(da), np.abs(db)), prec)
        # float arithmetic on values of the size w_i rho (w_i rho c_v T for g,
        # whose blend and source scale with the energy density), in a
        # different order on the two paths
        arith = 64 * 2.0 ** -24 * wt * scale
        excess = np.abs(da - db) / (ulp + arith)
        k = np.unravel_index(np.argmax(excess), excess.shape)
        _log(f"  {lat}: worst {float(excess[k]):.2f} at (i, z, y, x) = {tuple(int(v) for v in k)}: "
             f"{da[k]:.9e} vs {db[k]:.9e}")
        worst = max(worst, float(excess[k]))
    _log(f"{name} {prec} ty={ty}: fused vs unfused worst difference {worst:.2f} of the bound")
    assert worst <= 1.0


def test_fused_xcd_block_mapping_is_bitwise_the_same(P, monkeypatch):
    """The optional tile-to-XCD mapping (LBM_FUSED_MAP=1: each XCD a 2 x 4
    block of tiles, one chunk per column) changes only the schedule: every
    tile computes its cells the same way, so the state is bitwise the same."""
    w = synth.blobs_closed(nx=128, ny=32, nz=24, mean_blobs=3, rmin=4.0, rmax=6.0, seed=9)
    out = []
    for mapping in ("0", "1"):
        monkeypatch.setenv("LBM_FUSED_MAP", mapping)
        monkeypatch.setenv("LBM_FUSED_CHUNK", "24")
        sim = P.from_workload(w, precision="fp32")
        sim.step(12)
        out.append(sim.fields())
        sim.close()
    for a, b, what in zip(out[0], out[1], ("rho", "u", "T")):
        assert np.array_equal(a, b), what


@pytest.mark.parametrize("chunk", ["", "5"])
@pytest.mark.parametrize("name", ["droplet_periodic_128x16x24", "blobs_closed_64x32x40", "wetting_64x16x24",
                                  "heated_wall_64x16x24", "outlet_below_64x16x24", "open_z_64x16x32"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multi_step_call_is_bitwise_single_steps(P, prec, name, chunk, monkeypatch):
    """Within one multi-step call the single-pass kernel passes x-deferred
    states between its steps with FP64 storage (streamed in y and z,
    finished in x by the next step's loads); every cell is computed from the
    same values, so k steps in
    one call leave bitwise the populations of k one-step calls, also with the
    z range cut into 5-plane chunks (boundary planes inside the march).  Slots
    no step defines (fed from beyond a bounded face) are left out."""
    if chunk:
        monkeypatch.setenv("LBM_FUSED_CHUNK", chunk)
    w = FUSED[name]()
    _log(f"[x-deferred] {name} {prec} chunk={chunk or 'all'}")
    out = []
    for calls in ((7,), (2, 5), (1,) * 7):
        sim = P.from_workload(w, precision=prec)
        for k in calls:
            sim.step(k)
        out.append(sim.populations())
        sim.close()
    masks = _defined_slots(w)
    for got in out[:2]:
        for a, b, m, what in zip(got, out[2], masks, ("f", "g")):
            m = np.broadcast_to(m[:, :, None, None], a.shape)
            assert np.array_equal(a[m], b[m]), what


def test_multi_step_call_can_switch_off_x_deferral(P, monkeypatch):
    """LBM_FUSED_XDEFER=0 keeps the ordinary state between steps: the same
    result bitwise."""
    w = FUSED["heated_wall_64x16x24"]()
    out = []
    for xd in ("1", "0"):
        monkeypatch.setenv("LBM_FUSED_XDEFER", xd)
        sim = P.from_workload(w, precision="fp64")
        sim.step(9)
        out.append(sim.populations())
        sim.close()
    masks = _defined_slots(w)
    for a, b, m, what in zip(out[0], out[1], masks, ("f", "g")):
        m = np.broadcast_to(m[:, :, None, None], a.shape)
        assert np.array_equal(a[m], b[m]), what


# ---------------------------------------------------------------- vartheta = 1

def _theta1(w):
    w = dict(w)
    w["theta_corr"] = 1
    return w


THETA1 = {
    "droplet_open_37x34x29": lambda: _theta1(synth.droplet_open(nx=37, ny=34, nz=29, R0=9.0)),
    "heated_wall_35x31x27": lambda: _theta1(synth.heated_wall(nx=35, ny=31, nz=27, R0=10.0, Tw_jitter=0.02,
                                                               seed=5, kappa_w=0.3)),
    "droplet_periodic_128x16x24": lambda: _theta1(FUSED["droplet_periodic_128x16x24"]()),
}


@pytest.mark.parametrize("name", list(THETA1))
def test_theta1_parity_fp64(P, name):
    """The correction term of eq. (16) (vartheta = 1) against the oracle,
    across the steps where the temperature history fills up."""
    w = THETA1[name]()
    steps = 60
    _log(f"[theta=1] {name}")
    ref = oracle_run(w, steps, record=(1, 2, 3, steps))
    sim = P.from_workload(w, precision="fp64")
    done = 0
    for s in (1, 2, 3, steps):
        sim.step(s - done)
        done = s
        _compare(f"{name} theta=1 step {s}", sim.fields(), ref[s], TOL64, TOL64, TOL64)
    sim.close()


def test_theta1_changes_the_result(P):
    """vartheta = 1 is not a no-op: after the history fills, T differs from vartheta = 0."""
    w = THETA1["heated_wall_35x31x27"]()
    w0 = dict(w)
    w0["theta_corr"] = 0
    out = []
    for ww in (w0, w):
        sim = P.from_workload(ww, precision="fp64")
        sim.step(20)
        out.append(sim.fields()[2])
        sim.close()
    d = float(np.max(np.abs(out[1] - out[0])))
    _log(f"max |T(theta=1) - T(theta=0)| after 20 steps: {d:.3e}")
    assert d > 1e-12
