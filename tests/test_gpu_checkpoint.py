"""Checkpoint and resume through the C ABI (lbm_save / lbm_load): a context
restored from an image continues bitwise like the context that wrote it —
unfused kernels with a wall temperature field, wetting and an outlet, the
single-pass kernel in FP32 and (outlet variant) in BF16, and vartheta = 1
with its temperature history —
and malformed or mismatched images are refused."""
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


def _theta1(w):
    w = dict(w)
    w["theta_corr"] = 1
    return w


CASES = {
    "heated_wall_20x18x16_fp64": (lambda: synth.heated_wall(nx=20, ny=18, nz=16, R0=6.0, Tw_jitter=0.02,
                                                            kappa_w=0.2), "fp64"),
    "blobs_closed_64x32x40_fp32": (lambda: synth.blobs_closed(nx=64, ny=32, nz=40, mean_blobs=3, rmin=5.0,
                                                              rmax=8.0, seed=9), "fp32"),
    "droplet_open_37x34x29_theta1_fp64": (lambda: _theta1(synth.droplet_open(nx=37, ny=34, nz=29, R0=9.0)),
                                          "fp64"),
    "heated_wall_64x16x24_bf16": (lambda: synth.heated_wall(nx=64, ny=16, nz=24, R0=6.0, Tw_jitter=0.02,
                                                            kappa_w=0.2), "bf16"),
}


def _state(sim):
    return list(sim.fields()) + [sim.reduce()]


@pytest.mark.parametrize("name", list(CASES))
def test_resume_is_bitwise(P, name):
    make, prec = CASES[name]
    w = make()
    _log(f"checkpoint {name}")
    a = P.from_workload(w, precision=prec)
    a.step(4)                  # fills the vartheta = 1 history, moves off the initial state
    image = a.save()
    a.step(5)
    ref = _state(a)
    a.close()
    # a fresh context of the same set-up, initialised differently and with other
    # wall temperatures and kappa_w: the image overrides all of it
    w2 = dict(w)
    w2["rho0"] = np.full_like(w["rho0"], w["rho_v"])
    w2["T0"] = np.full_like(w["T0"], w["T_ref"])
    w2["Tw"] = {}
    b = P.from_workload(w2, precision=prec)
    b.set_kappa(0.0)
    b.load(image)
    b.step(5)
    got = _state(b)
    b.close()
    for x, y, what in zip(ref[:3], got[:3], ("rho", "u", "T")):
        assert np.array_equal(x, y), f"{name}: {what} differs after resume"
    for key in ("mass", "energy", "evap_mass", "step"):
        assert ref[3][key] == got[3][key], (name, key, ref[3][key], got[3][key])
    assert got[3]["step"] == 9


def test_refused_images(P):
    w = synth.heated_wall(nx=20, ny=18, nz=16, R0=6.0, Tw_jitter=0.02, kappa_w=0.2)
    a = P.from_workload(w, precision="fp64")
    a.step(2)
    image = a.save()
    # too short
    with pytest.raises(P.LbmError) as e:
        a.load(image[: image.size - 8])
    assert e.value.status == 1
    # not an image
    bad = image.copy()
    bad[:8] = 0
    with pytest.raises(P.LbmError) as e:
        a.load(bad)
    assert e.value.status == 1
    # another grid
    w_other = synth.heated_wall(nx=21, ny=18, nz=16, R0=6.0, Tw_jitter=0.02, kappa_w=0.2)
    o = P.from_workload(w_other, precision="fp64")
    with pytest.raises(P.LbmError) as e:
        o.load(image)
    assert e.value.status == 1
    o.close()
    # another precision
    f32 = P.from_workload(w, precision="fp32")
    with pytest.raises(P.LbmError) as e:
        f32.load(image)
    assert e.value.status == 1
    f32.close()
    # the refused loads left the context as it was: it still resumes its own image
    a.load(image)
    assert a.reduce()["step"] == 2
    a.close()
    # save before init
    fresh = P.Lbm3D(P.params_from_workload(w, "fp64"))
    with pytest.raises(P.LbmError) as e:
        fresh.save()
    assert e.value.status == 5
    fresh.close()
