"""Python binding of liblbm3d.so (argument marshalling only).

Every step of the update runs in the HIP library; torch only provides device
memory and the stream.  Importing this module fails loudly if the library
has not been built (``python -c "import __graft_entry__ as g; g.build()"``).
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm3d.so")

FP64, FP32_DEV, FP16_DEV, BF16_DEV = 0, 1, 2, 3
PERIODIC, WALL, PRESSURE = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32_DEV, "fp16": FP16_DEV, "bf16": BF16_DEV}

STATUS = {0: "LBM_OK", 1: "LBM_EINVAL", 2: "LBM_ENOMEM", 3: "LBM_EHIP", 4: "LBM_ENONPHYS",
          5: "LBM_ESTATE", 6: "LBM_EUNSUPPORTED"}


class LbmParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double), ("omega", ctypes.c_double),
        ("G", ctypes.c_double),
        ("s_e", ctypes.c_double), ("s_nu", ctypes.c_double), ("s_q", ctypes.c_double), ("s_pi", ctypes.c_double),
        ("wbar", ctypes.c_double), ("lambda_", ctypes.c_double), ("cv", ctypes.c_double),
        ("s_T_other", ctypes.c_double),
        ("theta_corr", ctypes.c_int32),
        ("face", ctypes.c_int32 * 6),
        ("face_T", ctypes.c_double * 6),
        ("face_rho", ctypes.c_double * 6),
        ("kappa_w", ctypes.c_double),
        ("rho_ref", ctypes.c_double), ("T_ref", ctypes.c_double),
        ("diag_rho_v", ctypes.c_double), ("diag_rho_l", ctypes.c_double),
        ("lambda_vapour", ctypes.c_double), ("lambda_liquid", ctypes.c_double),
        ("lambda_rho_v", ctypes.c_double), ("lambda_rho_l", ctypes.c_double),
    ]


class LbmDiag(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("energy", ctypes.c_double), ("vol_hard", ctypes.c_double),
                ("vol_smooth", ctypes.c_double), ("evap_mass", ctypes.c_double), ("step", ctypes.c_int64)]


class LbmAdjointSpec(ctypes.Structure):
    _fields_ = [("nsteps", ctypes.c_int32), ("n_checkpoints", ctypes.c_int32), ("objective", ctypes.c_int32),
                ("wall_face", ctypes.c_int32)]


EXPORTS = ["lbm_default_params", "lbm_required_bytes", "lbm_create", "lbm_init", "lbm_set_wall_T",
           "lbm_set_kappa", "lbm_step", "lbm_fields", "lbm_populations", "lbm_save_bytes", "lbm_save",
           "lbm_load", "lbm_reduce", "lbm_adjoint_bytes", "lbm_adjoint", "lbm_adjoint_noalloc", "lbm_last_error",
           "lbm_destroy"]

_lib = None


def load_library():
    """Load liblbm3d.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    # torch brings its own HIP runtime with the same soname as the one the
    # library links; loading torch first makes the process use exactly one
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    dp = P(ctypes.c_double)
    lib.lbm_default_params.argtypes = [P(LbmParams), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.lbm_required_bytes.argtypes = [P(LbmParams), P(ctypes.c_size_t), P(ctypes.c_size_t)]
    lib.lbm_create.argtypes = [P(LbmParams), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                               P(ctypes.c_void_p)]
    lib.lbm_init.argtypes = [ctypes.c_void_p, dp, dp, dp]
    lib.lbm_set_wall_T.argtypes = [ctypes.c_void_p, ctypes.c_int32, dp]
    lib.lbm_set_kappa.argtypes = [ctypes.c_void_p, ctypes.c_double]
    lib.lbm_step.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.lbm_fields.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
    lib.lbm_populations.argtypes = [ctypes.c_void_p, dp, dp]
    lib.lbm_reduce.argtypes = [ctypes.c_void_p, P(LbmDiag)]
    lib.lbm_save_bytes.argtypes = [ctypes.c_void_p, P(ctypes.c_size_t)]
    lib.lbm_save.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
    lib.lbm_load.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
    lib.lbm_adjoint_bytes.argtypes = [ctypes.c_void_p, P(LbmAdjointSpec), P(ctypes.c_size_t)]
    lib.lbm_adjoint.argtypes = [ctypes.c_void_p, P(LbmAdjointSpec), dp, ctypes.c_void_p, dp, ctypes.c_int32]
    lib.lbm_adjoint_noalloc.argtypes = [ctypes.c_void_p, P(LbmAdjointSpec), dp, ctypes.c_void_p, dp,
                                        ctypes.c_int32]
    lib.lbm_last_error.argtypes = [ctypes.c_void_p]
    lib.lbm_last_error.restype = ctypes.c_char_p
    lib.lbm_destroy.argtypes = [ctypes.c_void_p]
    lib.lbm_destroy.restype = None
    for name in EXPORTS:
        if name not in ("lbm_last_error", "lbm_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(nx, ny, nz, precision="fp32", faces: Sequence[int] = (PERIODIC,) * 6, face_T=None,
                face_rho=None, kappa_w=0.0, rho_ref=None, T_ref=None, diag_rho_v=None, diag_rho_l=None,
                **overrides) -> LbmParams:
    lib = load_library()
    p = LbmParams()
    lib.lbm_default_params(ctypes.byref(p), nx, ny, nz)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    for k in range(6):
        p.face[k] = int(faces[k])
        if face_T is not None:
            p.face_T[k] = float(face_T[k])
        if face_rho is not None:
            p.face_rho[k] = float(face_rho[k])
    p.kappa_w = float(kappa_w)
    if rho_ref is not None:
        p.rho_ref = float(rho_ref)
    if T_ref is not None:
        p.T_ref = float(T_ref)
    if diag_rho_v is not None:
        p.diag_rho_v = float(diag_rho_v)
    if diag_rho_l is not None:
        p.diag_rho_l = float(diag_rho_l)
    for k, v in overrides.items():
        setattr(p, "lambda_" if k == "lam" else k, v)
    return p


def params_from_workload(w: Dict, precision="fp32") -> LbmParams:
    extra = {k: w[k] for k in ("lambda_vapour", "lambda_liquid", "lambda_rho_v", "lambda_rho_l", "cv", "theta_corr")
             if w.get(k) is not None}
    return make_params(w["nx"], w["ny"], w["nz"], precision=precision, faces=w["faces"], face_T=w["face_T"],
                       face_rho=w["face_rho"], kappa_w=w["kappa_w"], rho_ref=w["rho_ref"], T_ref=w["T_ref"],
                       diag_rho_v=w["rho_v"], diag_rho_l=w["rho_l"], **extra)


class Lbm3D:
    """One simulation context on the current torch CUDA (HIP) device.

    The device buffer is a torch uint8 tensor owned by this object; the
    library enqueues on torch's current stream at construction time.
    """

    def __init__(self, params: LbmParams, device: str = "cuda", torch_buffer: bool = True):
        import torch

        self.lib = load_library()
        self.params = params
        self.torch = torch
        st = ctypes.c_size_t()
        sc = ctypes.c_size_t()
        self._check(self.lib.lbm_required_bytes(ctypes.byref(params), ctypes.byref(st), ctypes.byref(sc)), None)
        self.state_bytes, self.scratch_bytes = st.value, sc.value
        self.buffer = None
        ptr = None
        nbytes = 0
        if torch_buffer:
            self.buffer = torch.empty(st.value + sc.value + 256, dtype=torch.uint8, device=device)
            base = self.buffer.data_ptr()
            ptr = (base + 255) // 256 * 256
            nbytes = st.value + sc.value
        self.stream = torch.cuda.current_stream(torch.device(device))
        ctx = ctypes.c_void_p()
        self._check(self.lib.lbm_create(ctypes.byref(params), ptr, nbytes, ctypes.c_void_p(self.stream.cuda_stream),
                                        ctypes.byref(ctx)), None)
        self.ctx = ctx
        self.n = params.nx * params.ny * params.nz
        self.shape = (params.nz, params.ny, params.nx)

    def _check(self, status, ctx):
        if status != 0:
            msg = self.lib.lbm_last_error(ctx.value if isinstance(ctx, ctypes.c_void_p) else ctx)
            raise LbmError(status, (msg or b"").decode())

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.lib.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- API
    def init(self, rho0: np.ndarray, T0: np.ndarray, u0: Optional[np.ndarray] = None):
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64).reshape(-1)
        T0 = np.ascontiguousarray(T0, dtype=np.float64).reshape(-1)
        if rho0.size != self.n or T0.size != self.n:
            raise ValueError("rho0 and T0 need nx*ny*nz values")
        u = None
        if u0 is not None:
            u = np.ascontiguousarray(u0, dtype=np.float64).reshape(-1)
            if u.size != 3 * self.n:
                raise ValueError("u0 needs 3*nx*ny*nz values")
        self._check(self.lib.lbm_init(self.ctx, _dptr(rho0), _dptr(u), _dptr(T0)), self.ctx)

    def set_wall_T(self, face: int, Tw: Optional[np.ndarray]):
        arr = None if Tw is None else np.ascontiguousarray(Tw, dtype=np.float64).reshape(-1)
        if arr is not None and arr.size != self.params.nx * self.params.ny:
            raise ValueError("wall field needs nx*ny values")
        self._check(self.lib.lbm_set_wall_T(self.ctx, int(face), _dptr(arr)), self.ctx)

    def set_kappa(self, kappa_w: float):
        self._check(self.lib.lbm_set_kappa(self.ctx, float(kappa_w)), self.ctx)

    def step(self, nsteps: int = 1):
        self._check(self.lib.lbm_step(self.ctx, int(nsteps)), self.ctx)

    def fields(self):
        rho = np.empty(self.n)
        u = np.empty(3 * self.n)
        T = np.empty(self.n)
        self._check(self.lib.lbm_fields(self.ctx, rho.ctypes.data, u.ctypes.data, T.ctypes.data, 0), self.ctx)
        return rho.reshape(self.shape), u.reshape((3,) + self.shape), T.reshape(self.shape)

    def fields_device(self):
        """Fields into torch float64 tensors on the device (no host copy)."""
        t = self.torch
        dev = self.buffer.device if self.buffer is not None else "cuda"
        rho = t.empty(self.n, dtype=t.float64, device=dev)
        u = t.empty(3 * self.n, dtype=t.float64, device=dev)
        T = t.empty(self.n, dtype=t.float64, device=dev)
        self._check(self.lib.lbm_fields(self.ctx, rho.data_ptr(), u.data_ptr(), T.data_ptr(), 1), self.ctx)
        return rho.view(self.shape), u.view((3,) + self.shape), T.view(self.shape)

    def populations(self):
        f = np.empty(19 * self.n)
        g = np.empty(7 * self.n)
        self._check(self.lib.lbm_populations(self.ctx, _dptr(f), _dptr(g)), self.ctx)
        return f.reshape((19,) + self.shape), g.reshape((7,) + self.shape)

    def save(self) -> np.ndarray:
        """Host image of the whole state (lbm_save), as a uint8 array."""
        n = ctypes.c_size_t()
        self._check(self.lib.lbm_save_bytes(self.ctx, ctypes.byref(n)), self.ctx)
        buf = np.empty(n.value, dtype=np.uint8)
        self._check(self.lib.lbm_save(self.ctx, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes), self.ctx)
        return buf

    def load(self, image: np.ndarray) -> None:
        """Resume from an image written by save() (lbm_load)."""
        image = np.ascontiguousarray(image, dtype=np.uint8)
        self._check(self.lib.lbm_load(self.ctx, image.ctypes.data_as(ctypes.c_void_p), image.nbytes), self.ctx)

    def reduce(self) -> Dict[str, float]:
        d = LbmDiag()
        self._check(self.lib.lbm_reduce(self.ctx, ctypes.byref(d)), self.ctx)
        return dict(mass=d.mass, energy=d.energy, vol_hard=d.vol_hard, vol_smooth=d.vol_smooth,
                    evap_mass=d.evap_mass, step=d.step)

    def adjoint_bytes(self, nsteps: int, wall_face: int = 4, n_checkpoints: int = 0) -> int:
        spec = LbmAdjointSpec(int(nsteps), int(n_checkpoints), 0, int(wall_face))
        n = ctypes.c_size_t()
        self._check(self.lib.lbm_adjoint_bytes(self.ctx, ctypes.byref(spec), ctypes.byref(n)), self.ctx)
        return n.value

    def adjoint(self, nsteps: int, wall_face: int = 4, n_checkpoints: int = 0, noalloc: bool = False):
        """Advance nsteps and return (J, dJ/dT_w as (ny, nx), dJ/dkappa_w) for the
        evaporated mass J = M(t0) - M(t0 + nsteps).  noalloc: use
        lbm_adjoint_noalloc (workspace in the library's fixed device array)."""
        spec = LbmAdjointSpec(int(nsteps), int(n_checkpoints), 0, int(wall_face))
        J = ctypes.c_double()
        dk = ctypes.c_double()
        grad = np.empty(self.params.nx * self.params.ny)
        fn = self.lib.lbm_adjoint_noalloc if noalloc else self.lib.lbm_adjoint
        self._check(fn(self.ctx, ctypes.byref(spec), ctypes.byref(J), grad.ctypes.data, ctypes.byref(dk), 0),
                    self.ctx)
        return J.value, grad.reshape(self.params.ny, self.params.nx), dk.value


def from_workload(w: Dict, precision="fp32", device="cuda") -> Lbm3D:
    sim = Lbm3D(params_from_workload(w, precision), device=device)
    sim.init(w["rho0"], w["T0"])
    for face, field in (w.get("Tw") or {}).items():
        sim.set_wall_T(face, field)
    return sim


def evaporated_mass_function():
    """torch.autograd.Function: J = EvaporatedMass.apply(sim, rho0, T0, nsteps, face, Tw, kappa).

    Tw: float64 tensor (ny, nx) of wall temperatures; kappa: float64 scalar
    tensor.  The forward pass runs lbm_adjoint once (the discrete adjoint
    needs the forward trajectory anyway) and keeps the gradients; backward
    scales them by the incoming gradient.  rho0, T0 (numpy) fix the state
    the simulation restarts from on every call."""
    import torch

    class EvaporatedMass(torch.autograd.Function):
        @staticmethod
        def forward(ctx, sim, rho0, T0, nsteps, face, Tw, kappa):
            sim.init(rho0, T0)
            sim.set_wall_T(face, Tw.detach().cpu().numpy().astype(np.float64))
            sim.set_kappa(float(kappa))
            J, dTw, dk = sim.adjoint(int(nsteps), wall_face=int(face))
            ctx.save_for_backward(torch.as_tensor(dTw, dtype=torch.float64, device=Tw.device),
                                  torch.tensor(dk, dtype=torch.float64, device=kappa.device))
            return torch.tensor(J, dtype=torch.float64, device=Tw.device)

        @staticmethod
        def backward(ctx, gJ):
            dTw, dk = ctx.saved_tensors
            return None, None, None, None, None, gJ * dTw, gJ * dk

    return EvaporatedMass
