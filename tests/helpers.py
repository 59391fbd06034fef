"""Test helpers: run the oracle on a workload dict, compare fields."""
import numpy as np

from oracle import lbm_oracle as O


def oracle_params(w, **kw):
    extra = {}
    if w.get("lambda_vapour") is not None:
        extra = dict(lam_vapour=w["lambda_vapour"], lam_liquid=w["lambda_liquid"], lam_rho_v=w["lambda_rho_v"],
                     lam_rho_l=w["lambda_rho_l"])
    if w.get("cv") is not None:
        extra["cv"] = w["cv"]
    if w.get("theta_corr"):
        extra["theta_corr"] = int(w["theta_corr"])
    extra.update(kw)
    return O.Params(w["nx"], w["ny"], w["nz"], faces=tuple(w["faces"]), face_T=tuple(w["face_T"]),
                    face_rho=tuple(w["face_rho"]), kappa_w=w["kappa_w"], **extra)


def oracle_run(w, steps, record=(), check=True):
    """Run the oracle; returns {step: (rho, u, T)} for the requested steps.
    check=False lets cells leave the physical range without an error (for
    blocks cut out of a larger domain, whose artificial sides may do so
    outside the cells that are compared)."""
    p = oracle_params(w)
    f, g = O.init_populations(w["rho0"], w["T0"], p)
    Tw = w.get("Tw") or None
    out = {}
    hist = []
    if 0 in record:
        out[0] = O.fields(f, g, p, Tw)
    for s in range(1, steps + 1):
        f, g, mac = O.step(f, g, p, Tw, hist)
        if check and mac["bad"].any():
            raise FloatingPointError(f"oracle left the physical range at step {s - 1}")
        hist = [mac["T"]] + hist[:1]
        if s in record:
            out[s] = O.fields(f, g, p, Tw)
    return out


def rel_err_scalar(a, b):
    """max_x |a - b| / |b| (rho and T are bounded away from zero)."""
    return float(np.max(np.abs(a - b) / np.abs(b)))


def rel_err_vector(a, b):
    """max_x |a - b| / max_x |b| (normwise: u vanishes in the bulk)."""
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def sub_block(w, center, half, margin=6):
    """Workload restricted to the box of half-width `half` around `center`.

    Along a periodic axis the box wraps around (and is the whole axis if it
    would cover it).  Along a bounded axis it is clipped to the domain; if it
    touches one real face, that face's kind and values are used on both sides,
    otherwise the cut axis is made periodic.  Cells `margin` or more away from
    every artificial (cut) side evolve exactly as in the full domain for one
    step (the fields of one step reach 6 cells, the wetting ghost one more).
    Returns the block workload with 'index' (per-axis global indices of the
    block) and 'local' (the centre's position in the block)."""
    n = (w["nx"], w["ny"], w["nz"])
    faces = list(w["faces"])
    face_T = list(w["face_T"])
    face_rho = list(w["face_rho"])
    index = []
    local = []
    valid = []
    for a in range(3):
        c = center[a]
        if faces[2 * a] == 0:                      # periodic axis
            if 2 * half + 1 >= n[a]:
                idx = np.arange(n[a])
                index.append(idx)
                local.append(c)
                valid.append((0, n[a]))
                continue
            idx = np.arange(c - half, c + half + 1) % n[a]
            index.append(idx)
            local.append(half)
            valid.append((margin, 2 * half + 1 - margin))
            continue
        lo, hi = max(0, c - half), min(n[a], c + half + 1)
        idx = np.arange(lo, hi)
        index.append(idx)
        local.append(c - lo)
        if lo == 0 and hi == n[a]:
            valid.append((0, hi - lo))
        elif lo == 0:
            k = 2 * a
            faces[k + 1], face_T[k + 1], face_rho[k + 1] = faces[k], face_T[k], face_rho[k]
            valid.append((0, hi - lo - margin))
        elif hi == n[a]:
            k = 2 * a + 1
            faces[k - 1], face_T[k - 1], face_rho[k - 1] = faces[k], face_T[k], face_rho[k]
            valid.append((margin, hi - lo))
        else:
            faces[2 * a] = faces[2 * a + 1] = 0
            valid.append((margin, hi - lo - margin))
    ix, iy, iz = index
    sel = np.ix_(iz, iy, ix)
    b = dict(w)
    b.update(nx=len(ix), ny=len(iy), nz=len(iz), faces=faces, face_T=face_T, face_rho=face_rho,
             rho0=w["rho0"][sel].copy(), T0=w["T0"][sel].copy())
    Tw = {}
    for face, field in (w.get("Tw") or {}).items():
        if w["faces"][face] == 1:
            lo_z = iz[0] == 0 if face == 4 else iz[-1] == n[2] - 1
            if lo_z:
                Tw[face] = field[np.ix_(iy, ix)].copy()
    b["Tw"] = Tw
    b["index"] = index
    b["local"] = local
    b["valid"] = valid
    return b
