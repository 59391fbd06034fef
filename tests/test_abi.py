"""CPU-only checks of the C ABI: the library loads, exports every declared
entry point, its structs match the header, and host-side validation works.
No call here touches a GPU."""
import ctypes
import os
import re
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm3d.h")


def _lib():
    import paper_2206_00946_amd as P
    return P, P.load_library()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:lbm_status|const char\*|void)\s+(lbm_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_entry_point():
    P, lib = _lib()
    names = declared_functions()
    assert len(names) >= 10
    out = subprocess.run(["nm", "-D", "--defined-only", P.lbm3d.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT\s+(lbm_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(lib, n)
    assert set(P.lbm3d.EXPORTS) == set(names)


def test_struct_layout_matches_header(tmp_path):
    """Compile a C probe of the header with gcc and compare sizes/offsets
    with the ctypes mirrors."""
    P, _ = _lib()
    src = tmp_path / "probe.c"
    fields = [f[0] for f in P.LbmParams._fields_]
    cfields = ["lambda" if f == "lambda_" else f for f in fields]
    body = "\n".join(f'  printf("%zu\\n", offsetof(lbm_params, {c}));' for c in cfields)
    dfields = [f[0] for f in P.lbm3d.LbmDiag._fields_]
    dbody = "\n".join(f'  printf("%zu\\n", offsetof(lbm_diag, {c}));' for c in dfields)
    afields = [f[0] for f in P.lbm3d.LbmAdjointSpec._fields_]
    abody = '  printf("%zu\\n", sizeof(lbm_adjoint_spec));\n' + "\n".join(
        f'  printf("%zu\\n", offsetof(lbm_adjoint_spec, {c}));' for c in afields)
    src.write_text(textwrap.dedent("""
        #include <stdio.h>
        #include <stddef.h>
        #include "lbm3d.h"
        int main(void) {
          printf("%zu\\n", sizeof(lbm_params));
        """) + body + '\n  printf("%zu\\n", sizeof(lbm_diag));\n' + dbody + "\n" + abody + "\n  return 0;\n}\n")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    expect = [ctypes.sizeof(P.LbmParams)] + [getattr(P.LbmParams, f).offset for f in fields]
    expect += [ctypes.sizeof(P.lbm3d.LbmDiag)] + [getattr(P.lbm3d.LbmDiag, f).offset for f in dfields]
    expect += [ctypes.sizeof(P.lbm3d.LbmAdjointSpec)] + [getattr(P.lbm3d.LbmAdjointSpec, f).offset for f in afields]
    assert vals == expect


def test_default_params_are_the_papers():
    P, lib = _lib()
    p = P.LbmParams()
    assert lib.lbm_default_params(ctypes.byref(p), 4, 5, 6) == 0
    assert (p.nx, p.ny, p.nz) == (4, 5, 6)
    assert p.a == 3 / 49 and p.b == 2 / 21 and p.R == 1 and p.omega == 0.344 and p.G == -1
    assert p.s_nu == 0.8 and p.s_e == 1.25 and p.s_q == 1 and p.s_pi == 1
    assert abs(p.lambda_ - 1 / 3) < 1e-16 and p.cv == 5 and p.wbar == 0.75
    assert list(p.face) == [0] * 6 and p.theta_corr == 0
    assert lib.lbm_default_params(None, 1, 1, 1) == 1


def _required(P, lib, p):
    st, sc = ctypes.c_size_t(), ctypes.c_size_t()
    s = lib.lbm_required_bytes(ctypes.byref(p), ctypes.byref(st), ctypes.byref(sc))
    return s, st.value, sc.value


@pytest.mark.parametrize("prec,es", [("fp64", 8), ("fp32", 4), ("fp16", 2), ("bf16", 2)])
def test_required_bytes(prec, es):
    P, lib = _lib()
    p = P.make_params(40, 30, 20, precision=prec)
    s, st, sc = _required(P, lib, p)
    assert s == 0
    # two states of 26 direction planes per z level, each plane padded to
    # nx*ny + 64 elements, each buffer aligned to 256 bytes
    slots = 20 * (40 * 30 + 64)
    assert st >= 2 * 26 * slots * es and st < 2 * 26 * slots * es + 4 * 256
    assert sc > 0


@pytest.mark.parametrize("change,status", [
    (dict(nx=0), 1),
    (dict(faces=(0, 2, 0, 0, 0, 0)), 1),                      # unpaired periodic face
    (dict(faces=(2, 2, 0, 0, 0, 0), nx=2), 1),                # bounded axis too short
    (dict(s_nu=2.0), 1),
    (dict(wbar=1.0), 1),
    (dict(lam=0.0), 1),
    (dict(cv=-1.0), 1),
    (dict(faces=(2, 2, 0, 0, 0, 0), face_T=(0.1,) * 6, face_rho=(0.0,) * 6), 1),   # rho_out missing
    (dict(faces=(0, 0, 0, 0, 1, 1), face_T=(0.0,) * 6), 1),   # wall without temperature
    (dict(theta_corr=2), 1),
    (dict(lambda_vapour=0.2), 1),                             # one conductivity only
    (dict(faces=(1, 1, 0, 0, 0, 0), face_T=(0.1,) * 6), 6),   # x walls
    (dict(faces=(2, 2, 0, 0, 1, 1), face_T=(0.1,) * 6, face_rho=(0.4,) * 6), 6),  # z wall needs periodic x
    (dict(precision=7), 1),
])
def test_parameter_validation(change, status):
    P, lib = _lib()
    kw = dict(change)
    nx = kw.pop("nx", 8)
    p = P.make_params(nx, 8, 8, **kw)
    s, _, _ = _required(P, lib, p)
    assert s == status
    assert lib.lbm_last_error(None)


def test_binding_fails_loudly_without_library(tmp_path):
    code = textwrap.dedent(f"""
        import sys
        sys.path.insert(0, {ROOT!r})
        import paper_2206_00946_amd.lbm3d as m
        m.LIB_PATH = {str(tmp_path / 'missing.so')!r}
        m._lib = None
        try:
            m.load_library()
        except ImportError as e:
            print("raised", e)
            sys.exit(0)
        sys.exit(1)
    """)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert r.returncode == 0 and "raised" in r.stdout


def test_product_path_never_touches_the_oracle():
    """The package, the HIP sources and the header do not import or include
    anything from oracle/."""
    pkg = os.path.join(ROOT, "paper_2206_00946_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"\boracle\b", text), fn
