"""Host checks of the library's per-cell adjoint arithmetic (no GPU):
tests/native/adjoint_local_check.cpp includes the library's own headers and
checks each reverse-mode routine against the forward routine it transposes
(dot-product identity for the linear maps, Richardson-extrapolated central
differences for the nonlinear ones)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

LIMITS = {"linear_transposes": 1e-12, "collide19": 1e-9, "collide7": 1e-11, "peng_robinson": 1e-10,
          "outlet_fill": 1e-12}


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = tmp_path_factory.mktemp("adj") / "adjoint_local_check"
    csrc = os.path.join(ROOT, "paper_2206_00946_amd", "csrc")
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-I", csrc, os.path.join(ROOT, "tests", "native", "adjoint_local_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {line.split()[0]: float(line.split()[1]) for line in out.splitlines() if line.strip()}


@pytest.mark.parametrize("name", sorted(LIMITS))
def test_local_adjoint(results, name):
    assert results[name] < LIMITS[name], results
