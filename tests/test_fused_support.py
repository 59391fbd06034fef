"""Host check (no GPU) of the set-ups that take the single-pass kernel:
x/y periodic, z periodic or bounded by walls or pressure outlets (both z
faces bounded), at least 8 columns, tile-divisible y, at least 4 planes,
and direction planes small enough for the kernel's 32-bit buffer offsets
(larger planes run the unfused kernels, which index with 64 bits), and the z
planes per workgroup the context picks."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

EXPECTED = {
    "blobs_512x512x384_fp32": 1, "blobs_512x512x384_fp64": 1, "periodic_64x8x4_fp16": 1,
    "ragged_96x8x8_fp32": 1, "narrow_4x8x8_fp32": 0, "short_64x8x3_fp32": 0, "outlet_512x512x384_fp32": 1,
    "outlets_256x256x256_fp64": 1, "half_open_256x256x256_fp32": 0, "side_outlet_128x128x128_fp32": 0,
    "plane_4096x4096_fp64": 1, "plane_8192x4096_fp32": 1, "plane_8192x4096_fp64": 0,
    "plane_8192x8192_fp32": 0,
    "limit_5184x5104_fp64": 1, "over_5184x5112_fp64": 0, "limit_7296x7256_fp32": 1, "over_7296x7264_fp32": 0,
    "ty16_512x512x384_fp32": 1, "ty16_512x512x384_fp64": 0, "ty16_64x8x8_fp32": 0,
    "ty16_ragged_96x16x8_fp32": 0,
    # z planes per workgroup: one round of 256 workgroups where the tiles
    # allow (256^3: 128 tiles x 2 chunks), whole columns at 512^2 (512 tiles)
    "chunk_512x512x384": 384, "chunk_256x256x256": 128, "chunk_128x128x128": 16,
    "chunk_64x16x24": 8, "chunk_64x8x4": 4,
}


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = tmp_path_factory.mktemp("fs") / "fused_support_check"
    csrc = os.path.join(ROOT, "paper_2206_00946_amd", "csrc")
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-I", csrc, os.path.join(ROOT, "tests", "native", "fused_support_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {line.split()[0]: int(line.split()[1]) for line in out.splitlines() if line.strip()}


@pytest.mark.parametrize("name", sorted(EXPECTED))
def test_fused_support(results, name):
    assert results[name] == EXPECTED[name], results
