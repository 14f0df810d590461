"""Occupancy budget of the hot kernels, from the compiler's resource report
(gfx950): a change that costs a kernel a wave per SIMD fails here, on the CPU,
before it shows up as a slower benchmark.  The floors are the measured
occupancies of the tuned kernels (waves per SIMD)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1611_07289_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

FLOORS = {
    "pvr_forward.hip": {
        "_Z10k_simulateIfE": 7,
        "_Z10k_registerILb1ELb0ELi0E": 2,   # exact gradient, x-fastest volume
        "_Z10k_registerILb1ELb1ELi0E": 2,   # exact gradient, y-fastest copy
        "_Z10k_registerILb0ELb0ELi0E": 4,   # central differences (held to 128 VGPRs)
        "_Z10k_registerILb0ELb0ELi1E": 2,   # central differences, sinc PSF
    },
    "pvr_adjoint.hip": {
        "_Z13k_backprojectIfLb1ELi1ELb0E": 8,
    },
}


def occupancies(src):
    out = subprocess.run(
        [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-I", os.path.join(ROOT, "include"),
         "-I", CSRC, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-c",
         "-o", os.devnull, "-Rpass-analysis=kernel-resource-usage", os.path.join(CSRC, src)],
        capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    occ, name = {}, None
    for line in out.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"Occupancy \[waves/SIMD\]: (\d+)", line)
        if m and name:
            occ[name] = int(m.group(1))
    return occ


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("src", sorted(FLOORS))
def test_hot_kernels_keep_their_occupancy(src):
    occ = occupancies(src)
    for prefix, floor in FLOORS[src].items():
        got = [v for k, v in occ.items() if k.startswith(prefix)]
        assert got, f"kernel {prefix} not found in {src}"
        assert min(got) >= floor, f"{prefix}: occupancy {min(got)} < {floor} waves/SIMD"
