"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the face
topology, renumbering and aggregates (csrc/topology.cpp, Section 2 item 1 and
Section 3.2 items 5 and 7) built with g++ into tests/host/topology_sanitized.cpp,
run on valid and invalid 2D and 3D meshes.  No GPU; skipped without g++ or the
ROCm headers that csrc/internal.h includes."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM_INCLUDE = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INCLUDE),
                    reason="needs g++ and the ROCm headers")
def test_topology_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "topology_sanitized")
    # __HIP_PLATFORM_AMD__ lets the HIP runtime header compile under g++; no
    # device code is built here
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INCLUDE,
           os.path.join(ROOT, "tests", "host", "topology_sanitized.cpp"),
           os.path.join(ROOT, "paper_2101_03777_amd", "csrc", "topology.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "ok (0 failures)" in r.stdout, (r.stdout[-4000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
