"""CPU: the host planner under the address and undefined-behaviour
sanitizers (host code only; no GPU).  tests/plan_check.cpp builds the host
tables of many decompositions (Sec. 3.2, Fig. 3: boxes tiling the periodic
grid, guard cells per side) and checks the exchange pieces cover every guard
cell exactly once from its owner, that every piece lies inside its boxes'
field ranges, and that the work lists add up; invalid decompositions must be
rejected."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.timeout(600)
def test_planner_under_asan_and_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "plan_check")
    # -Xarch_host: the sanitizers instrument the host compilation only
    cmd = [HIPCC, "-std=c++17", "-O2", "-g", "--offload-host-only", "-x", "hip",
           os.path.join(ROOT, "tests", "plan_check.cpp"),
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1707_08500_amd", "csrc"),
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
           "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "plan_check: ok" in r.stdout
