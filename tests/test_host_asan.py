"""AddressSanitizer and UBSan over the host-side plan of the library.

Builds paper_2603_08582_amd/csrc/host_plan.cpp (configuration checks, edgelet
atom tables, workspace layout, the pure-host ABI calls) with the host
compiler alone, together with tests/c/host_plan_check.cpp, which drives those
calls over valid, invalid and pseudo-random configurations.  Needs g++ with
libasan; no GPU and no HIP.
"""

import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
GXX = shutil.which("g++")

pytestmark = pytest.mark.skipif(GXX is None, reason="g++ not available")


def test_host_plan_under_address_sanitizer(tmp_path):
    exe = tmp_path / "host_plan_check"
    cmd = [GXX, "-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-Wno-unknown-pragmas", f"-I{ROOT / 'include'}",
           f"-I{ROOT / 'paper_2603_08582_amd' / 'csrc'}",
           str(ROOT / "paper_2603_08582_amd" / "csrc" / "host_plan.cpp"),
           str(ROOT / "tests" / "c" / "host_plan_check.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                         env={"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
                              "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert run.returncode == 0, (run.stdout + run.stderr)[-3000:]
    assert run.stdout.strip() == "ok"
