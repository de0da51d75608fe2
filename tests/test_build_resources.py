"""Every HIP kernel compiles for gfx950 without scratch memory or spills.

Private (scratch) memory on the hot path turned a register array into HBM
traffic twice during development (a lambda-captured prefetch array and a HIP
struct-vector array), multiplying the Gram kernel's write traffic ~8x; this
check keeps that from coming back.  Needs hipcc, no GPU.
"""

import re
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2603_08582_amd" / "csrc"
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

pytestmark = pytest.mark.skipif(not Path(HIPCC).exists(), reason="hipcc not available")


@pytest.mark.parametrize("src", sorted(p.name for p in CSRC.glob("*.hip")))
def test_no_scratch_no_spills(src, tmp_path):
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "--cuda-device-only",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           f"-I{ROOT / 'include'}", f"-I{CSRC}", "-c", str(CSRC / src), "-o",
           str(tmp_path / "k.o"), "-Rpass-analysis=kernel-resource-usage"]
    out = subprocess.run(cmd, capture_output=True, text=True)
    assert out.returncode == 0, out.stderr[-2000:]
    names = re.findall(r"Function Name: (\S+)", out.stderr)
    scratch = [int(x) for x in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", out.stderr)]
    vspill = [int(x) for x in re.findall(r"VGPRs Spill: (\d+)", out.stderr)]
    assert names and len(names) == len(scratch) == len(vspill)
    bad = [(n, s, v) for n, s, v in zip(names, scratch, vspill) if s or v]
    assert not bad, bad
