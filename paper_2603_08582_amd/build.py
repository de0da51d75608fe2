"""Build libofista.so in-tree with hipcc for gfx950.

    python -m paper_2603_08582_amd.build        (or build() from Python)

Every HIP source is compiled with packed-FP32 instructions disabled
(-target-feature -packed-fp32-ops) and linked into one shared library next
to this file.  The test suite's plain-C driver of the ABI (tests/c) is built
against it with the host C compiler, and the plain streaming-read reference
(tests/c/read_ceiling.hip) with hipcc.  The oracle's C parts (if any) are built
by __graft_entry__.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
from pathlib import Path

HERE = Path(__file__).resolve().parent
CSRC = HERE / "csrc"
INCLUDE = HERE.parent / "include"
LIB = HERE / "libofista.so"
BUILD = HERE.parent / "_build" / "ofista"

ARCH = os.environ.get("OFISTA_ARCH", "gfx950")
SOURCES = ["rows.hip", "gram.hip", "fista.hip", "adjoint.hip", "host_plan.cpp", "runtime.cpp"]
# Per-source extra flags.  The Gram kernels keep their MFMA accumulators in
# ordinary VGPRs (no copies to and from the accumulation registers around
# each LDS stage): same results bit for bit, fewer registers, higher occupancy.
EXTRA = {"gram.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and Path(cand).exists():
            return cand
    raise RuntimeError("hipcc not found: install ROCm or set HIPCC")


def _flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            f"-I{INCLUDE}", f"-I{CSRC}", "-Wall", "-Wno-unused-function",
            "-Wno-unknown-warning-option"]


def _compile(src: str) -> Path:
    BUILD.mkdir(parents=True, exist_ok=True)
    obj = BUILD / (src + ".o")
    cmd = [hipcc(), *_flags(), *EXTRA.get(src, []), "-c", str(CSRC / src), "-o", str(obj)]
    if src.endswith(".cpp"):
        cmd.insert(1, "-x")
        cmd.insert(2, "hip")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


ROCM = Path(os.environ.get("ROCM_PATH", "/opt/rocm"))
CDRIVER = HERE.parent / "tests" / "c" / "ofista_run.c"


def build_c_driver(lib: Path = LIB) -> Path:
    """Compile tests/c/ofista_run.c (C11, HIP runtime C API) against lib."""
    cc = os.environ.get("CC") or shutil.which("gcc") or shutil.which("cc")
    if not cc:
        raise RuntimeError("no C compiler for the ABI driver")
    exe = CDRIVER.with_suffix("")
    cmd = [cc, "-std=c11", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           f"-I{ROCM / 'include'}", f"-I{INCLUDE}", str(CDRIVER), "-o", str(exe),
           f"-L{lib.parent}", "-lofista", f"-L{ROCM / 'lib'}", "-lamdhip64", "-lm",
           f"-Wl,-rpath,$ORIGIN/{os.path.relpath(lib.parent, exe.parent)}",
           f"-Wl,-rpath,{ROCM / 'lib'}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"C driver build failed:\n{r.stdout}\n{r.stderr}")
    return exe


READ_CEILING = HERE.parent / "tests" / "c" / "read_ceiling.hip"


def build_read_ceiling() -> Path:
    """Compile tests/c/read_ceiling.hip (the plain streaming-read reference
    the tile pass is compared with; no library code)."""
    exe = READ_CEILING.with_suffix("")
    cmd = [hipcc(), "-O3", "-std=c++17", f"--offload-arch={ARCH}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           str(READ_CEILING), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"read_ceiling build failed:\n{r.stdout}\n{r.stderr}")
    return exe


def build(verbose: bool = False) -> Path:
    with cf.ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *map(str, objs),
           "-o", str(tmp)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    exe = build_c_driver(LIB)
    rc_exe = build_read_ceiling()
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
        print(f"built {exe}", file=sys.stderr)
        print(f"built {rc_exe}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
