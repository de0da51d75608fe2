"""The C ABI driven from plain C (tests/c/ofista_run.c): no Python, no PyTorch
between the caller and libofista.

CPU: the driver compiles and links as C11 against include/ofista.h, and its
host-only paths behave (usage error; an invalid configuration is rejected by
the pure host calls before any GPU work).
GPU: a run described in a file gives the image the Python binding gives on the
same inputs, bit for bit (one library, one deterministic launch sequence), and
matches the FP64 oracle within the FP32 image tolerance.
"""

import struct
import subprocess
from pathlib import Path

import numpy as np
import pytest

from oracle import sar
from oracle.online_fista import OnlineFistaOracle
from workload import library_kwargs, make_workload, spec

ROOT = Path(__file__).resolve().parents[1]
DRIVER = ROOT / "tests" / "c" / "ofista_run"


def write_problem(path, kw, iters, order, pulses):
    """The driver's input layout (see tests/c/ofista_run.c)."""
    pos = np.ascontiguousarray(kw["positions"], np.float64)
    f = kw["freq0"], kw["dfreq"]
    dic = {"identity": 0, "haar": 1}[kw.get("dictionary", "identity")]
    lam = kw.get("lam", 0.05)
    with open(path, "wb") as fh:
        fh.write(struct.pack("<ii", kw["n_x"], kw["n_y"]))
        fh.write(struct.pack("<dddd", kw["x0"], kw["y0"], kw["dx"], kw["dy"]))
        fh.write(struct.pack("<ii", pos.shape[0], kw["n_freq"]))
        fh.write(struct.pack("<dd", *f))
        fh.write(struct.pack("<ii", dic, kw.get("haar_levels", 1)))
        fh.write(struct.pack("<d", lam))
        fh.write(struct.pack("<iii", 1 if kw.get("lam_relative", True) else 0, iters, len(order)))
        fh.write(pos.tobytes())
        fh.write(np.asarray(order, np.int32).tobytes())
        fh.write(np.ascontiguousarray(pulses, np.complex64).tobytes())


def compile_driver(tmp_path):
    from paper_2603_08582_amd import build as b
    exe = tmp_path / "ofista_run"
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           f"-I{b.ROCM / 'include'}", f"-I{b.INCLUDE}", str(b.CDRIVER), "-o", str(exe),
           f"-L{b.LIB.parent}", "-lofista", f"-L{b.ROCM / 'lib'}", "-lamdhip64", "-lm",
           f"-Wl,-rpath,{b.LIB.parent}", f"-Wl,-rpath,{b.ROCM / 'lib'}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_driver_compiles_as_c_and_rejects_bad_input(tmp_path):
    from paper_2603_08582_amd import build as b
    if not b.LIB.exists():
        pytest.skip("libofista.so not built")
    exe = compile_driver(tmp_path)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 1 and "usage" in r.stderr
    # n_x = 0 is invalid: ofista_workspace_bytes returns 0, no GPU call is made
    wl = make_workload(spec("small", n_side=8, patch_m=8.0, n_pulses=2, n_freq=16, n_points=1))
    kw = library_kwargs(wl)
    kw["n_x"] = 0
    write_problem(tmp_path / "bad.bin", kw, 5, [0], np.zeros((1, 16), np.complex64))
    r = subprocess.run([str(exe), str(tmp_path / "bad.bin"), str(tmp_path / "o.bin")],
                       capture_output=True, text=True)
    assert r.returncode == 2 and "invalid configuration" in r.stderr


def test_read_ceiling_builds_and_rejects_bad_sizes():
    """The plain streaming-read reference (tests/c/read_ceiling.hip) is built by
    the package build and checks its arguments before any GPU call."""
    exe = ROOT / "tests" / "c" / "read_ceiling"
    if not exe.exists():
        pytest.skip("read_ceiling not built")
    for bad in (["-5"], ["0"], ["0.0001"], ["x"], ["70000"], ["--tiles"], ["--tiles", "10"],
                ["--tiles", "40000"]):
        r = subprocess.run([str(exe), *bad], capture_output=True, text=True)
        assert r.returncode == 2 and "usage" in r.stderr, bad


@pytest.mark.gpu
def test_read_ceiling_runs():
    """One small size through every launch shape (a smoke run of the timing
    program that profiles/read-ceiling.md comes from)."""
    exe = ROOT / "tests" / "c" / "read_ceiling"
    if not exe.exists():
        pytest.skip("read_ceiling not built")
    r = subprocess.run([str(exe), "8"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    lines = [ln for ln in r.stdout.splitlines() if "GB/s" in ln]
    assert len(lines) == 10 and r.stdout.strip().endswith("done")
    # the tile-pattern read on a ragged tile count (M = 200: 4 tile rows, 10 tiles)
    r = subprocess.run([str(exe), "--tiles", "200"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    lines = [ln for ln in r.stdout.splitlines() if "GB/s" in ln]
    assert len(lines) == 2 and all("6 work items" in ln for ln in lines), r.stdout


@pytest.mark.gpu
@pytest.mark.parametrize("dictionary", ["identity", "haar"])
def test_driver_matches_binding_and_oracle(tmp_path, dictionary):
    torch = pytest.importorskip("torch")
    from paper_2603_08582_amd import OnlineFista
    if not DRIVER.exists():
        pytest.fail("tests/c/ofista_run is not built (run the package build)")
    extra = dict(dictionary="haar", haar_levels=2) if dictionary == "haar" else {}
    wl = make_workload(spec("small", n_side=32, patch_m=30.0, n_pulses=10, n_freq=64,
                            n_points=6, **extra))
    d = sar.echoes(wl).astype(np.complex64)
    order = [0, 2, 3, 5, 6, 7, 9]
    iters = 15
    kw = library_kwargs(wl)
    write_problem(tmp_path / "p.bin", kw, iters, order, d[order])
    print(f"C driver: {dictionary}, 32x32, K=64, {len(order)} pulses", flush=True)
    r = subprocess.run([str(DRIVER), str(tmp_path / "p.bin"), str(tmp_path / "img.bin")],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    img_c = np.fromfile(tmp_path / "img.bin", np.complex64)

    g = OnlineFista(**kw)
    dd = torch.from_numpy(d).cuda()
    o = OnlineFistaOracle.from_workload(wl)
    for s in order:
        g.push_pulse(dd[s], s)
        g.reconstruct(iters, copy=False)
        o.push_pulse(d[s].astype(np.complex128), s)
        o.reconstruct(iters)
    img_py = g.image().cpu().numpy()
    assert np.array_equal(img_c.view(np.uint32), img_py.view(np.uint32))
    ref = o.image()
    err = np.linalg.norm(img_c.astype(np.complex128) - ref) / np.linalg.norm(ref)
    assert err < 1e-4, err
    emax = np.max(np.abs(img_c.astype(np.complex128) - ref)) / np.max(np.abs(ref))
    assert emax < 1e-4, emax  # element by element against the largest magnitude
