"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, sizes workspaces consistently and rejects bad arguments with the
documented status codes before touching the device."""

import ctypes
import re
from pathlib import Path

import numpy as np
import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "ofista.h"
LIB = ROOT / "paper_2603_08582_amd" / "libofista.so"

pytestmark = pytest.mark.skipif(not LIB.exists(), reason="libofista.so not built")


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ofista_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    from paper_2603_08582_amd import ofista
    L = ofista.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def small_cfg(**kw):
    from paper_2603_08582_amd import ofista
    from workload import library_kwargs, make_workload
    wl = make_workload("small")
    args = library_kwargs(wl)
    args.update(kw)
    return ofista.make_config(**args)


def test_workspace_size_covers_packed_gram():
    from paper_2603_08582_amd import ofista
    cfg, keep = small_cfg()
    nbytes = ofista.workspace_bytes(cfg)
    nb = 1024 // 64
    packed = nb * (nb + 1) // 2 * 64 * 64 * 8
    assert nbytes >= packed + 64 * 1024 * 8
    assert nbytes % 256 == 0 or nbytes > 0
    assert ofista.lib().ofista_tile() == 64


@pytest.mark.parametrize("field,value,status", [
    ("n_x", 0, -1), ("n_freq", 0, -1), ("n_freq", 4096, -1), ("dict", 7, -1),
    ("precision", 9, -1), ("lipschitz", 5, -1), ("momentum", 4, -1), ("lambda_", -1.0, -1),
    ("record_every", -2, -1),
])
def test_bad_config_rejected(field, value, status):
    from paper_2603_08582_amd import ofista
    cfg, keep = small_cfg()
    setattr(cfg, field, value)
    assert ofista.check_config(cfg) == status
    assert ofista.workspace_bytes(cfg) == 0


def test_haar_constraints():
    from paper_2603_08582_amd import ofista
    cfg, keep = small_cfg(dictionary="haar", haar_levels=3)
    assert ofista.check_config(cfg) == 0
    cfg.haar_levels = 6  # 32 not divisible by 64
    assert ofista.check_config(cfg) == -1
    cfg2, keep2 = small_cfg(dictionary="haar", haar_levels=1, n_x=128, n_y=128)
    assert ofista.check_config(cfg2) == -5  # N > 8192 unsupported for Haar


def test_create_rejects_missing_workspace_without_gpu():
    from paper_2603_08582_amd import ofista
    L = ofista.lib()
    cfg, keep = small_cfg()
    out = ctypes.c_void_p()
    st = L.ofista_create(ctypes.byref(cfg), None, 0, None, ctypes.byref(out))
    assert st == -4 and not out.value
    # misaligned pointer is rejected before any device access
    st = L.ofista_create(ctypes.byref(cfg), ctypes.c_void_p(0x1001), 1 << 40, None, ctypes.byref(out))
    assert st == -4
    assert L.ofista_create(ctypes.byref(cfg), None, 0, None, None) == -1


def test_null_ctx_and_error_strings():
    from paper_2603_08582_amd import ofista
    L = ofista.lib()
    assert L.ofista_reset(None) == -1
    assert L.ofista_push_pulse(None, None, 0, 0.0) == -1
    assert L.ofista_reconstruct(None, 1, None) == -1
    assert L.ofista_reconstruct_static(None, 1, None) == -1
    L.ofista_destroy(None)
    for st in (0, -1, -2, -3, -4, -5, -6):
        assert L.ofista_error_string(None, st)
    assert L.ofista_workspace_bytes(None) == 0


def test_state_bytes_grows_with_problem():
    from paper_2603_08582_amd import ofista
    L = ofista.lib()
    a, ka = small_cfg()
    b, kb = small_cfg(n_x=64, n_y=64)
    sa = L.ofista_state_bytes(ctypes.byref(a))
    sb = L.ofista_state_bytes(ctypes.byref(b))
    assert 0 < sa < sb
    assert sb >= (64 * 64 // 64) * (64 * 64 // 64 + 1) // 2 * 64 * 64 * 8


def edgelet_cfg(n=10, lengths=(4,), rotations=(0.0, 90.0), **kw):
    from paper_2603_08582_amd import ofista
    from workload import library_kwargs, make_workload, spec
    wl = make_workload(spec("small", n_side=n, patch_m=float(n), n_freq=16, n_points=2))
    args = library_kwargs(wl, dictionary="edgelet", edge_lengths=lengths, edge_rotations=rotations)
    args.update(kw)
    return ofista.make_config(**args)


@pytest.mark.parametrize("n,l", [(10, 4), (16, 2), (12, 5)])
def test_edgelet_coefficient_count_closed_form(n, l):
    """Axis-aligned atoms of l consecutive pixels: n (n - l + 1) per rotation."""
    from paper_2603_08582_amd import ofista
    cfg, keep = edgelet_cfg(n, (l,), (0.0, 90.0))
    assert ofista.coef_count(cfg) == 2 * n * (n - l + 1)
    one, keep1 = edgelet_cfg(n, (1,), (0.0,))
    assert ofista.coef_count(one) == n * n


def test_edgelet_counts_match_the_oracle_on_oblique_atoms():
    from oracle import dictionary
    from paper_2603_08582_amd import ofista
    lens, rots = (2, 3, 5), (0.0, 30.0, 45.0, 100.0, 135.0)
    cfg, keep = edgelet_cfg(12, lens, rots)
    assert ofista.coef_count(cfg) == len(dictionary.edgelet_atoms(12, lens, rots))


@pytest.mark.parametrize("kw", [
    dict(edge_lengths=(0,)), dict(edge_lengths=(10,)), dict(edge_lengths=()),
    dict(edge_rotations=()), dict(edge_rotations=(float("nan"),)),
])
def test_bad_edgelet_config_rejected(kw):
    from paper_2603_08582_amd import ofista
    cfg, keep = edgelet_cfg(10, **{"lengths": kw.get("edge_lengths", (4,)),
                                   "rotations": kw.get("edge_rotations", (0.0, 90.0))})
    assert ofista.check_config(cfg) == -1
    assert ofista.coef_count(cfg) == -1
    assert ofista.workspace_bytes(cfg) == 0


def test_edgelet_needs_a_square_grid():
    from paper_2603_08582_amd import ofista
    cfg, keep = edgelet_cfg(10)
    cfg.n_y = 8
    assert ofista.check_config(cfg) == -1


def test_edgelet_workspace_grows_with_the_atom_count():
    from paper_2603_08582_amd import ofista
    a, ka = edgelet_cfg(16, (4,), (0.0,))
    b, kb = edgelet_cfg(16, (4,), (0.0, 90.0))
    assert ofista.workspace_bytes(b) > ofista.workspace_bytes(a) > 0


def test_store_all_workspace_grows_with_capacity():
    """Store-all keeps n pulses (K x M complex64 rows each) instead of the M x M
    Gram: its workspace grows linearly with the capacity, by at least the
    K x M operator per pulse; the Gram mode fits in the FP32 bytes of Table
    I's Online FISTA count (it keeps only the upper triangle of H)."""
    from oracle import memory
    from paper_2603_08582_amd import ofista
    from workload import library_kwargs, make_workload, spec
    wl = make_workload(spec("small", n_side=32, patch_m=30.0, n_freq=64, n_points=2))
    gram, kg = ofista.make_config(**library_kwargs(wl))
    ws_gram = ofista.workspace_bytes(gram)
    assert ws_gram <= 4 * memory.online_values(1024, 1024)
    sizes = []
    for cap in range(1, 41):
        c, k = ofista.make_config(**library_kwargs(wl, storage="pulses", max_pulses=cap))
        sizes.append(ofista.workspace_bytes(c))
    steps = np.diff(sizes)
    assert np.all(steps >= 64 * 1024 * 8) and np.ptp(steps) <= 4096
    assert sizes[0] < ws_gram < sizes[-1]
    bad, kb = ofista.make_config(**library_kwargs(wl, storage="pulses", max_pulses=0))
    assert ofista.check_config(bad) == -1
    rec, kr = ofista.make_config(**library_kwargs(wl, storage="pulses", max_pulses=4,
                                                  record_every=2, max_iters=3))
    assert ofista.check_config(rec) == -5
