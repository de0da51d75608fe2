"""The resident step kernel (all FISTA steps of a reconstruct call in one
cooperative launch, grid barriers between the tile pass and the update of
every step) against the two-launches-per-step path: the same arithmetic in
the same order, so c, the power vector, rho, L and the image agree bit for
bit.  Shapes: one and several work items per workgroup (nb = 16 and the
64-tile-row haar64 grid), a ragged grid (30 x 30 pixels: a partial last tile
and a one-tile run), more than 64 steps in one call (several launches), the
three momentum modes, and the allocation-free entry point.
"""

import numpy as np
import pytest

from oracle import sar
from workload import library_kwargs, make_workload, spec

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def run(wl, d, mode, pulses, iters, static=False, **kw):
    from paper_2603_08582_amd import OnlineFista
    g = OnlineFista(**library_kwargs(wl, step_kernel=mode, **kw))
    for p in pulses:
        g.push_pulse(d[p], p)
        if static:
            g.reconstruct_static(iters, copy=False)
        else:
            g.reconstruct(iters, copy=False)
    st = g.state()
    out = dict(c=g.vector("c").cpu(), w=g.vector("w").cpu(), image=g.image().cpu(),
               L=st["L"], rho=st["rho"], t=st["t"], n_iters=st["n_iters"])
    del g
    torch.cuda.empty_cache()
    return out


def same(a, b):
    for k in ("c", "w", "image"):
        assert torch.equal(a[k].view(torch.float32), b[k].view(torch.float32)), k
    for k in ("L", "rho", "t", "n_iters"):
        assert a[k] == b[k], (k, a[k], b[k])


CASES = [
    ("small", dict(), [0, 5, 9], 20, {}),
    ("small", dict(n_side=30, patch_m=28.0), [0, 3, 7, 11], 20, {}),
    ("small", dict(), [0, 1], 70, {}),                       # two launches per call
    ("small", dict(), [0, 4, 8], 15, dict(momentum="restart")),
    ("small", dict(), [0, 4, 8], 15, dict(momentum="ista")),
    ("small", dict(), [0, 4, 8], 15, dict(lipschitz="bound")),
    ("haar64", dict(), [0, 40, 80, 127], 20, {}),
]


@pytest.mark.parametrize("name,over,pulses,iters,kw", CASES)
def test_resident_matches_launches_bitwise(name, over, pulses, iters, kw):
    wl = make_workload(spec(name, **over)) if over else make_workload(name)
    d = torch.from_numpy(sar.echoes(wl, pulses=pulses).astype(np.complex64)).cuda()
    print(f"{name} {over} pulses {pulses} iters {iters} {kw}", flush=True)
    a = run(wl, d, "launches", pulses, iters, **kw)
    b = run(wl, d, "resident", pulses, iters, **kw)
    same(a, b)
    assert b["n_iters"] == len(pulses) * iters
    assert np.all(np.isfinite(b["c"].numpy()))


def test_resident_static_entry_point():
    """The allocation-free entry point takes the resident path too (its
    partials in the static array) and agrees with ofista_reconstruct."""
    wl = make_workload("small")
    pulses = [0, 6, 12]
    d = torch.from_numpy(sar.echoes(wl, pulses=pulses).astype(np.complex64)).cuda()
    a = run(wl, d, "resident", pulses, 20)
    b = run(wl, d, "resident", pulses, 20, static=True)
    same(a, b)


def test_resident_profile_class():
    """With profiling on, the resident kernel is timed under its own class and
    the two per-step classes stay empty."""
    from paper_2603_08582_amd import OnlineFista
    wl = make_workload("small")
    d = torch.from_numpy(sar.echoes(wl, pulses=[0]).astype(np.complex64)).cuda()
    g = OnlineFista(**library_kwargs(wl, step_kernel="resident"))
    g.push_pulse(d[0], 0)
    g.profile(True)
    g.reconstruct(10, copy=False)
    ms, n = g.kernel_time("resident")
    ms_step, n_step = g.kernel_time("step")
    g.profile(False)
    assert n == 1 and ms > 0 and n_step == 0
