"""The allocation-free entry point ofista_reconstruct_static against
ofista_reconstruct, through the C ABI.

Both run the same kernels in the same order; only the home of the matvec
partials differs (the library's per-GPU static array instead of the ctx's
workspace), so the coefficients must agree bit for bit.  Two calls in a row
share the static array, the second with a smaller problem.
"""

import numpy as np
import pytest

from oracle import sar
from workload import library_kwargs, make_workload, spec

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _pair(wl, **kw):
    from paper_2603_08582_amd import OnlineFista
    return (OnlineFista(**library_kwargs(wl, **kw)), OnlineFista(**library_kwargs(wl, **kw)))


def _run(n_side, n_freq, pulses, m, dictionary="identity"):
    s = spec("small", n_side=n_side, patch_m=float(n_side), n_pulses=pulses, n_freq=n_freq,
             n_points=5)
    if dictionary == "haar":
        s = spec("haar64", n_side=n_side, patch_m=float(n_side), n_pulses=pulses,
                 n_freq=n_freq, n_points=5, n_lines=1)
    wl = make_workload(s)
    print(f"no-alloc case: {n_side}x{n_side} {dictionary} K={n_freq} pulses={pulses} m={m}",
          flush=True)
    d = torch.from_numpy(sar.echoes(wl).astype(np.complex64)).cuda()
    ref, st = _pair(wl)
    out_ref = torch.empty(ref.M, dtype=torch.complex64, device="cuda")
    out_st = torch.empty(st.M, dtype=torch.complex64, device="cuda")
    for p in range(pulses):
        ref.push_pulse(d[p], p)
        st.push_pulse(d[p], p)
        ref.reconstruct(m, out=out_ref)
        st.reconstruct_static(m, out=out_st)
        torch.cuda.synchronize()
        a, b = out_ref.cpu().numpy(), out_st.cpu().numpy()
        assert np.all(np.isfinite(a))
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), p
    assert st.state()["n_iters"] == pulses * m
    xr, xs = ref.image().cpu().numpy(), st.image().cpu().numpy()
    assert np.array_equal(xr.view(np.uint32), xs.view(np.uint32))
    assert np.abs(xr).max() > 0


def test_static_partials_match_workspace_partials_large_then_small():
    # 48 x 48 (36 tile rows, 1.3 MiB of partials), then 16 x 16 (4 tile rows)
    _run(48, 64, 4, 20)
    _run(16, 32, 5, 20)


def test_static_partials_near_the_largest_supported_size():
    # 90 x 90 pixels: 127 tile rows, 15.75 of the 16 MiB; then a Haar case
    _run(90, 32, 2, 3)
    _run(32, 64, 3, 20, dictionary="haar")


def test_static_partials_reject_oversize_and_pulses_storage():
    from paper_2603_08582_amd import OnlineFista, OfistaError
    wl = make_workload(spec("small", n_side=96, patch_m=96.0, n_pulses=1, n_freq=32,
                            n_points=2))
    g = OnlineFista(**library_kwargs(wl))
    d = torch.from_numpy(sar.echoes(wl).astype(np.complex64)).cuda()
    g.push_pulse(d[0], 0)
    with pytest.raises(OfistaError) as e:
        g.reconstruct_static(1, copy=False)
    assert e.value.status == -5 and "16 MiB" in str(e.value)
    g.reconstruct(1, copy=False)  # the ordinary entry point still serves it
    ws = make_workload(spec("small", n_side=16, patch_m=16.0, n_pulses=2, n_freq=32))
    gs = OnlineFista(**library_kwargs(ws, storage="pulses", max_pulses=2))
    ds = torch.from_numpy(sar.echoes(ws).astype(np.complex64)).cuda()
    gs.push_pulse(ds[0], 0)
    with pytest.raises(OfistaError) as e:
        gs.reconstruct_static(1, copy=False)
    assert e.value.status == -5
