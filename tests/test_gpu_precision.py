"""Precision form: split-BF16 Gram update against FP32 and the FP64 oracle.

Error model: hi = bf16(x), lo = bf16(x - hi) keeps ~16 significant bits of
each FP32 component; the three products hi*hi + hi*lo + lo*hi drop lo*lo
(relative 2^-16 of a product) and the representation residual (~2^-17), so a
Gram entry carries a relative error of order 1e-5 of its scale (n K for unit
phasors).  The stated tolerance for split-BF16 images is 1e-3 relative L2.
"""

import numpy as np
import pytest

from oracle import sar
from oracle.online_fista import OnlineFistaOracle
from workload import library_kwargs, make_workload, spec

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_split_bf16_small_against_oracle():
    from paper_2603_08582_amd import OnlineFista
    wl = make_workload(spec("small", n_side=32, patch_m=30.0, n_pulses=12, n_freq=64,
                            n_points=6, precision="split_bf16"))
    d = sar.echoes(wl).astype(np.complex64)
    g = OnlineFista(**library_kwargs(wl))
    o = OnlineFistaOracle.from_workload(wl)
    dd = torch.from_numpy(d).cuda()
    for p in range(wl.spec.n_pulses):
        g.push_pulse(dd[p], p)
        o.push_pulse(d[p].astype(np.complex128), p)
        g.reconstruct(20, copy=False)
        o.reconstruct(20)
    H = g.gram().cpu().numpy().astype(np.complex128)
    eH = rel(H, o.H)
    x = g.image().cpu().numpy().astype(np.complex128)
    ex = rel(x, o.image())
    print(f"split-BF16 32x32: Gram rel err {eH:.2e}, image rel err {ex:.2e}")
    assert eH < 2e-5
    assert ex < 1e-3
    assert rel(g.vector("b").cpu().numpy(), o.b) < 1e-6  # b stays FP32


def test_split_bf16_rejects_ragged_frequency_count():
    from paper_2603_08582_amd import OfistaError, OnlineFista
    wl = make_workload(spec("small", n_freq=50, precision="split_bf16"))
    with pytest.raises(OfistaError) as e:
        OnlineFista(**library_kwargs(wl))
    assert e.value.status == -5


def test_xlarge_split_bf16_against_fp32_run():
    """256x256 pixels, K = 1024, H = 17.2 GB of upper tiles; 16 pulses of the
    512-pulse trajectory, 10 FISTA steps each: split-BF16 run vs FP32 run on
    the same GPU, plus sampled Gram entries vs direct FP64 sums."""
    from paper_2603_08582_amd import OnlineFista
    wl = make_workload("xlarge")
    s = wl.spec
    pulses = list(range(0, s.n_pulses, s.n_pulses // 16))[:16]
    d = sar.echoes(wl, pulses=pulses).astype(np.complex64)
    dd = torch.from_numpy(d).cuda()
    images = {}
    samples = {}
    rng = np.random.default_rng(7)
    ii = rng.integers(0, s.n_pixels, 8)
    jj = np.minimum(ii + rng.integers(0, 3000, 8), s.n_pixels - 1)
    ii[:2] = jj[:2]
    pix = wl.pixel_xyz()
    f = wl.freqs()
    ref = np.array([sum(np.vdot(F[:, 0], F[:, 1]) for F in
                        (sar.forward_rows(wl.positions[p], pix[[i, j]], f) for p in pulses))
                    for i, j in zip(ii, jj)])
    scale = len(pulses) * s.n_freq
    for prec in ("split_bf16", "fp32"):
        g = OnlineFista(**library_kwargs(wl, precision=prec))
        for p in pulses:
            g.push_pulse(dd[p], p)
            g.reconstruct(s.inner_steps, copy=False)
        images[prec] = g.image().cpu().numpy().astype(np.complex128)
        st = g.state()
        assert st["n_pulses"] == len(pulses)
        samples[prec] = st
        ent = g.gram_entries(ii, jj).cpu().numpy().astype(np.complex128)
        e = np.max(np.abs(ent - ref)) / scale
        print(f"xlarge {prec}: sampled Gram entries, max error / (nK) = {e:.2e}")
        assert e < (2e-5 if prec == "split_bf16" else 2e-6)
        del g
        torch.cuda.empty_cache()
    err = rel(images["split_bf16"], images["fp32"])
    print(f"xlarge split-BF16 vs FP32 image: {err:.2e}")
    assert err < 1e-3
    assert np.all(np.isfinite(images["split_bf16"]))
    assert abs(samples["split_bf16"]["L"] / samples["fp32"]["L"] - 1) < 1e-4
