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


@pytest.mark.parametrize("layout", ["tile", "block"])
@pytest.mark.parametrize("shape", [dict(n_side=32, patch_m=30.0),      # 16 tile rows
                                   dict(n_side=30, patch_m=28.0)])     # 15: a partial block
def test_split_bf16_against_oracle(layout, shape):
    """Both workgroup layouts of the split-BF16 Gram against the oracle's dense
    H entry by entry (scale nK), and the image element by element."""
    from paper_2603_08582_amd import OnlineFista
    wl = make_workload(spec("small", n_pulses=12, n_freq=64, n_points=6,
                            precision="split_bf16", **shape))
    d = sar.echoes(wl).astype(np.complex64)
    g = OnlineFista(**library_kwargs(wl, gram_layout=layout))
    o = OnlineFistaOracle.from_workload(wl)
    dd = torch.from_numpy(d).cuda()
    for p in range(wl.spec.n_pulses):
        g.push_pulse(dd[p], p)
        o.push_pulse(d[p].astype(np.complex128), p)
        g.reconstruct(20, copy=False)
        o.reconstruct(20)
    H = g.gram().cpu().numpy().astype(np.complex128)
    nK = wl.spec.n_pulses * wl.spec.n_freq
    eH = float(np.max(np.abs(H - o.H))) / nK
    x = g.image().cpu().numpy().astype(np.complex128)
    xo = o.image()
    ex = rel(x, xo)
    ex_max = float(np.max(np.abs(x - xo)) / np.max(np.abs(xo)))
    print(f"split-BF16 {layout} {wl.spec.n_side}^2: max |dH|/(nK) {eH:.2e}, image rel "
          f"{ex:.2e}, max element {ex_max:.2e}")
    assert eH < 2e-5
    assert ex < 1e-3 and ex_max < 1e-3
    assert np.all(np.diag(H).imag == 0)
    assert rel(g.vector("b").cpu().numpy(), o.b) < 1e-6  # b stays FP32
    # support outside a band around the threshold: 1e-2 of the largest |c|
    band = 1e-2 * np.max(np.abs(o.c))
    c = g.vector("c").cpu().numpy()
    assert np.all(c[np.abs(o.c) > band] != 0)
    assert np.all(o.c[np.abs(c) > band] != 0)


def test_split_bf16_layouts_agree_bitwise_at_16384():
    """The 2 x 2-block and one-tile layouts form the same sums in the same
    order: H and the image agree bit for bit at N = 16384 (128 x 128 pixels,
    K = 512, 256 tile rows)."""
    from paper_2603_08582_amd import OnlineFista
    wl = make_workload(spec("large", precision="split_bf16"))
    pulses = [0, 85, 170]
    d = torch.from_numpy(sar.echoes(wl, pulses=pulses).astype(np.complex64)).cuda()
    out = {}
    for layout in ("tile", "block"):
        g = OnlineFista(**library_kwargs(wl, gram_layout=layout))
        for p in pulses:
            g.push_pulse(d[p], p)
            g.reconstruct(3, copy=False)
        out[layout] = (g.gram(), g.image())
        del g
        torch.cuda.empty_cache()
    assert torch.equal(out["tile"][0].view(torch.float32), out["block"][0].view(torch.float32))
    assert torch.equal(out["tile"][1].view(torch.float32), out["block"][1].view(torch.float32))


def test_split_bf16_rejects_ragged_frequency_count():
    from paper_2603_08582_amd import OfistaError, OnlineFista
    wl = make_workload(spec("small", n_freq=50, precision="split_bf16"))
    with pytest.raises(OfistaError) as e:
        OnlineFista(**library_kwargs(wl))
    assert e.value.status == -5


def test_xlarge_split_bf16_against_fp32_run():
    """256x256 pixels, K = 1024, H = 17.2 GB of upper tiles; the whole
    512-pulse trajectory at 10 FISTA steps per pulse: split-BF16 run vs FP32
    run on the same GPU (1e-3 relative, and element by element against the
    largest |x|), plus sampled Gram entries vs direct FP64 sums over all
    pulses."""
    from paper_2603_08582_amd import OnlineFista
    wl = make_workload("xlarge")
    s = wl.spec
    pulses = list(range(s.n_pulses))
    d = sar.echoes(wl).astype(np.complex64)
    dd = torch.from_numpy(d).cuda()
    images, coefs, samples = {}, {}, {}
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
        print(f"xlarge {prec}: {len(pulses)} pulses", flush=True)
        g = OnlineFista(**library_kwargs(wl, precision=prec))
        for p in pulses:
            g.push_pulse(dd[p], p)
            g.reconstruct(s.inner_steps, copy=False)
        images[prec] = g.image().cpu().numpy().astype(np.complex128)
        coefs[prec] = g.vector("c").cpu().numpy()
        st = g.state()
        assert st["n_pulses"] == len(pulses)
        samples[prec] = st
        ent = g.gram_entries(ii, jj).cpu().numpy().astype(np.complex128)
        e = np.max(np.abs(ent - ref)) / scale
        print(f"xlarge {prec}: sampled Gram entries, max error / (nK) = {e:.2e}", flush=True)
        assert e < (2e-5 if prec == "split_bf16" else 2e-6)
        del g
        torch.cuda.empty_cache()
    xb, xf = images["split_bf16"], images["fp32"]
    err = rel(xb, xf)
    emax = float(np.max(np.abs(xb - xf)) / np.max(np.abs(xf)))
    print(f"xlarge split-BF16 vs FP32 image: {err:.2e} (max element {emax:.2e})")
    assert np.all(np.isfinite(xb))
    assert err < 1e-3 and emax < 1e-3
    band = 1e-2 * np.max(np.abs(coefs["fp32"]))
    assert np.all(coefs["split_bf16"][np.abs(coefs["fp32"]) > band] != 0)
    assert abs(samples["split_bf16"]["L"] / samples["fp32"]["L"] - 1) < 1e-4
