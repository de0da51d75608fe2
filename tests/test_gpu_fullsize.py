"""Full-size GPU checks at the benchmark workloads' real shapes.

* haar64 (64x64 pixels, Haar(3), K=256, 128 pulses, m=20), run exactly as
  bench.py runs it, against the oracle's stored result (written by
  tests/golden/make_golden.py, which calls only the oracle): final image
  within the FP32 image tolerance 1e-4, every L_n and lambda within 1e-6.
* large (128x128 pixels, K=512, 256 pulses, m=20, 200 scatterers over a
  40 dB range) against the oracle's stored result (tests/golden/
  large_oracle.npz, same script): the image within 1e-4 relative L2 and
  element by element within 1e-3 of max |x|, the support of c outside a band
  of 1e-3 max |c| on both sides, every L_n and lambda within 1e-6; plus
  sampled entries the oracle computes one by one -- H_n[i, j] and b_n[i] as
  direct FP64 sums over pulses and frequencies, sigma^2 of sample positions,
  and lambda from the first pulse.
"""

from pathlib import Path

import numpy as np
import pytest

from oracle import sar
from oracle.online_fista import spectral_norm_sq
from workload import library_kwargs, make_workload

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = Path(__file__).resolve().parent / "golden"


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_haar64_full_run_matches_stored_oracle():
    from paper_2603_08582_amd import OnlineFista
    ref = np.load(GOLDEN / "haar64_oracle.npz")
    wl = make_workload("haar64")
    d = sar.echoes(wl).astype(np.complex64)
    g = OnlineFista(**library_kwargs(wl))
    dd = torch.from_numpy(d).cuda()
    Ls, lams = [], []
    for p in range(wl.spec.n_pulses):
        g.push_pulse(dd[p], p)
        st = g.state()
        Ls.append(st["L"])
        lams.append(st["lam"])
        g.reconstruct(wl.spec.inner_steps, copy=False)
    x = g.image().cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(np.array(Ls) / ref["L"] - 1)) < 1e-6
    assert np.max(np.abs(np.array(lams) / ref["lam"] - 1)) < 1e-6
    err = rel(x, ref["image"])
    emax = float(np.max(np.abs(x - ref["image"])) / np.max(np.abs(ref["image"])))
    print(f"haar64 full run: relative image error {err:.3e}, largest pixel error {emax:.3e} of max |x|")
    assert err < 1e-4
    # element by element at the same tolerance against the largest magnitude
    assert emax < 1e-4
    assert abs(g.state()["t"] - float(ref["t"])) < 1e-9 * float(ref["t"])


def direct_gram_entry(wl, pix, i, j, pulses):
    """H_n[i, j] = sum_s sum_k conj(F_s[k, i]) F_s[k, j] in FP64."""
    f = wl.freqs()
    tot = 0j
    for s in range(pulses):
        F = sar.forward_rows(wl.positions[s], pix[[i, j]], f)
        tot += np.vdot(F[:, 0], F[:, 1])
    return tot


def direct_b_entry(wl, pix, d, i, pulses):
    f = wl.freqs()
    tot = 0j
    for s in range(pulses):
        F = sar.forward_rows(wl.positions[s], pix[[i]], f)
        tot += np.vdot(F[:, 0], d[s])
    return tot


def test_large_full_run_against_oracle():
    from paper_2603_08582_amd import OnlineFista
    wl = make_workload("large")
    s = wl.spec
    N, K, P = s.n_pixels, s.n_freq, s.n_pulses
    d = sar.echoes(wl).astype(np.complex64)
    g = OnlineFista(**library_kwargs(wl))
    dd = torch.from_numpy(d).cuda()
    Ls, lams = [], []
    for p in range(P):
        g.push_pulse(dd[p], p)
        st = g.state()
        Ls.append(st["L"])
        lams.append(st["lam"])
        g.reconstruct(s.inner_steps, copy=False)
    lam = lams[0]
    st = g.state()
    assert st["n_pulses"] == P and st["n_iters"] == P * s.inner_steps
    # the whole run against the oracle's stored result
    ref = np.load(GOLDEN / "large_oracle.npz")
    assert np.max(np.abs(np.array(Ls) / ref["L"] - 1)) < 1e-6
    assert np.max(np.abs(np.array(lams) / ref["lam"] - 1)) < 1e-6
    assert abs(st["t"] - float(ref["t"])) < 1e-9 * float(ref["t"])
    x = g.image().cpu().numpy().astype(np.complex128)
    xo = ref["image"]
    err = rel(x, xo)
    emax = float(np.max(np.abs(x - xo)) / np.max(np.abs(xo)))
    c = g.vector("c").cpu().numpy().astype(np.complex128)
    co = ref["c"]
    band = 1e-3 * np.max(np.abs(co))
    sup = wl.support
    found_o = int(np.count_nonzero(np.abs(co[sup]) > band))
    found_g = int(np.count_nonzero(np.abs(c[sup]) > band))
    print(f"large full run: image rel {err:.3e}, max element {emax:.3e}; scatterer pixels "
          f"above the band: oracle {found_o}, GPU {found_g} of {len(sup)}")
    assert err < 1e-4 and emax < 1e-3
    # support outside the band: what one side holds above it, the other holds too
    assert np.all(c[np.abs(co) > band] != 0)
    assert np.all(co[np.abs(c) > band] != 0)
    pix = wl.pixel_xyz()
    d64 = d.astype(np.complex128)
    # lambda from the first pulse
    F0 = sar.forward_rows(wl.positions[0], pix, wl.freqs())
    lam_ref = s.lambda_rel * np.max(np.abs(F0.conj().T @ d64[0]))
    assert abs(lam / lam_ref - 1) < 1e-6
    # sampled Gram and correlation entries
    rng = np.random.default_rng(5)
    ii = rng.integers(0, N, 24)
    jj = rng.integers(0, N, 24)
    ii[:4] = jj[:4]  # a few diagonal entries
    Hs = g.gram_entries(ii, jj).cpu().numpy()
    Hd = g.gram()  # the dense expansion agrees with the packed entries
    assert np.array_equal(Hd[torch.from_numpy(ii).cuda(), torch.from_numpy(jj).cuda()].cpu().numpy(), Hs)
    del Hd
    torch.cuda.empty_cache()
    scale = P * K
    for n, (i, j) in enumerate(zip(ii, jj)):
        ref = direct_gram_entry(wl, pix, int(i), int(j), P)
        assert abs(Hs[n] - ref) <= 2e-6 * scale, (i, j, Hs[n], ref)
    b = g.vector("b").cpu().numpy()
    bscale = np.max(np.abs(b))
    for i in ii[:12]:
        ref = direct_b_entry(wl, pix, d64, int(i), P)
        assert abs(b[i] - ref) <= 2e-6 * bscale
    # sigma^2 of sample positions, from the state after pushing them again
    for pos in (0, P // 2, P - 1):
        F = sar.forward_rows(wl.positions[pos], pix, wl.freqs())
        ref = spectral_norm_sq(F)
        g.push_pulse(dd[pos], pos)
        # FP64 on both sides; the oracle's F F^H carries ~4e-10 relative
        # rounding from its ~4e6 rad phases
        assert abs(g.state()["sigma2"] / ref - 1) < 3e-9
    assert np.all(np.isfinite(g.image().cpu().numpy()))
