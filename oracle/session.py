"""Collection session of Section IV-A and the evaluation of Section IV-B
(test infrastructure).

Section IV-A: the platform passes linearly spaced positions; at each one a
Bernoulli trial with success probability p decides whether a pulse is sent
(the randomness compressive sensing asks for).  The uniforms u_s are inputs;
position s transmits when u_s < p.  After every received pulse Online FISTA
runs m steps; the run stops early once the number of large coefficients
(|c| > 2e-2, Section IV-B) equals the scene's ideal count.

Section IV-A also defines the baseline BP (backprojection): the average of the
adjoint-imaged pulses, (1/n) sum_k F_k^H d_k in the pixel domain, shown in dB
as 20 log10 of its magnitude.

Section IV-B's SNR is 20 log10(mu_signal / mu_noise) with mu the power of
signal and noise (printed that way, although both are powers): here mu_signal
is the mean |x|^2 over the true scene support and mu_noise the mean |x|^2
over the remaining pixels.

Pinned by: backprojection of a noiseless single scatterer equals K rho at its
pixel; with W = I it equals b_n / n; p = 1 selects every position and the
session equals the plain run; the stop index is the first pulse whose count
equals the ideal; SNR closed forms.
"""

from __future__ import annotations

import math

import numpy as np

from . import sar
from .online_fista import OnlineFistaOracle


def bernoulli_positions(u, p: float) -> np.ndarray:
    """Indices s with u_s < p, in trajectory order."""
    return np.flatnonzero(np.asarray(u, np.float64) < p)


def large_count(c, thresh: float = 2e-2) -> int:
    return int(np.count_nonzero(np.abs(c) > thresh))


def backprojection(wl, d, pulses, sign: int = -1) -> np.ndarray:
    """(1/n) sum over the given pulses of F_s^H d_s (pixel domain)."""
    pix = wl.pixel_xyz()
    acc = np.zeros(pix.shape[0], np.complex128)
    for s in pulses:
        F = sar.forward_rows(wl.positions[s], pix, wl.freqs(), sign)
        acc += F.conj().T @ np.asarray(d[s], np.complex128)
    return acc / max(len(pulses), 1)


def to_db(x) -> np.ndarray:
    """20 log10 |x| (BP's display scale); -inf where x = 0."""
    with np.errstate(divide="ignore"):
        return 20.0 * np.log10(np.abs(x))


def snr_db(x, support) -> float:
    x = np.asarray(x)
    mask = np.zeros(x.size, bool)
    mask[np.asarray(support)] = True
    mu_s = float(np.mean(np.abs(x[mask]) ** 2))
    mu_n = float(np.mean(np.abs(x[~mask]) ** 2)) if (~mask).any() else 0.0
    if mu_n == 0.0:
        return math.inf
    return 20.0 * math.log10(mu_s / mu_n)


def run_session(wl, d=None, p=None, m=None, ideal=None, thresh=None, **kw):
    """Online FISTA over the Bernoulli-selected positions, stopping early at
    the ideal large-coefficient count.  Returns (oracle, pushed positions,
    count after each pushed pulse, stop index or None)."""
    s = wl.spec
    p = s.bernoulli_p if p is None else p
    m = s.inner_steps if m is None else m
    ideal = s.ideal_count if ideal is None else ideal
    ideal = ideal if ideal and ideal > 0 else None   # 0: run to the end
    thresh = s.large_thresh if thresh is None else thresh
    if d is None:
        d = sar.echoes(wl)
    o = OnlineFistaOracle.from_workload(wl, **kw)
    pushed, counts, stop = [], [], None
    for pos in bernoulli_positions(wl.select_u, p):
        o.push_pulse(d[pos], int(pos))
        o.reconstruct(m)
        pushed.append(int(pos))
        counts.append(large_count(o.c, thresh))
        if ideal is not None and counts[-1] == ideal:
            stop = len(pushed) - 1
            break
    return o, pushed, counts, stop
