"""Discretised SAR forward model in FP64 (test infrastructure).

Section II models the echo as a Fourier integral operator with amplitude
A = 1 and phase phi = t - (2/c)|gamma(s_n) - x|; after discretisation
d_n = F rho + eps_n.  Over a stepped-frequency grid f_k the kernel of F at
pulse s and pixel i is the two-way delay term

    F_s[k, i] = exp(-i * 4 pi f_k R_{s,i} / c0),   R_{s,i} = |gamma(s) - x_i|_2

(the overall sign convention does not change |image|: conjugating both the
kernel and the data conjugates the coefficients).  Range and phase are kept
in float64 throughout.

Pinned by: |F| = 1 exactly; a 50-digit mpmath evaluation of the phase for
sample elements; the conjugation and global-phase symmetries of the full run.
"""

from __future__ import annotations

import math

import numpy as np

C0 = 299_792_458.0  # speed of light in vacuum, m/s


def ranges(position: np.ndarray, pixel_xyz: np.ndarray) -> np.ndarray:
    """R_i = |gamma(s) - x_i|_2 for every pixel, float64."""
    diff = pixel_xyz - np.asarray(position, dtype=np.float64)[None, :]
    return np.sqrt(np.sum(diff * diff, axis=1))


def forward_rows(position, pixel_xyz, freqs, sign: int = -1) -> np.ndarray:
    """F_s (K x N complex128): exp(sign * i * 4 pi f_k R_i / c0)."""
    R = ranges(position, pixel_xyz)
    phase = (4.0 * math.pi / C0) * np.outer(np.asarray(freqs, np.float64), R)
    return np.exp(sign * 1j * phase)


def clean_echo(position, pixel_xyz, freqs, rho, support=None, sign: int = -1):
    """F_s rho for one pulse (K complex128); only the support columns are used."""
    if support is None:
        support = np.flatnonzero(rho)
    if len(support) == 0:
        return np.zeros(len(freqs), dtype=np.complex128)
    F = forward_rows(position, pixel_xyz[support], freqs, sign)
    return F @ rho[support]


def echoes(wl, sign: int = -1, with_noise: bool = True,
           with_phase_error: bool = True, pulses=None) -> np.ndarray:
    """Synthetic radar returns for the pulses of a workload (P x K complex128;
    rows not listed in `pulses`, when given, stay zero).

    d_s = exp(i phi_s) F_s rho + sigma_s eps_s, with eps_s the workload's
    unit-variance complex draws and sigma_s^2 = (|F_s rho|^2 / K) 10^(-SNR/10),
    i.e. the per-pulse SNR is the stated power ratio.
    """
    s = wl.spec
    pix = wl.pixel_xyz()
    f = wl.freqs()
    P, K = s.n_pulses, s.n_freq
    d = np.zeros((P, K), dtype=np.complex128)
    for p in (range(P) if pulses is None else pulses):
        clean = clean_echo(wl.positions[p], pix, f, wl.rho, wl.support, sign)
        if with_phase_error:
            clean = clean * np.exp(1j * wl.phase_err[p])
        if with_noise:
            sigma2 = (np.vdot(clean, clean).real / K) * 10.0 ** (-s.snr_db / 10.0)
            clean = clean + math.sqrt(sigma2) * wl.noise[p]
        d[p] = clean
    return d
