"""Collection session of Section IV-A on the GPU library (host-side driver).

The platform passes linearly spaced positions and sends a pulse at position s
when its Bernoulli trial succeeds (uniform draw u_s < p).  Each received pulse
goes through ofista_push_pulse and m FISTA steps; after it the library counts
the large coefficients (|c| > threshold, Section IV-B) and the session stops at
the first pulse whose count equals the scene's ideal count, if one is given.
The random draws are inputs; this module only sequences library calls.
"""

from __future__ import annotations

import math

import numpy as np


def bernoulli_schedule(u, p: float) -> np.ndarray:
    """Positions that transmit: indices s with u[s] < p, in trajectory order."""
    return np.flatnonzero(np.asarray(u, dtype=np.float64) < p)


def run_session(model, pulses, schedule, m: int, ideal: int = 0, threshold: float = 2e-2,
                after_pulse=None) -> dict:
    """Push pulses[s] for s in schedule (each followed by m FISTA steps) until
    the large-coefficient count equals `ideal` (0: never stop early).

    pulses: device tensor indexed by position (positions x K, complex64).
    after_pulse(k, s, count), if given, runs after each pulse.
    Returns pushed positions, the count after each pulse, and the stop index
    (None when the schedule ran out first)."""
    pushed, counts, stop = [], [], None
    for s in schedule:
        s = int(s)
        model.push_pulse(pulses[s], s)
        model.reconstruct(int(m), copy=False)
        count = model.count_large(threshold)
        pushed.append(s)
        counts.append(count)
        if after_pulse is not None:
            after_pulse(len(pushed) - 1, s, count)
        if ideal > 0 and count == ideal:
            stop = len(pushed) - 1
            break
    return {"pushed": pushed, "counts": counts, "stop": stop}


def to_db(x):
    """20 log10 |x|, BP's display scale (host array in, host array out)."""
    with np.errstate(divide="ignore"):
        return 20.0 * np.log10(np.abs(np.asarray(x)))


def snr_db(x, support) -> float:
    """Section IV-B SNR of an image: 20 log10(mu_signal / mu_noise), mu the mean
    |x|^2 over the true support and over the other pixels (host arrays)."""
    x = np.asarray(x)
    mask = np.zeros(x.size, dtype=bool)
    mask[np.asarray(support)] = True
    mu_s = float(np.mean(np.abs(x[mask]) ** 2))
    mu_n = float(np.mean(np.abs(x[~mask]) ** 2)) if (~mask).any() else 0.0
    return math.inf if mu_n == 0.0 else 20.0 * math.log10(mu_s / mu_n)
