"""Workload specifications and seeded input draws.

The five named workloads follow the experiment description of the paper's
Section IV-A in spirit (monostatic spotlight collection, point and line targets,
m inner steps per pulse) at the sizes of the five benchmark configurations:

  ``small``      32x32 pixels,   32 pulses over 10 deg,  K=64,   identity, 20 dB
  ``haar64``     64x64 pixels,  128 pulses over 20 deg,  K=256,  Haar(3),  30 dB
  ``autofocus``  64x64 pixels,   64 pulses over 20 deg,  K=256,  identity, phase errors
  ``large``     128x128 pixels, 256 pulses over 30 deg,  K=512,  identity, 40 dB range
  ``xlarge``    256x256 pixels, 512 pulses over 40 deg,  K=1024, identity, split-BF16
  ``edgelet64``  64x64 pixels,  128 pulses over 20 deg,  K=256,  edgelets (length 4,
                 0 and 90 deg), scene of axis-aligned segments
  ``session32``  32x32 pixels, 1000 candidate positions over 2 deg at 4 km (the
                 collection of Section IV-A), Bernoulli pulse selection, K=64,
                 edgelets (length 4, 0 and 90 deg), one square target

Readings of details the paper leaves open:

* pixel grid is cell-centred on a flat (z = 0) patch centred at the origin;
  pixel (iy, ix) sits at (-W/2 + (ix + 1/2) dx, -W/2 + (iy + 1/2) dx, 0) and has
  flat index iy * n + ix;
* the platform flies a circle of horizontal radius 10 km at 1 km altitude; pulse
  s sits at azimuth theta_s = s * span / (P - 1), s = 0 .. P-1;
* frequencies are evenly spaced with inclusive end points,
  f_k = f_lo + k (f_hi - f_lo) / (K - 1);
* a line target is sampled every pixel spacing along its length, each sample is
  snapped to the nearest pixel centre (duplicates removed) and the whole line
  carries one complex reflectivity; overlapping targets add;
* a segment target is an axis-aligned run of pixels (horizontal or vertical
  with probability 1/2, length drawn from ``segment_px``, start uniform among
  the positions that keep it on the grid) carrying one complex reflectivity;
* a square target is the outline of a ``square_px``-pixel square (its four
  sides, each a run of ``square_px`` pixels, added up, so corners count twice)
  with one complex reflectivity, placed uniformly on the grid;
* every position also gets one uniform draw u_s in [0, 1) for the Bernoulli
  selection of Section IV-A (position s transmits when u_s < bernoulli_p);
* noise draws are unit-variance circular complex normals (Re, Im ~ N(0, 1/2));
  the consumer scales them to the stated SNR per pulse.

Nothing here evaluates the forward model: the radar echo d_s is formed from
these draws by whoever consumes them.
"""

from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class WorkloadSpec:
    name: str
    n_side: int                 # n_x = n_y; N = n_side**2 pixels
    patch_m: float              # side of the square ground patch, metres
    n_pulses: int               # P
    azimuth_deg: float          # azimuth span of the P pulses
    n_freq: int                 # K
    f_lo: float                 # Hz, inclusive
    f_hi: float                 # Hz, inclusive
    n_points: int
    n_lines: int = 0
    line_len_m: tuple = (5.0, 10.0)
    magnitude: str = "uniform"  # "uniform": |rho| ~ U[0.5, 1]; "log40": 10**U(-2, 0)
    dictionary: str = "identity"  # "identity" | "haar" | "edgelet"
    haar_levels: int = 0
    edge_lengths: tuple = ()        # edgelet lengths in pixels
    edge_rotations_deg: tuple = ()  # edgelet rotations, degrees
    n_segments: int = 0             # axis-aligned segment targets
    segment_px: tuple = (4, 8)      # their lengths, pixels
    n_squares: int = 0              # square-outline targets
    square_px: int = 4              # their side, pixels
    bernoulli_p: float = 1.0        # probability that a position transmits
    ideal_count: int = 0            # stop once this many |c| > large_thresh (0: never)
    large_thresh: float = 2e-2      # "large coefficient" threshold of Section IV-B
    snr_db: float = 30.0
    inner_steps: int = 20       # m of Algorithm 1
    phase_error_rad: float = 0.0  # per-pulse phase errors U[-e, e] (0 = none)
    precision: str = "fp32"     # "fp32" | "split_bf16"
    record_every: int = 0       # checkpoint stride of the differentiation form
    lambda_rel: float = 0.05    # lambda = lambda_rel * max|A_1^H d_1|
    radius_m: float = 10_000.0
    altitude_m: float = 1_000.0
    seed: int = 2603

    @property
    def n_pixels(self) -> int:
        return self.n_side * self.n_side


CONFIGS = {
    "small": WorkloadSpec(
        name="small", n_side=32, patch_m=30.0, n_pulses=32, azimuth_deg=10.0,
        n_freq=64, f_lo=9.9e9, f_hi=10.1e9, n_points=10, snr_db=20.0,
        inner_steps=20, seed=2603),
    "haar64": WorkloadSpec(
        name="haar64", n_side=64, patch_m=60.0, n_pulses=128, azimuth_deg=20.0,
        n_freq=256, f_lo=9.8e9, f_hi=10.2e9, n_points=50, n_lines=3,
        dictionary="haar", haar_levels=3, snr_db=30.0, inner_steps=20,
        seed=2604),
    "autofocus": WorkloadSpec(
        name="autofocus", n_side=64, patch_m=60.0, n_pulses=64, azimuth_deg=20.0,
        n_freq=256, f_lo=9.8e9, f_hi=10.2e9, n_points=50, n_lines=3,
        snr_db=30.0, inner_steps=10, phase_error_rad=math.pi / 4,
        record_every=8, seed=2605),
    "large": WorkloadSpec(
        name="large", n_side=128, patch_m=120.0, n_pulses=256, azimuth_deg=30.0,
        n_freq=512, f_lo=9.75e9, f_hi=10.25e9, n_points=200, magnitude="log40",
        snr_db=30.0, inner_steps=20, seed=2606),
    "xlarge": WorkloadSpec(
        name="xlarge", n_side=256, patch_m=250.0, n_pulses=512, azimuth_deg=40.0,
        n_freq=1024, f_lo=9.7e9, f_hi=10.3e9, n_points=1000, n_lines=20,
        snr_db=30.0, inner_steps=10, precision="split_bf16", seed=2607),
    "edgelet64": WorkloadSpec(
        name="edgelet64", n_side=64, patch_m=60.0, n_pulses=128, azimuth_deg=20.0,
        n_freq=256, f_lo=9.8e9, f_hi=10.2e9, n_points=0, n_segments=8,
        dictionary="edgelet", edge_lengths=(4,), edge_rotations_deg=(0.0, 90.0),
        snr_db=30.0, inner_steps=20, seed=2608),
    "session32": WorkloadSpec(
        name="session32", n_side=32, patch_m=30.0, n_pulses=1000, azimuth_deg=2.0,
        n_freq=64, f_lo=9.9e9, f_hi=10.1e9, n_points=0, n_squares=1,
        dictionary="edgelet", edge_lengths=(4,), edge_rotations_deg=(0.0, 90.0),
        snr_db=30.0, inner_steps=20, radius_m=4_000.0, bernoulli_p=0.1, ideal_count=4,
        seed=2609),
}


def spec(name: str, **overrides) -> WorkloadSpec:
    """A named spec, optionally with fields replaced (tests shrink sizes)."""
    base = CONFIGS[name]
    return dataclasses.replace(base, **overrides) if overrides else base


@dataclass
class Workload:
    spec: WorkloadSpec
    # pixel grid: centre of pixel (0, 0) and spacing; z = 0
    x0: float
    y0: float
    dx: float
    dy: float
    positions: np.ndarray       # (P, 3) float64, platform position per pulse
    freq0: float                # f_0
    dfreq: float                # f_{k+1} - f_k
    rho: np.ndarray             # (N,) complex128 reflectivity, flat iy*n+ix
    noise: np.ndarray           # (P, K) complex128, unit-variance draws
    phase_err: np.ndarray       # (P,) float64 true per-pulse phase errors
    support: np.ndarray = field(default=None)  # sorted nonzero pixel indices
    select_u: np.ndarray = field(default=None)  # (P,) uniforms of the Bernoulli selection

    @property
    def n_pixels(self) -> int:
        return self.spec.n_pixels

    def pixel_xyz(self) -> np.ndarray:
        """(N, 3) float64 pixel centres, flat index iy*n_x + ix."""
        n = self.spec.n_side
        ix = np.arange(n, dtype=np.float64)
        xs = self.x0 + ix * self.dx
        ys = self.y0 + ix * self.dy
        gx, gy = np.meshgrid(xs, ys)  # gx[iy, ix] = xs[ix]
        return np.stack([gx.ravel(), gy.ravel(), np.zeros(n * n)], axis=1)

    def freqs(self) -> np.ndarray:
        return self.freq0 + self.dfreq * np.arange(self.spec.n_freq, dtype=np.float64)


def _draw_magnitudes(rng, kind: str, size: int) -> np.ndarray:
    if kind == "uniform":
        return rng.uniform(0.5, 1.0, size)
    if kind == "log40":
        return 10.0 ** rng.uniform(-2.0, 0.0, size)
    raise ValueError(f"unknown magnitude law {kind!r}")


def make_workload(s: WorkloadSpec | str, seed: int | None = None) -> Workload:
    """Draw one workload.  All draws come from one PCG64 stream in a fixed order:
    point pixels, point magnitudes, point phases, line parameters, segment
    parameters, square parameters, noise, phase errors, selection draws."""
    if isinstance(s, str):
        s = CONFIGS[s]
    rng = np.random.Generator(np.random.PCG64(s.seed if seed is None else seed))
    n = s.n_side
    N = n * n
    P, K = s.n_pulses, s.n_freq
    dx = s.patch_m / n
    x0 = -s.patch_m / 2 + dx / 2

    rho = np.zeros(N, dtype=np.complex128)
    n_pts = min(s.n_points, N)
    pts = rng.choice(N, size=n_pts, replace=False)
    mags = _draw_magnitudes(rng, s.magnitude, n_pts)
    phs = rng.uniform(0.0, 2 * math.pi, n_pts)
    np.add.at(rho, pts, mags * np.exp(1j * phs))

    if s.n_lines:
        L = rng.uniform(s.line_len_m[0], s.line_len_m[1], s.n_lines)
        half = np.minimum(L / 2, s.patch_m / 2 - dx)
        cx = rng.uniform(-s.patch_m / 2 + half, s.patch_m / 2 - half)
        cy = rng.uniform(-s.patch_m / 2 + half, s.patch_m / 2 - half)
        ang = rng.uniform(0.0, math.pi, s.n_lines)
        lmag = _draw_magnitudes(rng, s.magnitude, s.n_lines)
        lph = rng.uniform(0.0, 2 * math.pi, s.n_lines)
        for j in range(s.n_lines):
            ns = int(math.floor(L[j] / dx)) + 1
            tt = -L[j] / 2 + dx * np.arange(ns)
            px = cx[j] + tt * math.cos(ang[j])
            py = cy[j] + tt * math.sin(ang[j])
            ix = np.clip(np.rint((px - x0) / dx).astype(np.int64), 0, n - 1)
            iy = np.clip(np.rint((py - x0) / dx).astype(np.int64), 0, n - 1)
            idx = np.unique(iy * n + ix)
            rho[idx] += lmag[j] * np.exp(1j * lph[j])

    if s.n_segments:
        horiz = rng.random(s.n_segments) < 0.5
        seg_len = rng.choice(np.asarray(s.segment_px), size=s.n_segments)
        start_u = rng.random(s.n_segments)
        start_v = rng.random(s.n_segments)
        smag = _draw_magnitudes(rng, s.magnitude, s.n_segments)
        sph = rng.uniform(0.0, 2 * math.pi, s.n_segments)
        for j in range(s.n_segments):
            ln = int(seg_len[j])
            a = int(start_u[j] * (n - ln + 1))   # along the segment
            b = int(start_v[j] * n)              # across it
            run = a + np.arange(ln)
            idx = b * n + run if horiz[j] else run * n + b
            rho[idx] += smag[j] * np.exp(1j * sph[j])

    if s.n_squares:
        side = s.square_px
        qa = rng.random(s.n_squares)
        qb = rng.random(s.n_squares)
        qmag = _draw_magnitudes(rng, s.magnitude, s.n_squares)
        qph = rng.uniform(0.0, 2 * math.pi, s.n_squares)
        for j in range(s.n_squares):
            x = int(qa[j] * (n - side + 1))
            y = int(qb[j] * (n - side + 1))
            run = np.arange(side)
            amp = qmag[j] * np.exp(1j * qph[j])
            for idx in (y * n + x + run, (y + side - 1) * n + x + run,
                        (y + run) * n + x, (y + run) * n + x + side - 1):
                rho[idx] += amp

    g = rng.standard_normal((P, K, 2))
    noise = (g[..., 0] + 1j * g[..., 1]) / math.sqrt(2.0)

    if s.phase_error_rad > 0:
        phase_err = rng.uniform(-s.phase_error_rad, s.phase_error_rad, P)
    else:
        phase_err = np.zeros(P)
    select_u = rng.random(P)

    theta = np.deg2rad(s.azimuth_deg) * np.arange(P) / max(P - 1, 1)
    positions = np.stack([s.radius_m * np.cos(theta), s.radius_m * np.sin(theta),
                          np.full(P, s.altitude_m)], axis=1)

    dfreq = (s.f_hi - s.f_lo) / (K - 1) if K > 1 else 0.0
    return Workload(spec=s, x0=x0, y0=x0, dx=dx, dy=dx, positions=positions,
                    freq0=s.f_lo, dfreq=dfreq, rho=rho, noise=noise,
                    phase_err=phase_err, support=np.flatnonzero(rho), select_u=select_u)


def library_kwargs(wl: Workload, **overrides) -> dict:
    """Keyword arguments describing this workload to the GPU library's binding
    (field mapping only)."""
    s = wl.spec
    kw = dict(n_x=s.n_side, n_y=s.n_side, x0=wl.x0, y0=wl.y0, dx=wl.dx, dy=wl.dy,
              positions=wl.positions, freq0=wl.freq0, dfreq=wl.dfreq, n_freq=s.n_freq,
              dictionary=s.dictionary, haar_levels=s.haar_levels, lam=s.lambda_rel,
              lam_relative=True, precision=s.precision,
              edge_lengths=tuple(s.edge_lengths), edge_rotations=tuple(s.edge_rotations_deg))
    kw.update(overrides)
    return kw
