"""Online FISTA in FP64, step by step (test infrastructure).

Follows Section III-C of the paper and its Algorithm 1 (Online FISTA per
pulse), with R_n = I (white noise; the noise power is absorbed into lambda).

One received pulse (``push_pulse``):
  * the per-pulse operator A_s = F_s W (Section III-A, eq. for G) and the data
    rotated by the autofocus correction, d~ = d_s exp(-i phase_corr);
  * the sufficient statistics grow by A_s^H A_s and A_s^H d~ (the Delta-A /
    Delta-b and A_n / b_n equations);
  * lambda = lambda_rel * max_i |A_1^H d~_1| at the first pulse only;
  * the step 1/L_n.  Section III-B asks for L >= ||sum G^H G||_2 and Section
    III-C bounds its growth by ||G_n||_2^2 per pulse.  sigma_n^2 = ||A_s||_2^2
    is the largest eigenvalue of the K x K matrix A_s A_s^H (its definition;
    a library eigen-solver is the step).  Three rules:
      "running": rho + (sum of sigma^2 of the pulses pushed since the last
                 FISTA step).  rho is the Rayleigh quotient of a power vector
                 advanced once per FISTA step on the H of that step (0 before
                 any step).  This is the incremental bound with the previous
                 bound replaced by the running spectral estimate; summing over
                 every pulse pushed since that estimate keeps it a Weyl bound
                 when several pulses arrive between reconstructions.
      "bound":   L_{n-1} + sigma_n^2 (the incremental bound taken literally).
      "exact":   lambda_max(H_n) (tests only); "given": replayed values.

Reconstruction (``reconstruct``, Algorithm 1 with `iters` inner steps) is a
proximal-gradient (forward-backward) iteration on J_n with Nesterov-type
extrapolation, warm-started at c_hat_{n-1}:
  * step: c = S_{lambda tau}(z - tau (H z - b)) (``prox_gradient``);
  * extrapolation weights from the momentum scalar carried across pulses
    (``momentum_schedule``); the extrapolated point starts at c_hat_{n-1};
  * the power vector advances once per step on the same H.

Readings of garbled or silent points: the shrink threshold is lambda*tau (the
printed subscript uses the momentum t), the shrink is the complex proximal map
u * max(0, 1 - alpha/|u|) (the printed formula drops the phase), coefficients
are complex, the power vector starts at 1/sqrt(M).

Test-only switches: momentum "restart" (t = 1 every pulse) and "ista"
(no momentum), the "exact" and "given" Lipschitz rules, and kernel sign +1.

Parity: the parts are pinned (see the package header); the full m-step
trajectory is "parity unpinned" as a whole.
"""

from __future__ import annotations

import math

import numpy as np

from . import sar
from .dictionary import synthesis_matrix


def soft_threshold(u: np.ndarray, alpha: float) -> np.ndarray:
    """Complex soft threshold S_alpha(u)_i = u_i max(0, 1 - alpha/|u_i|); 0 when
    |u_i| <= alpha (so u_i = 0 maps to 0)."""
    mag = np.abs(u)
    out = np.zeros_like(u)
    keep = mag > alpha
    out[keep] = u[keep] * (1.0 - alpha / mag[keep])
    return out


def spectral_norm_sq(A: np.ndarray) -> float:
    """||A||_2^2 = largest eigenvalue of the Hermitian PSD matrix A A^H (FP64)."""
    return float(np.linalg.eigvalsh(A @ A.conj().T)[-1])


def t_next(t: float) -> float:
    """Momentum scalar of the next step, the positive root of t'^2 - t' = t^2."""
    return (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0


def momentum_schedule(t0: float, iters: int, mode: str = "fista"):
    """Extrapolation weights beta_1..beta_iters of one reconstruction and the
    momentum scalar after it.  beta_k = (t_k - 1)/t_{k+1}, t_1 = t0; "ista"
    keeps beta = 0 (the scalar still advances, as it does not feed back)."""
    betas = []
    t = t0
    for _ in range(iters):
        tn = t_next(t)
        betas.append(0.0 if mode == "ista" else (t - 1.0) / tn)
        t = tn
    return betas, t


def prox_gradient(H: np.ndarray, b: np.ndarray, z: np.ndarray, tau: float,
                  alpha: float):
    """Forward-backward step on J(c) = 1/2 c^H H c - Re(b^H c) + lambda |c|_1:
    gradient step of length tau on the smooth part, then the l1 prox with
    threshold alpha = lambda tau.  Returns (u, c) with u the gradient point."""
    u = z - tau * (H @ z - b)
    return u, soft_threshold(u, alpha)


class OnlineFistaOracle:
    """Online FISTA state machine in complex128 (one object per image).

    pixel_xyz: (N, 3) pixel centres; positions: (P_pos, 3) platform positions;
    freqs: (K,) Hz; dictionary: "identity", "haar" (with n_side, levels) or
    "edgelet" (with n_side, edge_lengths, edge_rotations in degrees); the
    coefficient count M is the dictionary's column count.
    """

    def __init__(self, pixel_xyz, positions, freqs, dictionary="identity",
                 n_side=None, levels=0, lam=None, lam_rel=0.05, lip="running",
                 momentum="fista", kernel_sign=-1, edge_lengths=(), edge_rotations=()):
        self.pixel_xyz = np.asarray(pixel_xyz, np.float64)
        self.positions = np.asarray(positions, np.float64)
        self.freqs = np.asarray(freqs, np.float64)
        N = self.pixel_xyz.shape[0]
        if n_side is None:
            n_side = int(round(math.sqrt(N)))
        self.W = synthesis_matrix(dictionary, n_side, levels, edge_lengths, edge_rotations)
        self.M = N if self.W is None else self.W.shape[1]
        self.lam_abs = lam
        self.lam_rel = lam_rel
        self.lip = lip
        self.momentum = momentum
        self.sign = kernel_sign
        self.given_L = None
        self.reset()

    @classmethod
    def from_workload(cls, wl, **kw):
        s = wl.spec
        kw.setdefault("lam_rel", s.lambda_rel)
        kw.setdefault("edge_lengths", s.edge_lengths)
        kw.setdefault("edge_rotations", s.edge_rotations_deg)
        return cls(wl.pixel_xyz(), wl.positions, wl.freqs(), s.dictionary,
                   s.n_side, s.haar_levels, **kw)

    # -- state -----------------------------------------------------------
    def reset(self):
        M = self.M
        self.H = np.zeros((M, M), dtype=np.complex128)
        self.b = np.zeros(M, dtype=np.complex128)
        self.c = np.zeros(M, dtype=np.complex128)
        self.t = 1.0
        self.L = 0.0
        self.tau = 0.0
        self.lam = 0.0 if self.lam_abs is None else float(self.lam_abs)
        self.w = np.full(M, 1.0 / math.sqrt(M), dtype=np.complex128)
        self.rho_hat = 0.0      # Rayleigh quotient of w at the last FISTA step
        self.sigma2_acc = 0.0   # sum of sigma^2 pushed since that step
        self.n = 0
        self.history = []

    def rows(self, s: int) -> np.ndarray:
        """A_s = F_s W (K x M)."""
        F = sar.forward_rows(self.positions[s], self.pixel_xyz, self.freqs, self.sign)
        return F if self.W is None else F @ self.W

    # -- one pulse -------------------------------------------------------
    def push_pulse(self, d: np.ndarray, s: int, phase_corr: float = 0.0):
        A = self.rows(s)
        dt = np.asarray(d, np.complex128) * np.exp(-1j * phase_corr)
        db = A.conj().T @ dt
        self.H += A.conj().T @ A
        self.b += db
        self.n += 1
        if self.n == 1 and self.lam_abs is None:
            self.lam = self.lam_rel * float(np.max(np.abs(db)))
        self.sigma2 = spectral_norm_sq(A)
        self.sigma2_acc += self.sigma2
        if self.lip == "running":
            L = self.rho_hat + self.sigma2_acc
        elif self.lip == "bound":
            L = self.L + self.sigma2
        elif self.lip == "exact":
            L = float(np.linalg.eigvalsh(self.H)[-1])
        elif self.lip == "given":
            L = float(self.given_L[self.n - 1])
        else:
            raise ValueError(self.lip)
        self.L = L
        self.tau = 1.0 / L

    def _power_step(self):
        """One power-iteration step of the running spectral estimate on H."""
        y = self.H @ self.w
        self.rho_hat = float(np.vdot(self.w, y).real)
        self.w = y / np.linalg.norm(y)
        self.sigma2_acc = 0.0

    def reconstruct(self, iters: int, trace=None) -> np.ndarray:
        """Algorithm 1 with `iters` inner steps on the current (H_n, b_n)."""
        if self.n == 0:
            raise RuntimeError("reconstruct before any pulse")
        tau = self.tau
        alpha = self.lam * tau
        first = self.n == 1 or self.momentum == "restart"
        betas, t_end = momentum_schedule(1.0 if first else self.t, iters, self.momentum)
        c_prev = self.c.copy()   # c_hat_{n-1}
        z = c_prev               # warm start of the extrapolated point
        c = c_prev
        for beta in betas:
            self._power_step()
            u, c = prox_gradient(self.H, self.b, z, tau, alpha)
            if trace is not None:
                trace.append(dict(z=z, u=u, c=c, beta=beta))
            z = c + beta * (c - c_prev)
            c_prev = c
        self.c = c
        self.t = t_end
        self.history.append(dict(n=self.n, L=self.L, tau=self.tau, t=self.t,
                                 rho_hat=self.rho_hat, lam=self.lam))
        return c

    def image(self) -> np.ndarray:
        """x = W c (pixel domain)."""
        return self.c.copy() if self.W is None else self.W @ self.c

    # -- objective helpers (pins) ----------------------------------------
    def objective_stats(self, c: np.ndarray) -> float:
        """J_n(c) - const = 1/2 c^H H c - Re(b^H c) + lambda |c|_1."""
        return float(0.5 * np.vdot(c, self.H @ c).real - np.vdot(self.b, c).real
                     + self.lam * np.sum(np.abs(c)))


def run(wl, d=None, m=None, phase_corr=None, pulses=None, **kw):
    """Run a whole workload through the oracle; returns the oracle object."""
    o = OnlineFistaOracle.from_workload(wl, **kw)
    if d is None:
        d = sar.echoes(wl, sign=o.sign)
    m = wl.spec.inner_steps if m is None else m
    P = wl.spec.n_pulses if pulses is None else pulses
    for p in range(P):
        o.push_pulse(d[p], p, 0.0 if phase_corr is None else phase_corr[p])
        o.reconstruct(m)
    return o
