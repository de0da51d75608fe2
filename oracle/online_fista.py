"""Online FISTA in FP64, step by step (test infrastructure).

Follows Section III-C of the paper and its Algorithm 1 ("Online FISTA per
pulse"), with R_n = I (white noise; the noise power is absorbed into lambda):

push_pulse(d_s, s)                       -- one received pulse
    A_s   = F_s W                          (Section III-A, eq. for G)
    d~    = d_s * exp(-i phase_corr)       (autofocus correction; 0 by default)
    H    += A_s^H A_s,  b += A_s^H d~      (Delta-A / Delta-b and A_n / b_n eqs.)
    lambda = lambda_rel * max_i |A_1^H d~_1|   at the first pulse only
    L_n   from one of three rules, tau = 1 / L_n:
        "running": rho_{n-1} + sigma_n^2   (rho = Rayleigh quotient of the running
                   power vector w on H; sigma_n^2 = ||A_s||_2^2).  This is the
                   paper's incremental bound L_{n+1} <= L_n + ||G_n||^2 with the
                   previous bound replaced by the running spectral estimate of
                   the Section III-B condition L >= ||sum G^H G||_2.
        "bound":   L_{n-1} + sigma_n^2     (the incremental bound taken literally)
        "exact":   lambda_max(H_n)         (tests only)

reconstruct(iters)                       -- Algorithm 1, iters inner steps
    c0 = c_hat_{n-1}, z = c0, t = t_{n-1} (t = 1 at the first pulse)
    repeat: g = H z - b; u = z - tau g; c = S_{lambda tau}(u);
            t' = (1 + sqrt(1 + 4 t^2)) / 2;  z = c + ((t - 1) / t') (c - c_prev)
    every step also advances the power vector: y = H w, rho = Re(w^H y), w = y/|y|
    return c_hat_n = c, t_n = t'

Readings of garbled or silent points: the shrink threshold is lambda*tau (the
printed subscript uses the momentum t), the shrink is the complex proximal map
u * max(0, 1 - alpha/|u|) (the printed formula drops the phase), coefficients
are complex, sigma_n^2 comes from an FP64 power iteration on the K x K matrix
A_s A_s^H started at 1/sqrt(K), stopped when the Rayleigh quotient moves by at
most 1e-13 relative or after 200 steps; w starts at 1/sqrt(M) and rho_0 = 0.

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

POWER_MAX_STEPS = 200
POWER_REL_TOL = 1e-13


def soft_threshold(u: np.ndarray, alpha: float) -> np.ndarray:
    """Complex soft threshold S_alpha(u)_i = u_i max(0, 1 - alpha/|u_i|); 0 when
    |u_i| <= alpha (so u_i = 0 maps to 0)."""
    mag = np.abs(u)
    out = np.zeros_like(u)
    keep = mag > alpha
    out[keep] = u[keep] * (1.0 - alpha / mag[keep])
    return out


def power_sigma2(M: np.ndarray) -> float:
    """lambda_max of a Hermitian PSD matrix by power iteration (FP64).

    v_0 = 1/sqrt(K); each step y = M v, q = Re(v^H y), v = y/|y|; stop when
    |q - q_prev| <= 1e-13 |q| or after 200 steps; returns the last q.
    """
    K = M.shape[0]
    v = np.full(K, 1.0 / math.sqrt(K), dtype=np.complex128)
    q_prev = None
    q = 0.0
    for _ in range(POWER_MAX_STEPS):
        y = M @ v
        q = float(np.vdot(v, y).real)
        if q_prev is not None and abs(q - q_prev) <= POWER_REL_TOL * abs(q):
            break
        q_prev = q
        nrm = float(np.linalg.norm(y))
        if nrm == 0.0:
            break
        v = y / nrm
    return q


def t_next(t: float) -> float:
    return (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0


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
        self.rho_hat = 0.0
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
        dH = A.conj().T @ A
        db = A.conj().T @ dt
        self.H += dH
        self.b += db
        self.n += 1
        if self.n == 1 and self.lam_abs is None:
            self.lam = self.lam_rel * float(np.max(np.abs(db)))
        sigma2 = power_sigma2(A @ A.conj().T)
        if self.lip == "running":
            L = self.rho_hat + sigma2
        elif self.lip == "bound":
            L = self.L + sigma2
        elif self.lip == "exact":
            L = float(np.linalg.eigvalsh(self.H)[-1])
        elif self.lip == "given":
            L = float(self.given_L[self.n - 1])
        else:
            raise ValueError(self.lip)
        self.sigma2 = sigma2
        self.L = L
        self.tau = 1.0 / L

    def reconstruct(self, iters: int, trace=None) -> np.ndarray:
        """Algorithm 1 with `iters` inner steps on the current (H_n, b_n)."""
        if self.n == 0:
            raise RuntimeError("reconstruct before any pulse")
        H, b, tau = self.H, self.b, self.tau
        alpha = self.lam * tau
        c_prev = self.c.copy()
        z = c_prev.copy()
        t = 1.0 if (self.n == 1 or self.momentum == "restart") else self.t
        c = c_prev
        for _ in range(iters):
            yw = H @ self.w
            self.rho_hat = float(np.vdot(self.w, yw).real)
            self.w = yw / np.linalg.norm(yw)
            g = H @ z - b
            u = z - tau * g
            c = soft_threshold(u, alpha)
            tn = t_next(t)
            beta = 0.0 if self.momentum == "ista" else (t - 1.0) / tn
            if trace is not None:
                trace.append(dict(z=z, u=u, c=c, beta=beta))
            z = c + beta * (c - c_prev)
            c_prev = c
            t = tn
        self.c = c
        self.t = t
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
