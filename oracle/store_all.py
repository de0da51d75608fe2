"""Store-all-pulses FISTA, the comparator of Section III-D / Table I (test
infrastructure).

Instead of the running sufficient statistics (H_n, b_n) this method keeps every
received pulse: its data d_k (rotated by its phase correction) and its
operator G_k = F_k W.  After pulse n it runs the same m warm-started steps of
Algorithm 1, but the gradient of the data term is formed matrix-free from the
stored pulses,

    grad = sum_k G_k^H (G_k z - d_k),

and the running power vector is advanced with sum_k G_k^H (G_k w).  Since
sum_k G_k^H G_k = H_n and sum_k G_k^H d_k = b_n, the iterates are those of
Online FISTA in exact arithmetic; what differs is storage (Table I: n N_r
(1 + M + N_r) complex values against M (M + 1)) and work per step (two passes
over the n N_r x M stacked operator against one over the M x M Gram).  lambda
and sigma_n^2 follow the same rules as the online method.

Pinned by: the trajectory equals the Online FISTA oracle's to rounding, and
the stored-value count equals Table I's FISTA column.
"""

from __future__ import annotations

import math

import numpy as np

from . import sar
from .dictionary import synthesis_matrix
from .online_fista import momentum_schedule, soft_threshold, spectral_norm_sq


class StoreAllFistaOracle:
    def __init__(self, pixel_xyz, positions, freqs, dictionary="identity", n_side=None,
                 levels=0, lam=None, lam_rel=0.05, kernel_sign=-1, edge_lengths=(),
                 edge_rotations=()):
        self.pixel_xyz = np.asarray(pixel_xyz, np.float64)
        self.positions = np.asarray(positions, np.float64)
        self.freqs = np.asarray(freqs, np.float64)
        N = self.pixel_xyz.shape[0]
        if n_side is None:
            n_side = int(round(math.sqrt(N)))
        self.W = synthesis_matrix(dictionary, n_side, levels, edge_lengths, edge_rotations)
        self.M = N if self.W is None else self.W.shape[1]
        self.lam_abs, self.lam_rel, self.sign = lam, lam_rel, kernel_sign
        self.G, self.d = [], []
        self.c = np.zeros(self.M, np.complex128)
        self.w = np.full(self.M, 1.0 / math.sqrt(self.M), np.complex128)
        self.t, self.rho_hat, self.sigma2_acc, self.n = 1.0, 0.0, 0.0, 0
        self.lam = 0.0 if lam is None else float(lam)

    @classmethod
    def from_workload(cls, wl, **kw):
        s = wl.spec
        kw.setdefault("lam_rel", s.lambda_rel)
        kw.setdefault("edge_lengths", s.edge_lengths)
        kw.setdefault("edge_rotations", s.edge_rotations_deg)
        return cls(wl.pixel_xyz(), wl.positions, wl.freqs(), s.dictionary, s.n_side,
                   s.haar_levels, **kw)

    def _normal(self, v, with_data):
        """sum_k G_k^H (G_k v - d_k) (or without the data)."""
        y = np.zeros(self.M, np.complex128)
        for G, d in zip(self.G, self.d):
            r = G @ v
            if with_data:
                r = r - d
            y += G.conj().T @ r
        return y

    def push_pulse(self, d, s: int, phase_corr: float = 0.0):
        F = sar.forward_rows(self.positions[s], self.pixel_xyz, self.freqs, self.sign)
        G = F if self.W is None else F @ self.W
        dt = np.asarray(d, np.complex128) * np.exp(-1j * phase_corr)
        self.G.append(G)
        self.d.append(dt)
        self.n += 1
        if self.n == 1 and self.lam_abs is None:
            self.lam = self.lam_rel * float(np.max(np.abs(G.conj().T @ dt)))
        self.sigma2 = spectral_norm_sq(G)
        self.sigma2_acc += self.sigma2
        self.L = self.rho_hat + self.sigma2_acc
        self.tau = 1.0 / self.L

    def reconstruct(self, iters: int):
        tau, alpha = self.tau, self.lam * self.tau
        betas, t_end = momentum_schedule(1.0 if self.n == 1 else self.t, iters)
        c_prev = self.c.copy()
        z = c_prev
        c = c_prev
        for beta in betas:
            yw = self._normal(self.w, False)
            self.rho_hat = float(np.vdot(self.w, yw).real)
            self.w = yw / np.linalg.norm(yw)
            self.sigma2_acc = 0.0
            c = soft_threshold(z - tau * self._normal(z, True), alpha)
            z = c + beta * (c - c_prev)
            c_prev = c
        self.c, self.t = c, t_end
        return c

    def stored_values(self) -> int:
        """Real values kept (complex counted twice): c, the dictionary and every
        pulse's d_k, G_k and R_k = I (N_r x N_r), as Table I counts them."""
        N = self.pixel_xyz.shape[0]
        Nr = len(self.freqs)
        return self.M * (N + 1) + sum(2 * (d.size + G.size + Nr * Nr)
                                      for G, d in zip(self.G, self.d))
