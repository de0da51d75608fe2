"""Independent batch weighted-LASSO solver (test infrastructure).

Section III-B states the batch problem the online method tracks:
J_n(c) = 1/2 sum_k |d_k - G_k c|^2 + lambda |c|_1 (R_k = I).  This module
solves it directly on the stacked operator G = [G_1; ...; G_n] and data
d = [d_1; ...; d_n] by cyclic complex coordinate descent, without forming
the sufficient statistics, so it can pin the online result (after
continuation) from a different route.

Coordinate update for column j (residual r = d - G c, a_j = |G_j|^2):
    rho_j = G_j^H r + a_j c_j,   c_j <- S_lambda(rho_j) / a_j
Stops when the KKT residual (below) falls under tol.
"""

from __future__ import annotations

import numpy as np


def kkt_residual(grad: np.ndarray, c: np.ndarray, lam: float) -> float:
    """Max violation of the LASSO optimality conditions for gradient grad of
    the smooth part: grad_i = -lam c_i/|c_i| where c_i != 0, |grad_i| <= lam
    where c_i = 0."""
    mag = np.abs(c)
    nz = mag > 0
    r = np.zeros(c.shape[0])
    r[nz] = np.abs(grad[nz] + lam * c[nz] / mag[nz])
    r[~nz] = np.maximum(np.abs(grad[~nz]) - lam, 0.0)
    return float(r.max()) if r.size else 0.0


def objective(G, d, c, lam) -> float:
    r = d - G @ c
    return float(0.5 * np.vdot(r, r).real + lam * np.sum(np.abs(c)))


def solve_cd(G: np.ndarray, d: np.ndarray, lam: float, tol: float = 1e-12,
             max_sweeps: int = 20000, c0=None) -> np.ndarray:
    G = np.asarray(G, np.complex128)
    d = np.asarray(d, np.complex128)
    M = G.shape[1]
    c = np.zeros(M, np.complex128) if c0 is None else np.array(c0, np.complex128)
    a = np.sum(np.abs(G) ** 2, axis=0)
    r = d - G @ c
    for _ in range(max_sweeps):
        for j in range(M):
            if a[j] == 0.0:
                continue
            gj = G[:, j]
            rho = np.vdot(gj, r) + a[j] * c[j]
            mag = abs(rho)
            new = rho * (1.0 - lam / mag) / a[j] if mag > lam else 0.0
            if new != c[j]:
                r -= gj * (new - c[j])
                c[j] = new
        grad = G.conj().T @ (G @ c - d)
        if kkt_residual(grad, c, lam) < tol:
            break
    return c
