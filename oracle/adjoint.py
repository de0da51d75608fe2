"""Reverse mode through unrolled Online FISTA, FP64 (test infrastructure).

The differentiation form treats the l1 weight lambda and per-pulse phase
corrections phi_n (data used as d_n exp(-i phi_n)) as parameters of the whole
online run and returns dLoss/dlambda and dLoss/dphi_n for a real loss of the
final image.  Everything else (H_n, L_n, tau_n, the power vector, the momentum
sequence) does not depend on lambda or phi, so only b_n and the shrink
threshold alpha_n = lambda tau_n carry gradient.

Forward of pulse n (Algorithm 1, m steps, c_0 = c_hat_{n-1}, z_1 = c_0):
    u_k = z_k - tau (H_n z_k - b_n),  c_k = S_alpha(u_k),
    z_{k+1} = (1 + beta_k) c_k - beta_k c_{k-1},   c_hat_n = c_m.
Reverse, with complex adjoints xbar = dL/dRe x + i dL/dIm x:
    cbar_k += (1 + beta_k) zbar_{k+1};  cbar_{k-1} += -beta_k zbar_{k+1}
    ubar_k = J_S(u_k)^T cbar_k: for |u| > alpha, with uhat = u/|u| and
             p = Re(conj(cbar) uhat): ubar = p uhat + (1 - alpha/|u|)(cbar - p uhat);
             0 where |u| <= alpha;  alphabar += -p (active entries)
    zbar_k += ubar_k - tau H_n ubar_k;   bbar_n += tau ubar_k
    c_hat_bar_{n-1} = cbar_0 + zbar_1;   lambdabar += tau_n alphabar_n
Across pulses b_n = b_{n-1} + Delta b_n, Delta b_n = A^H d_n e^{-i phi_n}:
    B_n = sum_{n' >= n} bbar_{n'},   dL/dphi_n = Im(sum_i conj(B_n,i) Delta b_n,i).

Pinned by central finite differences of the forward oracle (two step sizes)
and by the exact invariance sum_n dL/dphi_n = 0 of |image| losses.
"""

from __future__ import annotations

import numpy as np

from .online_fista import OnlineFistaOracle


def magnitude_loss(x: np.ndarray, target_mag: np.ndarray):
    """L = sum_i (|x_i| - g_i)^2 and its adjoint (d|x|/dx := 0 at x = 0)."""
    mag = np.abs(x)
    L = float(np.sum((mag - target_mag) ** 2))
    xbar = np.zeros_like(x)
    nz = mag > 0
    xbar[nz] = 2.0 * (mag[nz] - target_mag[nz]) * x[nz] / mag[nz]
    return L, xbar


class RecordedRun:
    """Online FISTA forward that keeps what the reverse pass needs."""

    def __init__(self, oracle: OnlineFistaOracle):
        self.o = oracle
        self.pulses = []  # per pulse: dict(s, tau, alpha, dB, u=[...], beta=[...])

    def push_and_reconstruct(self, d, s, phase, iters):
        o = self.o
        A = o.rows(s)
        db = A.conj().T @ (np.asarray(d, np.complex128) * np.exp(-1j * phase))
        o.push_pulse(d, s, phase)
        rec = dict(s=s, tau=o.tau, alpha=o.lam * o.tau, dB=db, u=[], beta=[])
        trace = []
        o.reconstruct(iters, trace=trace)
        rec["u"] = [tr["u"].copy() for tr in trace]
        rec["beta"] = [tr["beta"] for tr in trace]
        self.pulses.append(rec)


def _shrink_vjp(u, cbar, alpha):
    """ubar = J_S(u)^T cbar and alphabar for the complex soft threshold."""
    mag = np.abs(u)
    ubar = np.zeros_like(u)
    act = mag > alpha
    uh = u[act] / mag[act]
    p = np.real(np.conj(cbar[act]) * uh)
    ubar[act] = p * uh + (1.0 - alpha / mag[act]) * (cbar[act] - p * uh)
    return ubar, -float(np.sum(p))


def backward(run: RecordedRun, cbar_final: np.ndarray, lam: float):
    """Returns (dL/dlambda, dL/dphi per pulse) for the adjoint cbar_final of
    the final coefficients."""
    P = len(run.pulses)
    H = run.o.H.copy()  # H_n of the last pulse; earlier ones by subtracting A_s^H A_s
    cbar_hat = np.array(cbar_final, np.complex128)
    Bbar = np.zeros_like(cbar_hat)
    lam_bar = 0.0
    phi_bar = np.zeros(P)
    for n in range(P - 1, -1, -1):
        rec = run.pulses[n]
        tau, alpha = rec["tau"], rec["alpha"]
        m = len(rec["u"])
        zbar_next = np.zeros_like(cbar_hat)   # zbar_{m+1}: z_{m+1} is not used
        cbar = cbar_hat.copy()                 # cbar_m
        cpart = np.zeros_like(cbar_hat)        # running partial of cbar_{k-1}
        bbar = np.zeros_like(cbar_hat)
        alpha_bar = 0.0
        for k in range(m, 0, -1):
            beta = rec["beta"][k - 1]
            cbar = cbar + (1.0 + beta) * zbar_next
            cpart = -beta * zbar_next
            ubar, ab = _shrink_vjp(rec["u"][k - 1], cbar, alpha)
            alpha_bar += ab
            zbar = ubar - tau * (H @ ubar)
            bbar += tau * ubar
            zbar_next = zbar
            cbar = cpart                        # becomes cbar_{k-1} (partial)
        cbar_hat = cbar + zbar_next             # cbar_0 + zbar_1
        lam_bar += tau * alpha_bar
        Bbar = Bbar + bbar
        phi_bar[n] = float(np.imag(np.vdot(Bbar, rec["dB"])))
        A = run.o.rows(rec["s"])
        H -= A.conj().T @ A
    return lam_bar, phi_bar


def run_loss(wl, d, lam, phases, m, target_mag, pulses=None, record=False):
    """Forward oracle with an absolute lambda; returns (L, image, xbar, run)."""
    o = OnlineFistaOracle.from_workload(wl, lam=lam)
    P = wl.spec.n_pulses if pulses is None else pulses
    run = RecordedRun(o) if record else None
    for p in range(P):
        if record:
            run.push_and_reconstruct(d[p], p, phases[p], m)
        else:
            o.push_pulse(d[p], p, phases[p])
            o.reconstruct(m)
    x = o.image()
    L, xbar = magnitude_loss(x, target_mag)
    return L, x, xbar, run


def gradients(wl, d, lam, phases, m, target_mag, pulses=None):
    """dL/dlambda and dL/dphi of the magnitude loss through the whole run."""
    L, x, xbar, run = run_loss(wl, d, lam, phases, m, target_mag, pulses, record=True)
    o = run.o
    cbar = xbar if o.W is None else o.W.T @ xbar
    lam_bar, phi_bar = backward(run, cbar, lam)
    return L, lam_bar, phi_bar
