"""Pins of the FP64 reverse pass through unrolled Online FISTA.

The gradients to lambda and to per-pulse phase corrections are checked
against central finite differences of the forward oracle at two step sizes
(agreement at both says no kink lies inside the stencil), against the exact
invariance sum_n dL/dphi_n = 0 (a common phase rotates every coefficient and
leaves |image| unchanged), and against the lambda >= max|b| regime where the
image is identically zero and both gradients vanish.
"""

import numpy as np
import pytest

from oracle import adjoint, sar
from oracle.online_fista import OnlineFistaOracle
from workload import make_workload, spec


def tiny(**kw):
    base = dict(n_side=8, patch_m=8.0, n_pulses=6, n_freq=16, n_points=3, n_lines=0,
                inner_steps=5)
    base.update(kw)
    return make_workload(spec("autofocus", **base))


def first_lambda(wl, d):
    o = OnlineFistaOracle.from_workload(wl)
    o.push_pulse(d[0], 0)
    return o.lam


def fd_grads(wl, d, lam, phases, m, target, h):
    g = np.zeros(len(phases))
    for n in range(len(phases)):
        pp = phases.copy()
        pp[n] += h
        pm = phases.copy()
        pm[n] -= h
        g[n] = (adjoint.run_loss(wl, d, lam, pp, m, target)[0]
                - adjoint.run_loss(wl, d, lam, pm, m, target)[0]) / (2 * h)
    hl = 1e-6 * lam
    gl = (adjoint.run_loss(wl, d, lam + hl, phases, m, target)[0]
          - adjoint.run_loss(wl, d, lam - hl, phases, m, target)[0]) / (2 * hl)
    return gl, g


@pytest.mark.parametrize("dictionary", ["identity", "haar"])
def test_adjoint_matches_central_differences(dictionary):
    wl = tiny(dictionary=dictionary, haar_levels=2 if dictionary == "haar" else 0)
    d = sar.echoes(wl)
    lam = first_lambda(wl, d)
    rng = np.random.default_rng(3)
    phases = rng.uniform(-0.3, 0.3, wl.spec.n_pulses)
    target = np.abs(wl.rho)
    m = wl.spec.inner_steps
    L, gl, gp = adjoint.gradients(wl, d, lam, phases, m, target)
    for h in (1e-5, 1e-6):
        fl, fp = fd_grads(wl, d, lam, phases, m, target, h)
        assert abs(gl - fl) <= 1e-6 * max(abs(fl), 1e-12)
        assert np.max(np.abs(gp - fp)) <= 1e-6 * np.max(np.abs(fp))


def test_phase_gradients_sum_to_zero():
    wl = tiny(n_pulses=8)
    d = sar.echoes(wl)
    lam = first_lambda(wl, d)
    phases = np.random.default_rng(4).uniform(-0.7, 0.7, wl.spec.n_pulses)
    L, gl, gp = adjoint.gradients(wl, d, lam, phases, wl.spec.inner_steps, np.abs(wl.rho))
    assert np.max(np.abs(gp)) > 1e-6
    assert abs(gp.sum()) <= 1e-12 * np.sum(np.abs(gp))


def test_zero_image_regime_has_zero_gradients():
    wl = tiny()
    d = sar.echoes(wl)
    L, gl, gp = adjoint.gradients(wl, d, 1e9, np.zeros(wl.spec.n_pulses), 5, np.abs(wl.rho))
    assert gl == 0.0 and np.all(gp == 0.0)
    assert L == pytest.approx(float(np.sum(np.abs(wl.rho) ** 2)))
