"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's
own formula: they use closed forms, invariants, an independent batch solver,
high-precision arithmetic or brute force on tiny inputs.
"""

import math

import mpmath
import numpy as np
import pytest

from oracle import dictionary, lasso, memory, sar
from oracle.online_fista import OnlineFistaOracle, soft_threshold, spectral_norm_sq, t_next
from workload import make_workload, spec


def tiny(**kw):
    base = dict(n_side=8, patch_m=8.0, n_pulses=8, n_freq=16, n_points=3,
                azimuth_deg=10.0, inner_steps=20)
    base.update(kw)
    return make_workload(spec("small", **base))


def stacked(o, d, P):
    G = np.concatenate([o.rows(p) for p in range(P)], axis=0)
    return G, np.concatenate([d[p] for p in range(P)])


# ---------------------------------------------------------------- forward model
def test_phase_matches_50_digit_evaluation():
    """Section II phase: exp(-i 4 pi f R / c) evaluated in 50-digit arithmetic
    from the same float64 geometry; FP64 range/phase must stay within 1e-8 rad."""
    wl = make_workload("haar64")
    pix = wl.pixel_xyz()
    f = wl.freqs()
    mpmath.mp.dps = 50
    rng = np.random.default_rng(0)
    for _ in range(12):
        s = int(rng.integers(wl.spec.n_pulses))
        k = int(rng.integers(wl.spec.n_freq))
        i = int(rng.integers(wl.n_pixels))
        F = sar.forward_rows(wl.positions[s], pix[i:i + 1], f[k:k + 1])[0, 0]
        p = [mpmath.mpf(float(v)) for v in wl.positions[s]]
        x = [mpmath.mpf(float(v)) for v in pix[i]]
        R = mpmath.sqrt(sum((a - b) ** 2 for a, b in zip(p, x)))
        ph = 4 * mpmath.pi * mpmath.mpf(float(f[k])) * R / mpmath.mpf(299792458)
        ref = complex(mpmath.cos(ph), -mpmath.sin(ph))
        assert abs(F - ref) < 1e-8


def test_rows_have_unit_modulus_and_fp32_phase_is_wrong():
    """A = 1 (Section II): |F| = 1.  Negative control: forming R in FP32 moves
    the phase by a large fraction of a radian at 10 km and X band."""
    wl = make_workload("haar64")
    pix = wl.pixel_xyz()
    f = wl.freqs()
    F = sar.forward_rows(wl.positions[3], pix, f)
    assert np.max(np.abs(np.abs(F) - 1.0)) < 1e-12
    R64 = sar.ranges(wl.positions[3], pix)
    R32 = R64.astype(np.float32).astype(np.float64)
    err = np.abs(4 * math.pi * f[-1] * (R64 - R32) / sar.C0)
    assert err.max() > 0.05


def test_conjugate_kernel_and_data_give_conjugate_coefficients():
    """Sign convention (Section II kernel): conj(kernel) with conj(data) gives
    conj(c) and the same |image|."""
    wl = tiny()
    d = sar.echoes(wl)
    a = OnlineFistaOracle.from_workload(wl)
    b = OnlineFistaOracle.from_workload(wl, kernel_sign=+1)
    for p in range(wl.spec.n_pulses):
        a.push_pulse(d[p], p)
        b.push_pulse(np.conj(d[p]), p)
        a.reconstruct(20)
        b.reconstruct(20)
    assert np.allclose(b.c, np.conj(a.c), atol=1e-12, rtol=0)


def test_global_phase_equivariance():
    """d -> e^{i theta} d gives c -> e^{i theta} c (complex soft threshold keeps phase)."""
    wl = tiny()
    d = sar.echoes(wl)
    rot = np.exp(0.7j)
    a = OnlineFistaOracle.from_workload(wl)
    b = OnlineFistaOracle.from_workload(wl)
    for p in range(wl.spec.n_pulses):
        a.push_pulse(d[p], p)
        b.push_pulse(rot * d[p], p)
        a.reconstruct(20)
        b.reconstruct(20)
    assert np.abs(a.c).max() > 0
    assert np.allclose(b.c, rot * a.c, atol=1e-12, rtol=0)


# ---------------------------------------------------------------- dictionary
def test_haar_one_level_2x2_written_out():
    r = 0.5
    expect = np.array([[r, r, r, r],      # LL
                       [r, -r, r, -r],    # low-y, high-x
                       [r, r, -r, -r],    # high-y, low-x
                       [r, -r, -r, r]])   # high-high
    assert np.allclose(dictionary.haar2d_analysis(2, 1), expect)


@pytest.mark.parametrize("n,levels", [(8, 1), (8, 3), (16, 2)])
def test_haar_is_orthonormal(n, levels):
    Psi = dictionary.haar2d_analysis(n, levels)
    assert np.allclose(Psi @ Psi.T, np.eye(n * n), atol=1e-13)


def test_haar_constant_image_lands_on_coarsest_band():
    n, levels = 16, 3
    Psi = dictionary.haar2d_analysis(n, levels)
    coef = (Psi @ np.full(n * n, 3.0)).reshape(n, n)
    m = n >> levels
    assert np.allclose(coef[:m, :m], 3.0 * 2 ** levels)
    coef[:m, :m] = 0
    assert np.abs(coef).max() < 1e-12


def test_haar_single_pixel_pattern():
    """One level on 4x4: pixel (0,0) feeds exactly the four subbands at (0,0)
    of each quadrant with +-1/2."""
    Psi = dictionary.haar2d_analysis(4, 1)
    e = np.zeros(16)
    e[0] = 1.0
    coef = (Psi @ e).reshape(4, 4)
    expect = np.zeros((4, 4))
    expect[0, 0] = expect[0, 2] = expect[2, 0] = expect[2, 2] = 0.5
    assert np.allclose(coef, expect)


# ---------------------------------------------------------------- sufficient statistics
@pytest.mark.parametrize("dict_kind", ["identity", "haar"])
def test_gram_is_hermitian_psd_with_known_diagonal(dict_kind):
    """Delta-A / A_n equations (Section III-C): H_n Hermitian PSD; for W = I,
    |A_ki| = 1 so diag(H_n) = nK; for orthonormal W, trace(H_n) = nKN."""
    wl = tiny(dictionary=dict_kind, haar_levels=2 if dict_kind == "haar" else 0)
    d = sar.echoes(wl)
    o = OnlineFistaOracle.from_workload(wl)
    K, N = wl.spec.n_freq, wl.n_pixels
    for p in range(5):
        o.push_pulse(d[p], p)
    n = 5
    assert np.allclose(o.H, o.H.conj().T, atol=1e-12)
    ev = np.linalg.eigvalsh(o.H)
    assert ev[0] >= -1e-10 * ev[-1]
    if dict_kind == "identity":
        assert np.allclose(np.diag(o.H), n * K, atol=1e-10)
    assert abs(np.trace(o.H).real - n * K * N) < 1e-8 * n * K * N


def test_recursion_equals_batch_statistics():
    """A_n = sum_k G_k^H G_k and b_n = sum_k G_k^H d_k (Section III-C) equal the
    stacked batch products of the Section III-B objective."""
    wl = tiny(dictionary="haar", haar_levels=1)
    d = sar.echoes(wl)
    o = OnlineFistaOracle.from_workload(wl)
    P = wl.spec.n_pulses
    for p in range(P):
        o.push_pulse(d[p], p)
    G, dd = stacked(o, d, P)
    assert np.allclose(o.H, G.conj().T @ G, atol=1e-9)
    assert np.allclose(o.b, G.conj().T @ dd, atol=1e-9)


# ---------------------------------------------------------------- shrink and momentum
def test_soft_threshold_special_cases():
    u = np.array([0.0, 0.3 + 0.4j, -2.0, 1j * 0.5, 3 * np.exp(1j * 1.1)])
    out = soft_threshold(u, 0.5)
    assert out[0] == 0 and out[1] == 0          # |u| < alpha and |u| = alpha -> 0
    assert out[3] == 0                            # tie |u| = alpha -> 0
    assert np.isclose(out[2], -1.5)
    assert np.isclose(out[4], 2.5 * np.exp(1j * 1.1))   # phase kept, modulus shrunk


def test_soft_threshold_is_the_prox_of_the_l1_norm():
    """Brute force: S_a(u) minimises 1/2|x - u|^2 + a|x| over a fine complex grid."""
    rng = np.random.default_rng(1)
    for _ in range(5):
        u = complex(rng.normal(), rng.normal())
        a = 0.4
        xs = np.linspace(-3, 3, 801)
        X = xs[None, :] + 1j * xs[:, None]
        obj = 0.5 * np.abs(X - u) ** 2 + a * np.abs(X)
        best = X.ravel()[np.argmin(obj)]
        assert abs(soft_threshold(np.array([u]), a)[0] - best) < 0.02


def test_momentum_sequence_bounds():
    """Algorithm 1 momentum: t_k >= (k+1)/2 and beta_k = (t_k - 1)/t_{k+1} in [0, 1)."""
    t = 1.0
    for k in range(1, 2000):
        tn = t_next(t)
        beta = (t - 1) / tn
        assert t >= (k + 1) / 2 - 1e-12
        assert 0.0 <= beta < 1.0
        t = tn


# ---------------------------------------------------------------- Lipschitz
C0 = 299_792_458.0


def _ring(n_pix, radius, h=1000.0, phase0=0.3):
    """n_pix pixels on the z = 0 circle of the given radius around the nadir
    of a platform at (0, 0, h): all of them at the same range."""
    a = phase0 + 2 * math.pi * np.arange(n_pix) / n_pix
    return np.stack([radius * np.cos(a), radius * np.sin(a), np.zeros(n_pix)], axis=1)


def test_spectral_norm_equal_ranges_closed_form():
    """Every pixel at one range makes every column of F_s the same unit-modulus
    vector u (|u|^2 = K): F_s F_s^H = N u u^H, so ||F_s||_2^2 = N K exactly,
    while the largest diagonal entry is only N."""
    pos = np.array([0.0, 0.0, 1000.0])
    pix = _ring(7, 35.0)
    f = 9.9e9 + 3.1e6 * np.arange(5)
    A = sar.forward_rows(pos, pix, f)
    assert math.isclose(spectral_norm_sq(A), 7 * 5, rel_tol=1e-12)


def test_spectral_norm_two_ranges_closed_form():
    """Two groups of n1 and n2 pixels at ranges R1, R2: F_s F_s^H =
    n1 a a^H + n2 b b^H with |a|^2 = |b|^2 = K, whose top eigenvalue is that of
    the 2 x 2 Gram of (sqrt(n1) a, sqrt(n2) b):
    (K(n1+n2) + sqrt(K^2 (n1-n2)^2 + 4 n1 n2 |a^H b|^2)) / 2, with a^H b the
    geometric sum  sum_k q^k e^{i w0 dR},  q = e^{i dw dR}."""
    pos = np.array([0.0, 0.0, 1000.0])
    n1, n2 = 5, 3
    pix = np.concatenate([_ring(n1, 20.0), _ring(n2, 40.0, phase0=1.1)])
    f0, df, K = 9.8e9, 1.5e6, 64
    f = f0 + df * np.arange(K)
    R1 = math.hypot(20.0, 1000.0)
    R2 = math.hypot(40.0, 1000.0)
    w0, dw = 4 * math.pi * f0 / C0, 4 * math.pi * df / C0
    q = np.exp(1j * dw * (R1 - R2))
    ab = np.exp(1j * w0 * (R1 - R2)) * (1 - q ** K) / (1 - q)
    expect = (K * (n1 + n2) + math.sqrt(K * K * (n1 - n2) ** 2 + 4 * n1 * n2 * abs(ab) ** 2)) / 2
    A = sar.forward_rows(pos, pix, f)
    got = spectral_norm_sq(A)
    assert math.isclose(got, expect, rel_tol=1e-9)
    # a partly coherent pair: neither the rank-one value nor the larger group alone
    assert K * max(n1, n2) * (1 + 1e-2) < got < K * (n1 + n2) * (1 - 1e-2)


@pytest.mark.parametrize("name", ["small", "haar64"])
def test_spectral_norm_two_frequencies_closed_form(name):
    """K = 2 on a workload's own geometry: F_s F_s^H = [[N, g], [conj g, N]] with
    g = sum_i exp(-i 4 pi (f_0 - f_1) R_i / c0), so ||F_s||_2^2 = N + |g|."""
    wl = make_workload(name)
    pix = wl.pixel_xyz()
    f = wl.freqs()[:2]
    for s in (0, wl.spec.n_pulses - 1):
        R = np.sqrt(np.sum((pix - wl.positions[s]) ** 2, axis=1))
        g = np.sum(np.exp(1j * 4 * math.pi * (f[1] - f[0]) * R / C0))
        expect = wl.n_pixels + abs(g)
        assert math.isclose(spectral_norm_sq(sar.forward_rows(wl.positions[s], pix, f)),
                            expect, rel_tol=1e-11)


@pytest.mark.parametrize("name", ["small", "haar64"])
def test_spectral_norm_between_rayleigh_and_trace(name):
    """On the full workload rows: every Rayleigh quotient |A^H v|^2 of a unit
    vector is below ||A||_2^2, the trace KN above it."""
    wl = make_workload(name)
    A = sar.forward_rows(wl.positions[1], wl.pixel_xyz(), wl.freqs())
    top = spectral_norm_sq(A)
    rng = np.random.default_rng(5)
    K, N = A.shape
    for _ in range(5):
        v = rng.normal(size=K) + 1j * rng.normal(size=K)
        v /= np.linalg.norm(v)
        assert np.linalg.norm(A.conj().T @ v) ** 2 <= top * (1 + 1e-12)
    assert top <= K * N * (1 + 1e-12)


@pytest.mark.parametrize("lip", ["running", "bound"])
@pytest.mark.parametrize("dict_kind", ["identity", "haar"])
def test_step_rule_is_an_upper_bound(lip, dict_kind):
    """Section III-B condition L >= ||sum G^H G||_2 at every pulse, the first
    one included (there L_1 = ||A_s||_2^2 = lambda_max(H_1))."""
    wl = tiny(n_pulses=10, dictionary=dict_kind, haar_levels=2 if dict_kind == "haar" else 0)
    d = sar.echoes(wl)
    o = OnlineFistaOracle.from_workload(wl, lip=lip)
    for p in range(wl.spec.n_pulses):
        o.push_pulse(d[p], p)
        top = np.linalg.eigvalsh(o.H)[-1]
        assert o.L >= top * (1 - 1e-9)
        if p == 0:
            assert math.isclose(o.L, top, rel_tol=1e-9)
        o.reconstruct(20)


@pytest.mark.parametrize("pattern", ["all_then_reconstruct", "reconstruct_zero_between"])
def test_step_rule_with_several_pulses_between_steps(pattern):
    """Pulses pushed with no FISTA step between them still add their
    ||G_n||_2^2 to the bound (Section III-C increments), so L stays above
    lambda_max(H_n) and the iteration stays bounded."""
    wl = tiny(n_pulses=8)
    d = sar.echoes(wl)
    o = OnlineFistaOracle.from_workload(wl)
    if pattern == "all_then_reconstruct":
        schedule = [0] * 7 + [40]
    else:
        schedule = [20, 0, 0, 20, 0, 0, 0, 20]
    for p, iters in enumerate(schedule):
        o.push_pulse(d[p], p)
        assert o.L >= np.linalg.eigvalsh(o.H)[-1] * (1 - 1e-9)
        o.reconstruct(iters)
    assert np.all(np.isfinite(o.c))
    assert np.abs(o.c).max() < 10 * np.abs(wl.rho).max()


# ---------------------------------------------------------------- momentum and warm start
def test_momentum_is_carried_across_pulses():
    """Algorithm 1 starts each pulse from t_{n-1}.  From t' = (1 + sqrt(1 + 4t^2))/2
    follow t + 1/2 <= t' <= t + 1, so after n pulses of m steps from t = 1 the
    carried scalar lies in [1 + nm/2, 1 + nm]; restarting every pulse would keep
    it in [1 + m/2, 1 + m].  Exact start: one step from t = 1 gives the golden
    ratio, the root of t^2 = t + 1."""
    wl = tiny(n_pulses=6)
    d = sar.echoes(wl)
    m = 7
    o = OnlineFistaOracle.from_workload(wl)
    r = OnlineFistaOracle.from_workload(wl, momentum="restart")
    for p in range(wl.spec.n_pulses):
        o.push_pulse(d[p], p)
        r.push_pulse(d[p], p)
        o.reconstruct(m)
        r.reconstruct(m)
        n = p + 1
        assert 1 + n * m / 2 <= o.t <= 1 + n * m
        assert 1 + m / 2 <= r.t <= 1 + m
    # one step per pulse: t_2 = phi (t^2 = t + 1), then t_3 solves t^2 - t = phi^2 = phi + 1
    e = OnlineFistaOracle.from_workload(wl)
    phi = (1 + math.sqrt(5)) / 2
    e.push_pulse(d[0], 0)
    e.reconstruct(1)
    assert math.isclose(e.t, phi, rel_tol=1e-15)
    e.push_pulse(d[1], 1)
    e.reconstruct(1)
    assert math.isclose(e.t, (1 + math.sqrt(5 + 4 * phi)) / 2, rel_tol=1e-15)


def _prox_polar(u, alpha):
    """argmin_x 1/2|x - u|^2 + alpha|x| per entry, solved in polar form:
    keep the phase of u, modulus max(|u| - alpha, 0)."""
    out = np.zeros_like(u)
    for i, ui in enumerate(u):
        r = abs(ui)
        if r > alpha:
            out[i] = (r - alpha) * (ui / r)
    return out


def test_warm_started_steps_by_hand():
    """The first step of pulse n is the forward-backward step from
    z_1 = c_hat_{n-1}; the second extrapolates with beta = (t - 1)/t' from the
    carried t = t_{n-1}.  Both written out here from (c_hat_{n-1}, H_n, b_n)."""
    wl = tiny(n_pulses=5)
    d = sar.echoes(wl)
    o = OnlineFistaOracle.from_workload(wl)
    for p in range(4):
        o.push_pulse(d[p], p)
        o.reconstruct(20)
    o.push_pulse(d[4], 4)
    c0, t0 = o.c.copy(), o.t
    H, b, tau, alpha = o.H.copy(), o.b.copy(), o.tau, o.lam * o.tau
    assert np.abs(c0).max() > 0
    c1 = _prox_polar(c0 - tau * (H @ c0 - b), alpha)
    t1 = (1 + math.sqrt(1 + 4 * t0 * t0)) / 2
    z2 = c1 + (t0 - 1) / t1 * (c1 - c0)
    c2 = _prox_polar(z2 - tau * (H @ z2 - b), alpha)
    keep = (o.c.copy(), o.t, o.w.copy(), o.rho_hat, o.sigma2_acc)
    o.reconstruct(1)
    assert np.allclose(o.c, c1, atol=1e-13 * np.abs(c1).max(), rtol=0)
    o.c, o.t, o.w, o.rho_hat, o.sigma2_acc = keep
    o.reconstruct(2)
    assert np.allclose(o.c, c2, atol=1e-13 * np.abs(c2).max(), rtol=0)
    # a cold start (z_1 = 0) is a different point
    cold = _prox_polar(tau * b, alpha)
    assert np.linalg.norm(cold - c1) > 1e-3 * np.linalg.norm(c1)


def test_phase_correction_undoes_the_phase_error():
    """Section II with a per-pulse phase error: d_s = e^{i phi_s} F_s rho.  Pushing
    it with the correction phi_hat_s = phi_s (data used as d_s e^{-i phi_hat_s})
    reproduces the error-free run; the opposite sign does not."""
    s = spec("autofocus", n_side=8, patch_m=8.0, n_pulses=6, n_freq=16, n_points=3,
             n_lines=0, inner_steps=10)
    wl = make_workload(s)
    assert np.abs(wl.phase_err).max() > 0.1
    d_err = sar.echoes(wl, with_noise=False, with_phase_error=True)
    d_ok = sar.echoes(wl, with_noise=False, with_phase_error=False)
    a = OnlineFistaOracle.from_workload(wl)
    b = OnlineFistaOracle.from_workload(wl)
    c = OnlineFistaOracle.from_workload(wl)
    for p in range(s.n_pulses):
        a.push_pulse(d_ok[p], p)
        b.push_pulse(d_err[p], p, wl.phase_err[p])
        c.push_pulse(d_err[p], p, -wl.phase_err[p])
        for o in (a, b, c):
            o.reconstruct(s.inner_steps)
    assert np.allclose(b.b, a.b, atol=1e-12 * np.abs(a.b).max(), rtol=0)
    assert np.allclose(b.c, a.c, atol=1e-12 * np.abs(a.c).max(), rtol=0)
    assert np.linalg.norm(c.c - a.c) > 1e-2 * np.linalg.norm(a.c)


# ---------------------------------------------------------------- fixed points
def test_single_scatterer_closed_form():
    """Noiseless single scatterer with W = I: the LASSO minimiser is
    (|rho| - lambda/(nK))_+ e^{i arg rho} e_j (KKT holds since |H_ij| <= H_jj = nK).
    Online FISTA plus continuation on the final (H, b) must reach it."""
    s = spec("small", n_side=8, patch_m=8.0, n_pulses=6, n_freq=16, n_points=1)
    wl = make_workload(s)
    d = sar.echoes(wl, with_noise=False)
    o = OnlineFistaOracle.from_workload(wl)
    P, K = s.n_pulses, s.n_freq
    for p in range(P):
        o.push_pulse(d[p], p)
        o.reconstruct(20)
    o.reconstruct(3000)
    j = int(wl.support[0])
    rho = wl.rho[j]
    expect = np.zeros(wl.n_pixels, complex)
    expect[j] = max(abs(rho) - o.lam / (P * K), 0.0) * np.exp(1j * np.angle(rho))
    assert np.allclose(o.c, expect, atol=1e-10)
    # lambda = 0.05 max|A_1^H d_1| = 0.05 K |rho| for one scatterer
    assert math.isclose(o.lam, 0.05 * K * abs(rho), rel_tol=1e-12)


def test_online_plus_continuation_equals_brute_force_lasso():
    """Weighted LASSO of Section III-B solved by coordinate descent on the
    stacked operator (no sufficient statistics) equals the online result after
    the last pulse plus continuation; both satisfy the KKT conditions."""
    wl = tiny(n_pulses=6, n_points=4)
    d = sar.echoes(wl)
    o = OnlineFistaOracle.from_workload(wl)
    P = wl.spec.n_pulses
    for p in range(P):
        o.push_pulse(d[p], p)
        o.reconstruct(20)
    at_m = o.c.copy()
    o.reconstruct(6000)
    G, dd = stacked(o, d, P)
    ref = lasso.solve_cd(G, dd, o.lam, tol=1e-11)
    grad = G.conj().T @ (G @ o.c - dd)
    assert lasso.kkt_residual(grad, o.c, o.lam) < 1e-7
    assert np.linalg.norm(o.c - ref) <= 1e-7 * np.linalg.norm(ref)
    # the m-step result is close to but not at the batch optimum
    assert lasso.objective(G, dd, at_m, o.lam) >= lasso.objective(G, dd, ref, o.lam) - 1e-9


def test_ista_mode_decreases_objective_every_step():
    """Descent lemma: with tau <= 1/L and no momentum every step lowers J_n."""
    wl = tiny(n_pulses=6)
    d = sar.echoes(wl)
    o = OnlineFistaOracle.from_workload(wl, momentum="ista")
    for p in range(wl.spec.n_pulses):
        o.push_pulse(d[p], p)
        J = [o.objective_stats(o.c)]
        for _ in range(20):
            o.reconstruct(1)
            J.append(o.objective_stats(o.c))
        assert all(b <= a + 1e-9 * abs(a) for a, b in zip(J, J[1:]))


def test_restart_mode_fista_rate_envelope():
    """Beck-Teboulle: J(c_k) - J* <= 2 L |c_0 - c*|^2 / (k+1)^2 on a fixed (H, b)."""
    wl = tiny(n_pulses=6)
    d = sar.echoes(wl)
    o = OnlineFistaOracle.from_workload(wl, momentum="restart", lip="exact")
    for p in range(wl.spec.n_pulses):
        o.push_pulse(d[p], p)
    c0 = o.c.copy()
    o.reconstruct(5000)
    cstar = o.c.copy()
    Jstar = o.objective_stats(cstar)
    o.c = c0.copy()
    for k in range(1, 60):
        o.c = c0.copy()
        o.reconstruct(k)
        gap = o.objective_stats(o.c) - Jstar
        assert gap <= 2 * o.L * np.linalg.norm(c0 - cstar) ** 2 / (k + 1) ** 2 + 1e-9


def test_large_lambda_gives_zero():
    """lambda >= max|b_n| makes 0 a KKT point; the shrink keeps c at 0."""
    wl = tiny()
    d = sar.echoes(wl)
    o = OnlineFistaOracle.from_workload(wl, lam=1e9)
    for p in range(wl.spec.n_pulses):
        o.push_pulse(d[p], p)
        o.reconstruct(20)
        assert np.all(o.c == 0)


def test_point_scatterers_land_on_their_pixels():
    """Section IV outcome on the 32x32 workload: the 10 largest |x| are the 10
    true scatterers after 32 pulses at m = 20."""
    wl = make_workload("small")
    d = sar.echoes(wl)
    o = OnlineFistaOracle.from_workload(wl)
    for p in range(wl.spec.n_pulses):
        o.push_pulse(d[p], p)
        o.reconstruct(wl.spec.inner_steps)
    top = np.sort(np.argsort(-np.abs(o.image()))[:10])
    assert np.array_equal(top, np.sort(wl.support))


# ---------------------------------------------------------------- data and accounting
def test_echo_snr_and_noiseless_echo():
    wl = make_workload("small")
    clean = sar.echoes(wl, with_noise=False)
    noisy = sar.echoes(wl)
    ratio = np.sum(np.abs(clean) ** 2) / np.sum(np.abs(noisy - clean) ** 2)
    assert abs(10 * np.log10(ratio) - wl.spec.snr_db) < 0.5
    # noiseless echo is linear in rho: two half scenes add up
    h1 = make_workload("small")
    h1.rho = wl.rho.copy()
    h1.rho[wl.support[5:]] = 0
    h1.support = np.flatnonzero(h1.rho)
    h2 = make_workload("small")
    h2.rho = wl.rho - h1.rho
    h2.support = np.flatnonzero(h2.rho)
    s1 = sar.echoes(h1, with_noise=False)
    s2 = sar.echoes(h2, with_noise=False)
    assert np.allclose(s1 + s2, clean, atol=1e-10)


def test_table1_counts():
    """Table I (Section III-D) counts, recounted from the listed variables:
    c (M), dictionary (M N), stored pulses (n N_r complex each for d, N_r M for
    G, N_r^2 for R) versus A_n (M^2 complex) and b_n (M complex)."""
    for (M, N, Nr, n) in [(1024, 1024, 64, 32), (4096, 4096, 256, 128), (50, 40, 7, 3)]:
        c_and_dict = M + M * N
        per_pulse_complex = Nr + Nr * M + Nr * Nr
        assert memory.fista_values(M, N, Nr, n) == c_and_dict + 2 * n * per_pulse_complex
        assert memory.online_values(M, N) == c_and_dict + 2 * (M * M + M)
    assert abs(memory.crossover_pulses(4096, 256) - 15.1) < 0.05


def test_workload_draws_are_reproducible_and_in_range():
    a = make_workload("haar64")
    b = make_workload("haar64")
    assert np.array_equal(a.rho, b.rho) and np.array_equal(a.noise, b.noise)
    assert len(a.support) > 50  # points plus line pixels
    assert np.all(np.abs(a.rho[a.support]) > 0)
    big = make_workload("large")
    mags = np.abs(big.rho[big.support])
    assert mags.min() >= 0.01 - 1e-12 and mags.max() <= 2.0
    assert np.allclose(np.linalg.norm(a.positions[:, :2], axis=1), 10_000.0)
    assert np.allclose(a.positions[:, 2], 1_000.0)
