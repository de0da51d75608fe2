"""Pins of the collection session (Section IV-A: Bernoulli pulse selection,
early stop at the ideal large-coefficient count) and of the evaluation of
Section IV-B (BP baseline, large-coefficient count, SNR)."""

import math

import numpy as np

from oracle import dictionary, sar, session
from oracle.online_fista import OnlineFistaOracle
from workload import make_workload, spec


def test_bernoulli_selection_is_the_trial_outcome():
    u = make_workload("session32").select_u
    for p in (0.0, 0.1, 0.5, 1.0):
        got = session.bernoulli_positions(u, p)
        want = [s for s in range(len(u)) if u[s] < p]
        assert list(got) == want
    assert session.bernoulli_positions(u, 1.0).size == len(u)
    assert session.bernoulli_positions(u, 0.0).size == 0
    # 1000 trials at p = 0.1: the count lies well inside the binomial bulk
    n = session.bernoulli_positions(u, 0.1).size
    assert abs(n - 100) < 5 * math.sqrt(1000 * 0.1 * 0.9)


def test_full_selection_equals_the_plain_run():
    wl = make_workload(spec("small", n_side=8, patch_m=8.0, n_pulses=6, n_freq=16, n_points=3))
    d = sar.echoes(wl)
    o, pushed, counts, stop = session.run_session(wl, d=d, p=1.0, m=10, ideal=0)
    ref = OnlineFistaOracle.from_workload(wl)
    for s in range(6):
        ref.push_pulse(d[s], s)
        ref.reconstruct(10)
    assert pushed == list(range(6)) and stop is None
    assert np.array_equal(o.c, ref.c)
    assert counts[-1] == int(np.sum(np.abs(ref.c) > 2e-2))


def test_stop_is_the_first_pulse_at_the_ideal_count():
    wl = make_workload(spec("session32", n_pulses=400))
    d = sar.echoes(wl)
    full, pushed, counts, _ = session.run_session(wl, d=d, ideal=0)
    first = counts.index(4)
    o, pushed4, counts4, stop = session.run_session(wl, d=d, ideal=4)
    assert stop == first and pushed4 == pushed[: first + 1] and counts4 == counts[: first + 1]


def test_backprojection_of_a_single_scatterer():
    """Noiseless single scatterer at pixel j: (1/n) sum F^H F rho has K rho_j
    at j (every |F_kj| = 1)."""
    wl = make_workload(spec("small", n_side=8, patch_m=8.0, n_pulses=5, n_freq=16, n_points=1))
    d = sar.echoes(wl, with_noise=False)
    bp = session.backprojection(wl, d, range(5))
    j = int(wl.support[0])
    assert abs(bp[j] - 16 * wl.rho[j]) <= 1e-12 * abs(16 * wl.rho[j])


def test_backprojection_is_b_over_n_for_the_identity_dictionary():
    wl = make_workload(spec("small", n_side=8, patch_m=8.0, n_pulses=7, n_freq=16, n_points=4))
    d = sar.echoes(wl)
    o = OnlineFistaOracle.from_workload(wl)
    for s in (0, 2, 3, 6):
        o.push_pulse(d[s], s)
    bp = session.backprojection(wl, d, (0, 2, 3, 6))
    assert np.allclose(bp, o.b / 4, rtol=0, atol=1e-12 * np.max(np.abs(o.b)))


def test_snr_closed_forms():
    x = np.full(10, 0.1 + 0j)
    x[[2, 5]] = 2.0
    # mu_signal = 4, mu_noise = 0.01 -> 20 log10(400)
    assert math.isclose(session.snr_db(x, [2, 5]), 20 * math.log10(400.0), rel_tol=1e-12)
    assert session.snr_db(np.where(np.arange(10) < 3, 1.0, 0.0), [0, 1, 2]) == math.inf
    assert session.large_count([0.03, -0.02, 0.019, 0.021j, 0.0]) == 2
    assert session.to_db([10.0])[0] == 20.0


def test_session32_settles_on_the_square():
    """Section IV-B outcome on the one-square scene: the large-coefficient count
    reaches the ideal 4 and the run stops there; the four atoms are the
    square's sides; Online FISTA's SNR beats BP's after the same pulses."""
    wl = make_workload("session32")
    s = wl.spec
    sel = session.bernoulli_positions(wl.select_u, s.bernoulli_p)
    d = sar.echoes(wl, pulses=sel)
    o, pushed, counts, stop = session.run_session(wl, d=d)
    assert stop is not None and counts[-1] == 4 and len(pushed) < len(sel)
    top = np.argsort(-np.abs(o.c))[:4]
    W = dictionary.synthesis_matrix("edgelet", 32, lengths=(4,), rotations=(0.0, 90.0))
    assert np.array_equal(np.flatnonzero(W[:, top].sum(axis=1)), wl.support)
    snr_ofista = session.snr_db(o.image(), wl.support)
    snr_bp = session.snr_db(session.backprojection(wl, d, pushed), wl.support)
    assert snr_ofista > snr_bp + 20


# ---------------------------------------------------------------- store-all comparator
def test_store_all_trajectory_equals_online():
    """Section III-D comparator: sum_k G_k^H (G_k z - d_k) = H_n z - b_n, so the
    stored-pulse method follows the Online FISTA trajectory (same lambda, L
    rule and momentum) up to rounding."""
    from oracle.store_all import StoreAllFistaOracle
    wl = make_workload(spec("haar64", n_side=16, patch_m=16.0, n_pulses=6, n_freq=24,
                            n_points=4, n_lines=1, haar_levels=2))
    d = sar.echoes(wl)
    a = OnlineFistaOracle.from_workload(wl)
    b = StoreAllFistaOracle.from_workload(wl)
    for s in range(6):
        a.push_pulse(d[s], s, 0.1 * s)
        b.push_pulse(d[s], s, 0.1 * s)
        assert math.isclose(a.L, b.L, rel_tol=1e-10) and math.isclose(a.lam, b.lam, rel_tol=1e-12)
        a.reconstruct(15)
        b.reconstruct(15)
        assert np.linalg.norm(a.c - b.c) <= 1e-10 * np.linalg.norm(a.c)


def test_store_all_counts_table1():
    from oracle import memory
    from oracle.store_all import StoreAllFistaOracle
    wl = make_workload(spec("small", n_side=8, patch_m=8.0, n_pulses=5, n_freq=16, n_points=2))
    d = sar.echoes(wl)
    b = StoreAllFistaOracle.from_workload(wl)
    for s in range(5):
        b.push_pulse(d[s], s)
        assert b.stored_values() == memory.fista_values(64, 64, 16, s + 1)
