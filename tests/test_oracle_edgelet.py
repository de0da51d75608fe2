"""Pins of the oracle's edgelet dictionary (Section III-A; the lengths and
rotations of Section IV-A) and of Online FISTA run with it.

Pixel sets are worked out by hand from the atom definition (centre, rotation,
length, rounding with ties going down); counts follow from the same
definition in closed form; length 1 reduces to the identity dictionary.  The
runs check the over-complete problem against an independent batch solver (the
fitted signal and the objective value are unique even where the coefficients
are not) and on a scene built from two atoms.
"""

import numpy as np
import pytest

from oracle import dictionary, lasso, sar
from oracle.online_fista import OnlineFistaOracle
from workload import make_workload, spec


def test_pixels_worked_by_hand():
    n = 10
    # horizontal, even length 4 centred on (5, 3): u = -1.5 .. 1.5 -> x = 3 .. 6
    assert dictionary.edgelet_pixels(n, 4, 0.0, 5, 3) == [33, 34, 35, 36]
    # odd length 5 centred on (4, 2): x = 2 .. 6
    assert dictionary.edgelet_pixels(n, 5, 0.0, 4, 2) == [22, 23, 24, 25, 26]
    # vertical: y = 1 .. 4 in column 5
    assert dictionary.edgelet_pixels(n, 4, 90.0, 5, 3) == [15, 25, 35, 45]
    # diagonal, length 3 centred on (5, 5): (4, 4), (5, 5), (6, 6)
    assert dictionary.edgelet_pixels(n, 3, 45.0, 5, 5) == [44, 55, 66]
    # anti-diagonal (135 deg): cos < 0 < sin -> (6, 4), (5, 5), (4, 6)
    assert dictionary.edgelet_pixels(n, 3, 135.0, 5, 5) == [46, 55, 64]
    # leaving the grid
    assert dictionary.edgelet_pixels(n, 4, 0.0, 1, 3) is None
    assert dictionary.edgelet_pixels(n, 4, 0.0, 9, 3) is None


@pytest.mark.parametrize("n,l", [(8, 2), (10, 4), (12, 5), (16, 6)])
def test_axis_aligned_counts(n, l):
    """An axis-aligned atom spans l consecutive pixels, so n - l + 1 centres
    per line fit: M = n (n - l + 1) per rotation."""
    atoms = dictionary.edgelet_atoms(n, (l,), (0.0, 90.0))
    assert len(atoms) == 2 * n * (n - l + 1)
    for a in atoms[: len(atoms) // 2]:           # horizontal: consecutive indices in one row
        assert len(a) == l and np.all(np.diff(a) == 1) and a[0] // n == a[-1] // n
    for a in atoms[len(atoms) // 2:]:            # vertical: stride n
        assert len(a) == l and np.all(np.diff(a) == n)


def test_order_and_binary_columns():
    W = dictionary.synthesis_matrix("edgelet", 8, lengths=(2, 4), rotations=(0.0,))
    assert set(np.unique(W)) == {0.0, 1.0}
    # rotation, then length, then centre row, then centre column
    assert W.shape == (64, 8 * 7 + 8 * 5)
    assert np.array_equal(np.flatnonzero(W[:, 0]), [0, 1])        # l = 2 at (1, 0)
    assert np.array_equal(np.flatnonzero(W[:, 56]), [0, 1, 2, 3])  # l = 4 at (2, 0)
    assert np.array_equal(W.sum(axis=0), np.r_[np.full(56, 2.0), np.full(40, 4.0)])


def test_length_one_is_the_identity():
    W = dictionary.synthesis_matrix("edgelet", 6, lengths=(1,), rotations=(0.0,))
    assert np.array_equal(W, np.eye(36))


def test_length_one_run_equals_identity_run():
    """With length-1 atoms the whole online run is the identity-dictionary run."""
    wl = make_workload(spec("small", n_side=8, patch_m=8.0, n_pulses=4, n_freq=16, n_points=3))
    d = sar.echoes(wl)
    a = OnlineFistaOracle.from_workload(wl)
    b = OnlineFistaOracle.from_workload(wl)
    b.W = dictionary.synthesis_matrix("edgelet", 8, lengths=(1,), rotations=(0.0,))
    for p in range(4):
        a.push_pulse(d[p], p)
        b.push_pulse(d[p], p)
        a.reconstruct(10)
        b.reconstruct(10)
    assert np.allclose(a.c, b.c, rtol=0, atol=1e-13)


def test_over_complete_online_plus_continuation_matches_batch_lasso():
    """Section III-B with an over-complete W (M = 112 > N = 64): online FISTA
    after the last pulse plus continuation and coordinate descent on the
    stacked operator reach the same objective and the same fitted signal."""
    s = spec("small", n_side=8, patch_m=8.0, n_pulses=6, n_freq=16, n_points=0,
             n_segments=3, segment_px=(2, 4), dictionary="edgelet", edge_lengths=(2,),
             edge_rotations_deg=(0.0, 90.0))
    wl = make_workload(s)
    d = sar.echoes(wl)
    o = OnlineFistaOracle.from_workload(wl)
    assert o.M == 112
    for p in range(s.n_pulses):
        o.push_pulse(d[p], p)
        o.reconstruct(20)
    o.reconstruct(20000)
    G = np.concatenate([o.rows(p) for p in range(s.n_pulses)], axis=0)
    dd = np.concatenate([d[p] for p in range(s.n_pulses)])
    ref = lasso.solve_cd(G, dd, o.lam, tol=1e-10)
    grad = G.conj().T @ (G @ o.c - dd)
    assert lasso.kkt_residual(grad, o.c, o.lam) < 1e-6
    J, Jr = lasso.objective(G, dd, o.c, o.lam), lasso.objective(G, dd, ref, o.lam)
    assert abs(J - Jr) <= 1e-9 * abs(Jr)
    assert np.linalg.norm(G @ o.c - G @ ref) <= 1e-5 * np.linalg.norm(G @ ref)


def test_scene_of_two_atoms_is_recovered():
    """Noiseless scene equal to two disjoint atoms (Section IV's squares and
    lines are unions of atoms): after the pulses and continuation the two
    largest coefficients are those atoms."""
    s = spec("small", n_side=12, patch_m=12.0, n_pulses=12, n_freq=32, n_points=0,
             dictionary="edgelet", edge_lengths=(4,), edge_rotations_deg=(0.0, 90.0))
    wl = make_workload(s)
    W = dictionary.synthesis_matrix("edgelet", 12, lengths=(4,), rotations=(0.0, 90.0))
    m1 = 3 * 9 + 4              # horizontal, centre (6, 3): pixels 40 .. 43
    m2 = 12 * 9 + 5 * 12 + 8    # vertical, centre (8, 7): column 8, rows 5 .. 8
    assert not set(np.flatnonzero(W[:, m1])) & set(np.flatnonzero(W[:, m2]))
    wl.rho = W[:, m1] * (0.9 * np.exp(0.4j)) + W[:, m2] * (0.7 * np.exp(-1.1j))
    wl.support = np.flatnonzero(wl.rho)
    d = sar.echoes(wl, with_noise=False)
    o = OnlineFistaOracle.from_workload(wl)
    for p in range(s.n_pulses):
        o.push_pulse(d[p], p)
        o.reconstruct(20)
    o.reconstruct(3000)
    top = set(np.argsort(-np.abs(o.c))[:2].tolist())
    assert top == {m1, m2}
