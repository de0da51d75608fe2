"""Synthesis dictionaries W (N x M real) with G = F W (test infrastructure).

Section III-A forms the per-pulse operator as G = F H with a real dictionary
(the paper's H; named W here because H names the Gram).  The workloads use
W = I, the over-complete binary edgelet dictionary of Section III-A, or an
orthonormal separable 2-D Haar basis.

Edgelets (Section III-A; lengths and rotations as in Section IV-A).  An atom
is given by a rotation psi (degrees, converted with the constant pi/180), a
length l in pixels and an integer centre (x0, y0) on the n x n pixel grid
(x = column, y = row, pixel index y*n + x).  Its pixels are the distinct
roundings of the l points

    (x0 + u cos psi, y0 + u sin psi),   u = t - (l - 1)/2,  t = 0 .. l-1,

each coordinate rounded to the nearest integer with ties going down:
floor(v + 0.5 - 1e-9).  (The guard makes the rule immune to one-ulp
differences between cos/sin implementations.)  An atom is kept only if all its
pixels lie on the grid.  Atoms are binary (value 1 on their pixels) and
ordered by rotation, then length (both in the order given), then centre row
y0, then centre column x0.

Haar: coefficients in the usual nested (Mallat) layout on the n x n array:
after one level the top-left quadrant holds low-low, top-right low-in-y /
high-in-x, bottom-left high-in-y / low-in-x, bottom-right high-high, and the
next level recurses on the top-left quadrant.  All coefficients, the coarsest
low-low band included, are penalised alike.

The 1-D analysis step is  lo_i = (x_{2i} + x_{2i+1}) / sqrt(2),
                          hi_i = (x_{2i} - x_{2i+1}) / sqrt(2).

Everything here is built as explicit dense matrices (Kronecker products of
1-D steps), which is slow but checkable by eye.  W is the transpose of the
analysis matrix, so A_s = F_s W applies the analysis to each row of F_s.

Pinned by: W^T W = I; the 2x2 one-level matrix written out; a constant image
mapping to 2^levels times the value on the coarsest band only; a single pixel
mapping to the expected +-2^(-l) pattern.  Edgelets: pixel sets worked out by
hand for horizontal, vertical and diagonal atoms; the atom count n (n - l + 1)
per axis-aligned rotation; length 1 giving W = I.
"""

from __future__ import annotations

import math

import numpy as np


def haar_1d_analysis(n: int) -> np.ndarray:
    """One level of 1-D orthonormal Haar analysis on length n (n even)."""
    if n % 2:
        raise ValueError("length must be even")
    a = np.zeros((n, n))
    r = 1.0 / math.sqrt(2.0)
    for i in range(n // 2):
        a[i, 2 * i] = r
        a[i, 2 * i + 1] = r
        a[n // 2 + i, 2 * i] = r
        a[n // 2 + i, 2 * i + 1] = -r
    return a


def haar2d_analysis(n: int, levels: int) -> np.ndarray:
    """Dense N x N analysis matrix (N = n*n, row-major pixel index iy*n+ix)."""
    if n % (1 << levels):
        raise ValueError("side must be divisible by 2**levels")
    N = n * n
    total = np.eye(N)
    for lev in range(levels):
        m = n >> lev
        one = np.kron(haar_1d_analysis(m), haar_1d_analysis(m))  # on the m x m block
        step = np.eye(N)
        idx = (np.arange(m)[:, None] * n + np.arange(m)[None, :]).ravel()
        step[np.ix_(idx, idx)] = one
        total = step @ total
    return total


DEG = math.pi / 180.0


def edgelet_pixels(n: int, length: int, rot_deg: float, x0: int, y0: int):
    """Sorted distinct pixel indices of one edgelet, or None if it leaves the grid."""
    psi = rot_deg * DEG
    c, s = math.cos(psi), math.sin(psi)
    pix = set()
    for t in range(length):
        u = t - (length - 1) / 2.0
        ix = math.floor(x0 + u * c + 0.5 - 1e-9)
        iy = math.floor(y0 + u * s + 0.5 - 1e-9)
        if not (0 <= ix < n and 0 <= iy < n):
            return None
        pix.add(iy * n + ix)
    return sorted(pix)


def edgelet_atoms(n: int, lengths, rotations_deg) -> list:
    """All atoms of the edgelet dictionary, in dictionary order."""
    atoms = []
    for rot in rotations_deg:
        for length in lengths:
            if not 1 <= length <= n - 1:
                raise ValueError("edgelet length must be in 1 .. n-1")
            for y0 in range(n):
                for x0 in range(n):
                    p = edgelet_pixels(n, int(length), float(rot), x0, y0)
                    if p is not None:
                        atoms.append(p)
    return atoms


def edgelet_synthesis(n: int, lengths, rotations_deg) -> np.ndarray:
    """Binary W (N x M) with W[p, m] = 1 for the pixels p of atom m."""
    atoms = edgelet_atoms(n, lengths, rotations_deg)
    W = np.zeros((n * n, len(atoms)))
    for m, pix in enumerate(atoms):
        W[pix, m] = 1.0
    return W


def synthesis_matrix(kind: str, n: int, levels: int = 0, lengths=(), rotations=()) -> np.ndarray | None:
    """W (N x M) for the named dictionary; None stands for the identity."""
    if kind == "identity":
        return None
    if kind == "haar":
        return haar2d_analysis(n, levels).T
    if kind == "edgelet":
        return edgelet_synthesis(n, lengths, rotations)
    raise ValueError(f"unknown dictionary {kind!r}")
