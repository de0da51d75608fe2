"""Synthesis dictionaries W (N x M real) with G = F W (test infrastructure).

Section III-A forms the per-pulse operator as G = F H with a real dictionary
(the paper's H; named W here because H names the Gram).  The workloads use
either W = I or an orthonormal separable 2-D Haar basis with a given number of
levels, coefficients in the usual nested (Mallat) layout on the n x n array:
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
mapping to the expected +-2^(-l) pattern.
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


def synthesis_matrix(kind: str, n: int, levels: int = 0) -> np.ndarray | None:
    """W (N x N) for the named dictionary; None stands for the identity."""
    if kind == "identity":
        return None
    if kind == "haar":
        return haar2d_analysis(n, levels).T
    raise ValueError(f"unknown dictionary {kind!r}")
