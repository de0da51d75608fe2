"""Stored-value counts of Table I (Section III-D), test infrastructure.

Table I counts the real values each method must keep after n pulses, with
complex values counted twice (its footnote):

    batch FISTA:  M (N + 1) + 2 n N_r (1 + M + N_r)     (c, dictionary, {d_k, G_k, R_k})
    Online FISTA: M (N + 1) + 2 M (M + 1)               (c, dictionary, A_n, b_n)

N pixels, M atoms, N_r samples per pulse.  Pinned by recounting the listed
variables' element counts directly.
"""


def fista_values(M: int, N: int, Nr: int, n: int) -> int:
    return M * (N + 1) + 2 * n * Nr * (1 + M + Nr)


def online_values(M: int, N: int) -> int:
    return M * (N + 1) + 2 * M * (M + 1)


def crossover_pulses(M: int, Nr: int) -> float:
    """n beyond which Online FISTA stores fewer values: M(M+1) / (Nr (1+M+Nr))."""
    return M * (M + 1) / (Nr * (1 + M + Nr))
