"""FP64 CPU oracle for Online FISTA -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously-correct numpy (complex128 / float64)
statement of what the per-pulse hot path of Online FISTA computes:

* ``sar``          the discretised SAR forward model (Section II, eqs. for the
                   FIO d = F[rho] and the phase phi = t - 2|gamma(s) - x|/c) and
                   the synthetic echo d_s = F_s rho + noise;
* ``dictionary``   the synthesis dictionary W (identity, or an orthonormal
                   multi-level 2-D Haar basis) so that G = F W (Section III-A,
                   eq. for G);
* ``online_fista`` the recursive sufficient statistics (Section III-C, the
                   Delta-A / Delta-b and A_n / b_n equations), the Lipschitz
                   step (Section III-B spectral-norm bound and the incremental
                   bound of Section III-C) and Algorithm 1;
* ``lasso``        an independent batch solver of the weighted-LASSO objective
                   (Section III-B) used only to pin the online result;
* ``memory``       the stored-value counts of Table I.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  The GPU library shares no code with it; both
consume the seeded draws of the separate ``workload`` package.

Parity status per function is stated in each module header.  The full
trajectory of Algorithm 1 at m inner steps is "parity unpinned" as a whole:
no closed form exists for it, so its parts are pinned separately (Hermitian
PSD Gram, batch identity, closed-form single-scatterer fixed point, KKT
certificate, brute-force batch LASSO after continuation, ISTA-mode descent,
scatterers landing on their pixels, phase equivariance, Lipschitz upper bound,
closed-form spectral norms, momentum carried across pulses, warm start, and
the sign of the autofocus phase correction).
"""

from . import dictionary, lasso, memory, sar
from .online_fista import OnlineFistaOracle, soft_threshold, spectral_norm_sq

__all__ = ["dictionary", "lasso", "memory", "sar", "OnlineFistaOracle",
           "soft_threshold", "spectral_norm_sq"]
