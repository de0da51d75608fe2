"""Write the oracle's expected outputs for the full-size workloads.

Calls only the oracle and the workload generator.  Run from the repository
root:  python tests/golden/make_golden.py haar64   (or large, autofocus)
(large: 256 pulses with a 4.3 GB complex128 H, about half an hour on 8 cores)
Output: tests/golden/<name>_oracle.npz with the final coefficients c_hat,
the image x = W c_hat, and per-pulse L_n, lambda, rho; for "autofocus" the
loss gradients to lambda and to the per-pulse phase corrections instead.
"""

import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

from oracle import sar  # noqa: E402
from oracle.online_fista import OnlineFistaOracle  # noqa: E402
from workload import make_workload  # noqa: E402


def autofocus(name: str = "autofocus"):
    """Gradients of the magnitude loss (final |x| vs the true |rho|) to lambda
    and to the per-pulse phase corrections, evaluated at zero corrections with
    lambda = lambda_rel max|A_1^H d_1| (which does not depend on the phases)."""
    from oracle import adjoint
    wl = make_workload(name)
    d = sar.echoes(wl).astype(np.complex64).astype(np.complex128)
    o = OnlineFistaOracle.from_workload(wl)
    o.push_pulse(d[0], 0)
    lam = o.lam
    phases = np.zeros(wl.spec.n_pulses)
    t0 = time.time()
    L, gl, gp = adjoint.gradients(wl, d, lam, phases, wl.spec.inner_steps, np.abs(wl.rho))
    print(f"gradients in {time.time() - t0:.1f}s: L={L} dL/dlam={gl}")
    out = Path(__file__).with_name(f"{name}_oracle.npz")
    np.savez_compressed(out, lam=np.array(lam), loss=np.array(L), grad_lambda=np.array(gl),
                        grad_phase=gp)
    print("wrote", out)


def main(name: str):
    wl = make_workload(name)
    d = sar.echoes(wl).astype(np.complex64).astype(np.complex128)
    o = OnlineFistaOracle.from_workload(wl)
    t0 = time.time()
    L, lam, rho = [], [], []
    for p in range(wl.spec.n_pulses):
        o.push_pulse(d[p], p)
        L.append(o.L)
        lam.append(o.lam)
        o.reconstruct(wl.spec.inner_steps)
        rho.append(o.rho_hat)
        if p % 16 == 0 or p == wl.spec.n_pulses - 1:
            print(f"pulse {p} {time.time() - t0:.1f}s", flush=True)
    out = Path(__file__).with_name(f"{name}_oracle.npz")
    np.savez_compressed(out, c=o.c, image=o.image(), L=np.array(L), lam=np.array(lam),
                        rho=np.array(rho), t=np.array(o.t))
    print("wrote", out)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "haar64"
    if which == "autofocus":
        autofocus()
    else:
        main(which)
