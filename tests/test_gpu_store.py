"""GPU parity of the store-all-pulses comparator (Section III-D, Table I):
the library's PULSES storage against its GRAM storage (same iterates in exact
arithmetic) and against the FP64 store-all oracle."""

import numpy as np
import pytest

from oracle import sar
from oracle.store_all import StoreAllFistaOracle
from workload import library_kwargs, make_workload, spec

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, np.complex64))).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.complex128)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def maxrel(a, b):
    """Largest element-wise difference over the largest magnitude of b."""
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def gpu(wl, **kw):
    from paper_2603_08582_amd import OnlineFista
    return OnlineFista(**library_kwargs(wl, **kw))


@pytest.mark.parametrize("kind", ["identity", "haar", "edgelet"])
def test_store_all_matches_gram_mode_and_oracle(kind):
    extra = {"haar": dict(dictionary="haar", haar_levels=2),
             "edgelet": dict(dictionary="edgelet", edge_lengths=(4,),
                             edge_rotations_deg=(0.0, 90.0), n_segments=3)}.get(kind, {})
    wl = make_workload(spec("small", n_side=16, patch_m=16.0, n_pulses=7, n_freq=40,
                            n_points=4, phase_error_rad=0.2, **extra))
    d = sar.echoes(wl).astype(np.complex64)
    P, m = wl.spec.n_pulses, 15
    a = gpu(wl)
    b = gpu(wl, storage="pulses", max_pulses=P)
    o = StoreAllFistaOracle.from_workload(wl)
    dd = dev(d)
    for s in range(P):
        ph = 0.05 * s
        a.push_pulse(dd[s], s, ph)
        b.push_pulse(dd[s], s, ph)
        o.push_pulse(d[s].astype(np.complex128), s, ph)
        sa, sb = a.state(), b.state()
        assert abs(sa["L"] - sb["L"]) <= 1e-5 * sa["L"]
        assert abs(sa["lam"] - sb["lam"]) <= 1e-6 * sa["lam"]
        ca = host(a.reconstruct(m))
        cb = host(b.reconstruct(m))
        o.reconstruct(m)
    print(f"{kind}: pulses vs gram {rel(cb, ca):.2e}, pulses vs oracle {rel(cb, o.c):.2e}")
    assert rel(cb, ca) < 2e-5 and maxrel(cb, ca) < 2e-5
    assert rel(cb, o.c) < 1e-4 and maxrel(cb, o.c) < 1e-4
    assert rel(host(b.image()), host(a.image())) < 2e-5


def test_store_all_capacity_and_unsupported_calls():
    from paper_2603_08582_amd import OfistaError
    wl = make_workload(spec("small", n_side=16, patch_m=16.0, n_pulses=4, n_freq=32, n_points=3))
    d = dev(sar.echoes(wl).astype(np.complex64))
    b = gpu(wl, storage="pulses", max_pulses=2)
    b.push_pulse(d[0], 0)
    b.push_pulse(d[1], 1)
    with pytest.raises(OfistaError):
        b.push_pulse(d[2], 2)
    for call in (b.gram, b.export_state, lambda: b.gram_entries([0], [0])):
        with pytest.raises(OfistaError):
            call()
    b.reset()                      # capacity is per image
    b.push_pulse(d[2], 2)
    b.reconstruct(3, copy=False)
