"""Stream capture: reset + pushes + reconstructs captured from the library's
stream into a HIP graph and replayed.  Every replay (with eager device work
and synchronisations between replays) must give the eager run's image,
coefficients and scalars bit for bit, for ofista_reconstruct and for the
allocation-free ofista_reconstruct_static, with the identity, Haar and
edgelet dictionaries and with the store-all comparator.
"""

import numpy as np
import pytest

from oracle import sar
from workload import library_kwargs, make_workload, spec

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def sequence(g, d, pulses, iters, static):
    g.reset()
    for p in pulses:
        g.push_pulse(d[p], p)
        if static:
            g.reconstruct_static(iters, copy=False)
        else:
            g.reconstruct(iters, copy=False)


def snapshot(g):
    out = dict(image=g.image(), c=g.vector("c"), w=g.vector("w"))
    torch.cuda.synchronize()
    return {k: v.clone() for k, v in out.items()}


EDGE = dict(n_side=16, patch_m=16.0, n_pulses=8, n_freq=32, n_points=0, n_segments=4,
            dictionary="edgelet", edge_lengths=(2, 4), edge_rotations_deg=(0.0, 90.0))

CASES = [
    ("small", dict(), [0, 5, 9, 14], 20, False, {}),
    ("small", dict(n_side=30, patch_m=28.0), [0, 3, 7], 15, False, {}),
    ("small", dict(), [0, 6, 12], 20, True, {}),
    ("haar64", dict(), [0, 40, 80], 20, False, {}),
    # the edgelet rows, Gram and image kernels
    ("small", EDGE, [0, 3, 6], 15, False, {}),
    # the store-all comparator's passes over the stored pulses
    ("small", dict(), [0, 4, 8], 10, False, dict(storage="pulses", max_pulses=3)),
]


@pytest.mark.parametrize("name,over,pulses,iters,static,kw", CASES)
def test_graph_replay_matches_eager_bitwise(name, over, pulses, iters, static, kw):
    from paper_2603_08582_amd import OnlineFista
    wl = make_workload(spec(name, **over)) if over else make_workload(name)
    dev = torch.device("cuda", 0)
    side = torch.cuda.Stream(dev)
    print(f"{name} {over} pulses {pulses} iters {iters} static {static} {kw}", flush=True)
    with torch.cuda.stream(side):
        d = torch.from_numpy(sar.echoes(wl, pulses=pulses).astype(np.complex64)).to(dev)
        g = OnlineFista(stream=side, **library_kwargs(wl, **kw))
        sequence(g, d, pulses, iters, static)
        ref = snapshot(g)
        ref_state = g.state()
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=side):
        sequence(g, d, pulses, iters, static)
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        for r in range(3):
            graph.replay()
            torch.cuda.synchronize()
            got = snapshot(g)
            for k in ref:
                assert torch.equal(got[k].view(torch.float32), ref[k].view(torch.float32)), (r, k)
            st = g.state()
            for k in ("L", "tau", "lam", "rho", "sigma2", "t"):
                assert st[k] == ref_state[k], (r, k, st[k], ref_state[k])
            # eager device work between replays
            x = torch.randn(1 << 20, device=dev)
            assert torch.isfinite(x.sum()).item()
    del g, graph
    torch.cuda.empty_cache()
