"""Online FISTA throughput on one MI355X: pulses/s on the 64x64 Haar workload.

One step = one whole image: reset of the online state, then for each of the
P = 128 pulses push_pulse (rows, Haar fold, b and Gram update, L_n) and
reconstruct(20) (20 fused matvec/shrink/momentum steps).  Echoes are
synthesised on the device before timing (inputs resident in HBM).  The
timed steps replay one HIP graph captured from the library's stream (the
same kernels in the same order; --launch stream launches them one by one).

Prints one JSON line with the metric, a roofline entry for the dominant
kernel (per-launch durations from HIP events on the library's stream) and
the FP64 oracle timed on the host as a reported CPU baseline.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = "pulses/sec (Gram update + 20 FISTA iters) at 64×64 scene; % HBM/MFMA peak"
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
# FP32 vector FMA without the packed (two-per-lane) form the kernels are built
# without: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 78.6
BF16_MFMA_PEAK_TFLOPS = 2500.0  # dense
# rocprofv3 FETCH_SIZE / WRITE_SIZE summary of the haar64 workload: a fenced
# JSON block holds, per kernel class, the scaled HBM bytes per launch and a
# hash of the sources those counters were taken on
TRAFFIC_FILE = ROOT / "profiles" / "traffic-haar64.md"


def source_hash(files) -> str:
    h = hashlib.sha256()
    for rel in files:
        h.update((ROOT / rel).read_bytes())
    return h.hexdigest()[:16]


def traffic_for(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary, or None when
    absent, for another workload, or taken on different kernel sources."""
    if workload != "haar64" or not TRAFFIC_FILE.exists():
        return None
    m = re.search(r"```json\n(.*?)\n```", TRAFFIC_FILE.read_text(), re.S)
    rec = json.loads(m.group(1)).get(kernel) if m else None
    if not rec or rec.get("source_sha") != source_hash(rec.get("files", [])):
        return None
    return rec.get("bytes_per_launch")


def host_description():
    """CPU model and the BLAS numpy is linked against (reported with the
    oracle's baseline)."""
    model = "unknown"
    try:
        for line in Path("/proc/cpuinfo").read_text().splitlines():
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = "unknown"
    try:
        cfg = np.show_config(mode="dicts")
        b = cfg.get("Build Dependencies", {}).get("blas", {})
        blas = f"{b.get('name', '?')} {b.get('version', '')}".strip()
    except Exception:
        pass
    return model, blas


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max((i.get("num_threads", 1) for i in threadpool_info()
                    if i.get("user_api") == "blas"), default=1)
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline(wl, pulses: int, positions=None, diff: bool = False, runs: int = 5):
    """The FP64 oracle as it stands, on the first `pulses` pulses (of
    `positions` when given: the Bernoulli-selected ones of a session): one
    untimed warm-up pulse, then `runs` timed runs from a fresh oracle, median
    reported.  With diff, the oracle's forward run plus its reverse pass for
    dL/dlambda and dL/dphase over those pulses (the differentiation form's
    step)."""
    from oracle import sar
    from oracle.online_fista import OnlineFistaOracle
    threads = blas_threads()
    model, blas = host_description()
    order_all = list(range(wl.spec.n_pulses)) if positions is None else [int(p) for p in positions]
    order = order_all[:pulses]
    d = sar.echoes(wl, pulses=order)
    m = wl.spec.inner_steps
    warm = OnlineFistaOracle.from_workload(wl)
    warm.push_pulse(d[order[0]], order[0])
    warm.reconstruct(m)
    times = []
    for _ in range(runs):
        o = OnlineFistaOracle.from_workload(wl)
        if diff:
            from oracle import adjoint
            o.push_pulse(d[0], 0)
            lam = o.lam
            t0 = time.perf_counter()
            adjoint.gradients(wl, d, lam, np.zeros(len(order)), m, np.abs(wl.rho),
                              pulses=len(order))
        else:
            t0 = time.perf_counter()
            for p in order:
                o.push_pulse(d[p], p)
                o.reconstruct(m)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    what = (f"recorded forward ({m} FISTA steps per pulse) and the reverse pass for "
            f"dL/dlambda and dL/dphase" if diff else f"push + {m} FISTA steps each")
    return {"value": len(order) / dt, "unit": "pulses/s", "cores": int(threads), "kind": "oracle",
            "sample": f"first {len(order)} of the {len(order_all)} pulses of the same workload "
                      f"({what}), numpy complex128; one warm-up pulse, median of {runs} runs "
                      f"of {dt:.2f} s (min {min(times):.2f}, max {max(times):.2f})",
            "cpu_model": model, "blas": blas, "runs": runs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="haar64")
    ap.add_argument("--cpu-pulses", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--step-kernel", default="auto", choices=("auto", "launches", "resident"),
                    help="how the FISTA steps run (the library's step_kernel setting)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="BLAS threads of the oracle baseline (0: the library's default, all cores)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (the reference "
                         "kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--launch", default="graph", choices=("graph", "stream"),
                    help="graph: capture one step (reset + all pulses) from the library's "
                         "stream into a HIP graph once and time its replays (plain Gram "
                         "workloads; sessions and the differentiation form always launch); "
                         "stream: launch every kernel of every step")
    ap.add_argument("--table1", action="store_true",
                    help="instead of the metric: time one pulse (push + m steps) at growing n "
                         "for the Gram (Online FISTA) and the stored-pulse comparator, with "
                         "their workspace sizes (Table I), as one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding of "
              "Online FISTA (row blocks of H per GPU, one exchange of z per step) is a design, "
              "not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_08582_amd import OnlineFista
    from workload import library_kwargs, make_workload

    wl = make_workload(args.workload)
    if args.table1:
        return table1(wl, args)
    s = wl.spec
    N, K, P, m = s.n_pixels, s.n_freq, s.n_pulses, s.inner_steps
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # the differentiation form (record_every > 0): one step is the forward run
    # with checkpoints plus the reverse pass for dL/dlambda and dL/dphases
    diff_mode = s.record_every > 0
    session_mode = s.bernoulli_p < 1.0 or s.ideal_count > 0
    # sessions take host decisions between pulses and the differentiation form
    # synchronises inside its step: those launch from the stream
    graph_mode = (args.launch == "graph" and not diff_mode and not session_mode
                  and args.step_kernel != "resident")
    if graph_mode:
        # capture needs a stream other than the null stream; everything of
        # this run goes to it, so no cross-stream ordering is involved
        torch.cuda.set_stream(torch.cuda.Stream(dev))
    g = OnlineFista(device=dev, **(library_kwargs(wl, record_every=s.record_every, max_pulses=P,
                                                  max_iters=m) if diff_mode
                                   else library_kwargs(wl, step_kernel=args.step_kernel)))
    stream = g.stream

    # a collection session (Section IV-A): Bernoulli-selected positions and an
    # early stop at the ideal large-coefficient count; otherwise every position
    if session_mode:
        from paper_2603_08582_amd import session as sess
        sched = sess.bernoulli_schedule(wl.select_u, s.bernoulli_p)
    else:
        sched = np.arange(P)

    # inputs: echoes synthesised on the device from the seeded scene and noise
    rho = torch.from_numpy(wl.rho.astype(np.complex64)).to(dev)
    noise = torch.from_numpy(wl.noise.astype(np.complex64)).to(dev)
    d = torch.zeros((P, K), dtype=torch.complex64, device=dev)
    for p in sched:
        g.echo(int(p), rho, noise[p], s.snr_db, float(wl.phase_err[p]), out=d[p])
    torch.cuda.synchronize()

    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    pulses_per_step = [P]
    if diff_mode:
        target = torch.from_numpy(np.abs(wl.rho).astype(np.float32)).to(dev)
        phases = np.zeros(P)
        g.reset()
        g.push_pulse(d[0], 0)
        torch.cuda.synchronize()
        lam_abs = g.state()["lam"]   # lambda of the relative rule, then held as an absolute value
        diff_split = {"forward_ms": 0.0, "loss_ms": 0.0, "backward_ms": 0.0, "n": 0}

    def step():
        g.reset()
        if diff_mode:
            # forward: the recorded online run at the absolute lambda
            g.set_lambda(lam_abs)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e2 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for p in range(P):
                g.push_pulse(d[p], p, float(phases[p]))
                g.reconstruct(m, copy=False)
            e1.record(stream)
            x = g.image()
            # gradient of sum (|x| - |rho|)^2 (the caller's loss, plain tensor ops)
            mag = x.abs()
            gx = (2.0 * (mag - target) / mag.clamp_min(1e-30)) * x
            em = torch.cuda.Event(enable_timing=True)
            em.record(stream)
            g.backward(gx.contiguous())
            e2.record(stream)
            torch.cuda.synchronize()
            diff_split["forward_ms"] += e0.elapsed_time(e1)
            diff_split["loss_ms"] += e1.elapsed_time(em)
            diff_split["backward_ms"] += em.elapsed_time(e2)
            diff_split["n"] += 1
            return
        if session_mode:
            res = sess.run_session(g, d, sched, m, ideal=s.ideal_count, threshold=s.large_thresh)
            pulses_per_step[0] = len(res["pushed"])
            return
        for p in range(P):
            g.push_pulse(d[p], p)
            g.reconstruct(m, copy=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if diff_mode:  # the split covers the timed steps only (the first run loads code)
        diff_split.update(forward_ms=0.0, loss_ms=0.0, backward_ms=0.0, n=0)
    timed = step
    if graph_mode:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            step()
        graph.replay()  # first replay uploads the graph: untimed
        torch.cuda.synchronize()
        timed = graph.replay
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record(stream)
    for k in range(args.steps):
        timed()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[-1]) / args.steps
    step_ms_each = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    if diff_mode:
        diff_timed = dict(diff_split)

    # per-kernel durations: the same steps again with HIP events around every
    # launch of the Gram update and of the FISTA step (library stream).  Not
    # under rocprofv3 counter collection: event-attached launches are the
    # suspected trigger of a fault seen in such a pass.
    under_counters = bool(os.environ.get("ROCPROF_COUNTER_COLLECTION"))
    res_ms, res_n, res_steps = 0.0, 0, 0
    if not under_counters:
        g.profile(True)
        for _ in range(args.steps):
            step()
        gram_ms, gram_n = g.kernel_time("gram")
        step_ms, step_n = g.kernel_time("step")
        res_ms, res_n = g.kernel_time("resident")
        g.profile(False)
        res_steps = args.steps * pulses_per_step[0] * m if res_n else 0
    else:
        gram_ms, gram_n, step_ms, step_n = float("nan"), 0, float("nan"), 0
    x = g.image()
    torch.cuda.synchronize()
    finite = bool(torch.isfinite(torch.view_as_real(x)).all().item())

    gram_avg = gram_ms / max(gram_n, 1)
    step_avg = step_ms / max(step_n, 1)
    M = g.M                                     # coefficients (= N except for edgelets)
    gram_flops = 4.0 * K * M * (M + 1)          # Hermitian upper triangle, per pulse
    step_bytes = 4.0 * M * (M + 1)              # upper-triangle complex64 H, per FISTA step
    # MFMA work the Gram kernels issue: every stored 64 x 64 tile (diagonal
    # tiles whole) over all K frequencies
    nbt = (M + 63) // 64
    tile_macs = K * 64 * 64 * nbt * (nbt + 1) // 2
    if s.precision == "split_bf16":
        # three BF16 products (hi*hi + hi*lo + lo*hi) of the four real products
        # of each complex product: 12 real multiply-adds per complex one
        issued = 2.0 * 12 * tile_macs
        rl_gram = {"bound": "mfma", "achieved": issued / (gram_avg * 1e-3) / 1e12,
                   "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "dtype": "bf16x3",
                   "traffic": None, "kernel": "k_gram_bf16x3", "avg_ms": gram_avg,
                   "launches": gram_n,
                   "algorithmic_tflops": gram_flops / (gram_avg * 1e-3) / 1e12,
                   "form": "achieved and frac count the BF16 flops the matrix cores issue "
                           "(12 real products per complex product over the stored tiles); "
                           "algorithmic_tflops the 4KN(N+1) of the FP32 product"}
    else:
        # Gauss's form: three real products per complex product
        issued = 2.0 * 3 * tile_macs
        rl_gram = {"bound": "mfma", "achieved": issued / (gram_avg * 1e-3) / 1e12,
                   "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "dtype": "fp32",
                   "traffic": traffic_for("gram", args.workload), "kernel": "k_gram_fp32",
                   "avg_ms": gram_avg, "launches": gram_n,
                   "algorithmic_tflops": gram_flops / (gram_avg * 1e-3) / 1e12,
                   "form": "achieved and frac count the FP32 flops the matrix cores issue "
                           "(three real products per complex product over the stored tiles); "
                           "algorithmic_tflops the 4KN(N+1) of the complex product"}
    if res_n:
        # resident steps: one launch runs every step of a reconstruct call; the
        # per-step time is the kernel time over the steps it ran.  The tile
        # pass reads most of H from LDS and L2, so the bound is the FP32 FMA
        # work: 16 FMAs per stored complex entry of the tiles (H z, H^H z,
        # H w, H^H w), against the vector FMA peak.
        step_avg = res_ms / max(res_steps, 1)
        step_flops = 2.0 * 16 * 64 * 64 * nbt * (nbt + 1) // 2
        rl_step = {"bound": "alu", "achieved": step_flops / (step_avg * 1e-3) / 1e12,
                   "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "traffic": traffic_for("resident", args.workload),
                   "kernel": "k_steps_resident", "avg_ms": step_avg, "launches": res_n,
                   "steps": res_steps, "hbm_equivalent_GBs": step_bytes / (step_avg * 1e-3) / 1e9,
                   "form": "per FISTA step: kernel time / steps run; achieved = FP32 flops of "
                           "the four products over the stored tiles; hbm_equivalent_GBs = the "
                           "4M(M+1) bytes of the upper triangle over the step time (H is read "
                           "from LDS and L2, not HBM)"}
        step_ms = res_ms
    else:
        rl_step = {"bound": "hbm", "achieved": step_bytes / (step_avg * 1e-3) / 1e9,
                   "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": traffic_for("step", args.workload),
                   "kernel": "k_step_tiles", "avg_ms": step_avg, "launches": step_n}
    for r in (rl_gram, rl_step):
        r["frac"] = r["achieved"] / r["peak"]
        if not np.isfinite(r["achieved"]):  # no per-kernel timing (counter collection)
            for k in ("achieved", "frac", "avg_ms", "algorithmic_tflops"):
                if k in r:
                    r[k] = None
    dominant, other = (rl_gram, rl_step) if gram_ms > step_ms else (rl_step, rl_gram)

    if s.dictionary == "edgelet":
        dict_desc = (f"edgelet(lengths {'/'.join(map(str, s.edge_lengths))}, rotations "
                     f"{'/'.join(f'{r:g}' for r in s.edge_rotations_deg)} deg)")
    elif s.dictionary == "haar":
        dict_desc = f"haar({s.haar_levels})"
    else:
        dict_desc = "identity"
    out = {
        "metric": METRIC,
        "value": pulses_per_step[0] / (ms * 1e-3),
        "unit": "pulses/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": f"{s.name}: {s.n_side}x{s.n_side} pixels (N={N}), "
                               f"{dict_desc} dictionary (M={M}), K={K}, "
                               + (f"session over {P} positions: Bernoulli p={s.bernoulli_p:g} "
                                  f"selects {len(sched)}, stop at {s.ideal_count} large "
                                  f"coefficients after {pulses_per_step[0]} pulses"
                                  if session_mode else f"P={P} pulses")
                               + f", m={m} FISTA steps per pulse, one step = one image",
                   "N": N, "M": M, "K": K, "pulses": pulses_per_step[0], "positions": P,
                   "inner_steps": m, "seed": s.seed, "generator": "numpy PCG64",
                   "storage": "packed Hermitian upper tiles 64x64, complex64",
                   "step_kernel": args.step_kernel,
                   "launch": "HIP graph replay of the captured step" if graph_mode
                             else "stream launches",
                   "parallelism": "single GPU"},
        "fista_iters_per_s": pulses_per_step[0] * m / (ms * 1e-3),
        "median_ms_per_step": float(np.median(step_ms_each)),
        "min_ms_per_step": float(np.min(step_ms_each)),
        "roofline": {k: dominant[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_kernel": dominant["kernel"],
        "roofline_other": other,
        "roofline_dominant_detail": {"avg_ms": dominant["avg_ms"], "launches": dominant["launches"]},
        "image_finite": finite,
    }
    if diff_mode:
        n = max(diff_timed["n"], 1)
        out["differentiation"] = {
            "gradients_per_s": 1e3 / ms, "forward_ms": diff_timed["forward_ms"] / n,
            "loss_ms": diff_timed["loss_ms"] / n,
            "backward_ms": diff_timed["backward_ms"] / n,
            "backward_over_forward": diff_timed["backward_ms"] / max(diff_timed["forward_ms"], 1e-9),
            "checkpoint_every": s.record_every,
            "what": "one step = recorded forward over all pulses (forward_ms) + image and loss "
                    "gradient (loss_ms) + reverse pass for dL/dlambda and dL/dphase with "
                    "L = sum(|x| - |rho|)^2 (backward_ms)"}
    if not args.no_cpu_baseline:
        limit = None
        if args.cpu_threads > 0:
            from threadpoolctl import threadpool_limits
            limit = threadpool_limits(limits=args.cpu_threads, user_api="blas")
        out["cpu_baseline"] = cpu_baseline(wl, min(args.cpu_pulses, 8) if diff_mode else args.cpu_pulses,
                                           sched if session_mode else None, diff=diff_mode)
        if limit is not None:
            limit.restore_original_limits()
    print(json.dumps(out), flush=True)


def table1(wl, args):
    """Section III-D / Table I comparison on one GPU: for n = 1, 2, 4, ... up to
    the workload's pulse count, the time of pulse n (push + m FISTA steps) and
    the workspace of each method holding n pulses."""
    import torch
    from paper_2603_08582_amd import OnlineFista, workspace_bytes
    from paper_2603_08582_amd.ofista import make_config
    from workload import library_kwargs
    s = wl.spec
    P, K, m = s.n_pulses, s.n_freq, s.inner_steps
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ns = sorted({1 << i for i in range(P.bit_length()) if (1 << i) <= P} | {P})
    out = {"table1": s.name, "K": K, "inner_steps": m, "n": ns, "gram": {}, "pulses": {}}
    rho = torch.from_numpy(wl.rho.astype(np.complex64)).to(dev)
    noise = torch.from_numpy(wl.noise.astype(np.complex64)).to(dev)
    for mode in ("gram", "pulses"):
        kw = library_kwargs(wl, storage=mode, max_pulses=P) if mode == "pulses" else library_kwargs(wl)
        g = OnlineFista(device=dev, **kw)
        d = torch.empty((P, K), dtype=torch.complex64, device=dev)
        for p in range(P):
            g.echo(p, rho, noise[p], s.snr_db, float(wl.phase_err[p]), out=d[p])
        times, mem = [], []
        for n in ns:
            g.reset()
            for p in range(n - 1):
                g.push_pulse(d[p], p)
                g.reconstruct(m, copy=False)
            torch.cuda.synchronize()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record(g.stream)
            g.push_pulse(d[n - 1], n - 1)
            g.reconstruct(m, copy=False)
            t1.record(g.stream)
            torch.cuda.synchronize()
            times.append(t0.elapsed_time(t1))
            cfg = make_config(**(library_kwargs(wl, storage=mode, max_pulses=n) if mode == "pulses"
                                 else library_kwargs(wl)))[0]
            mem.append(workspace_bytes(cfg))
        out[mode] = {"ms_per_pulse": times, "workspace_bytes": mem, "M": g.M}
        g.close()
        del d
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
