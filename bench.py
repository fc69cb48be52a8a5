#!/usr/bin/env python3
"""Throughput of the PMRF EM path on one MI355X.

A step is one full optimisation of the 2048 x 2048 slice with ~100k Voronoi
regions (L = 2, beta = 0.5, 30 EM iterations, FP64 energies, int32 labels):
starting labels and parameters are restored from device-resident copies, then
pmrf_em_run executes all 30 iterations.  Inputs are resident in HBM before the
timed region.  The metric is vertex-label energy evaluations per second
(M neighbourhood elements x L labels x iterations per step).

Printed as one JSON line on stdout.  The roofline object is the dominant kernel
(one EM iteration per launch): algorithmic bytes per launch divided by the
average launch duration, the duration coming from HIP events that the library
records around each launch on its stream during the timed region.  The CPU
baseline is the serial FP64 oracle on the same problem (EM loop only).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "vertex-label energy evals/sec + HBM GB/s % peak; batched vs plain at bit-exact labels"
HBM_PEAK_GBS = 8000.0
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_iter_slice2048_100k_traffic.md")
BATCH_COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_iter_batch64_traffic.md")
POWERLAW_COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_iter_powerlaw16_traffic.md")
KERNEL_SRC = os.path.join(ROOT, "paper_1809_05018_amd", "csrc", "em.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def alg_bytes(info) -> int:
    """Algorithmic bytes of one EM iteration: neighbourhood offsets and adjacency
    offsets (4 B each per neighbourhood), member ids (4 B), in-neighbourhood
    degree (1 B) and local neighbour indices (1 B per adjacency entry), the
    intensities (8 B), current labels (4 B), new labels (4 B) and the parameter
    update's re-read of intensities and labels (12 B) per vertex, one 8-byte
    energy sum per neighbourhood: 16 H + 5 M + A + 28 n."""
    return 16 * info.H + 5 * info.M + info.A + 28 * info.n


def kernel_sha() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic(path=None):
    """HBM bytes per launch (read + written) from a committed counter summary
    (default: the single-slice one), if it was taken on the current kernel
    source; else None.  The summary holds one line ``traffic: {json}`` with
    ``kernel_sha`` and ``bytes_per_launch``."""
    try:
        lines = open(path or COUNTERS_FILE).read().splitlines()
    except OSError:
        return None
    for line in lines:
        if line.startswith("traffic: "):
            try:
                d = json.loads(line[len("traffic: "):])
            except ValueError:
                return None
            if d.get("kernel_sha") != kernel_sha():
                return None
            return d.get("bytes_per_launch")
    return None


def copy_calibration(dev, mib=256, reps=3):
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters: each copy reads and writes ``mib`` MiB."""
    import torch

    a = torch.ones(mib << 17, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": mib << 20, "copies": reps}), flush=True)


def cpu_baseline(g, L, beta, iters, x0, M, runs=3):
    """The oracle's EM loop on the same problem, on one host core (the process
    is pinned to one core while it runs): the median of ``runs`` full runs."""
    import numpy as np

    import oracle

    og = oracle.OracleGraph(g.n, g.row_ptr, g.col_idx)
    pinned = None
    if hasattr(os, "sched_getaffinity"):
        pinned = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {min(pinned)})
    try:
        times, ref = [], None
        for _ in range(runs):
            t0 = time.perf_counter()
            ref = og.em_run(g.y, L, beta, x0, np.zeros(L), np.ones(L), iters, init_from_labels=True)
            times.append(time.perf_counter() - t0)
    finally:
        if pinned is not None:
            os.sched_setaffinity(0, pinned)
    dt = float(np.median(times))
    return ref, {"value": M * L * iters / dt, "unit": "evals/s", "cores": 1, "kind": "oracle",
                 "sample": f"the full workload, {iters} EM iterations, median of {runs} runs on one pinned core "
                           f"({sum(times):.1f} s); serial C oracle (-O2), EM loop only",
                 "seconds_per_run": round(dt, 3), "cpu": host_cpu()}


def host_cpu() -> dict:
    """CPU model and the cores this process may use, for the baseline records."""
    model = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"model": model, "cores_available": cores}


def cpu_baseline_parallel(graphs, L, beta, iters, threads):
    """The oracle's EM loop on one graph per host thread (the graphs are
    independent, so this is the embarrassingly parallel CPU rate): the first
    ``threads`` graphs of the workload, ``iters`` iterations each, all at once;
    graph construction is outside the timing (EM loop only).  Returns the
    baseline record and the oracle's results, graph by graph."""
    import concurrent.futures as cf

    import numpy as np

    import oracle
    from paper_1809_05018_amd import synth

    sample = graphs[:threads]
    # built one after another: the oracle's clique sort keeps its comparison
    # context in file-level variables, so only its EM loop may run concurrently
    ogs = [oracle.OracleGraph(g.n, g.row_ptr, g.col_idx) for g in sample]

    def run(i):
        g = sample[i]
        x0 = synth.threshold_labels(g.y, L)
        return ogs[i].em_run(g.y, L, beta, x0, np.zeros(L), np.ones(L), iters, init_from_labels=True)

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(len(sample)) as ex:  # the C EM loop runs without the GIL
        refs = list(ex.map(run, range(len(sample))))
    dt = time.perf_counter() - t0
    evals = sum(og.M for og in ogs) * L * iters
    return {"value": evals / dt, "unit": "evals/s", "cores": len(sample), "kind": "oracle",
            "sample": f"{len(sample)} of the workload's graphs, one per thread, {iters} EM iterations each "
                      f"({dt:.1f} s wall); serial C oracle (-O2) per graph, EM loop only",
            "cpu": host_cpu()}, refs


def parity_block(gpu, refs):
    """GPU results against the oracle's, graph by graph (same start, same
    iterations): labels must be identical unless the oracle counted a near tie
    (energy gap below 1e-9, where either label is correct and the runs may
    drift apart); mu, sigma and the energy trace are compared where the labels
    agree."""
    import numpy as np

    def rel(a, b):
        a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
        if a.size == 0:
            return 0.0
        return float(np.max(np.abs(a - b) / np.maximum(np.maximum(np.abs(a), np.abs(b)), 1e-300)))

    eq = [bool(np.array_equal(a["x"], b["x"])) for a, b in zip(gpu, refs)]
    ties = [int(b["total_near_ties"]) for b in refs]
    same = [i for i, e in enumerate(eq) if e]
    errs = {k: max([rel(gpu[i][k], refs[i][k]) for i in same] or [0.0]) for k in ("mu", "sigma", "trace")}
    ok = all(e or t > 0 for e, t in zip(eq, ties)) and all(v <= 1e-10 for v in errs.values()) and all(
        a["iters"] == b["iters"] for a, b in zip(gpu, refs))
    return {"graphs": len(refs), "iters": int(refs[0]["iters"]) if refs else 0, "ok": ok,
            "graphs_labels_bit_exact": sum(eq), "graphs_with_near_ties": sum(t > 0 for t in ties),
            "near_ties": sum(ties), "mu_rel": errs["mu"], "sigma_rel": errs["sigma"], "trace_rel": errs["trace"],
            "bar": "labels identical unless the oracle counted a near tie (gap < 1e-9); mu, sigma, trace within 1e-10 relative"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--iters", type=int, default=30, help="EM iterations per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="default workload only: skip the 64-slice batched-vs-plain leg")
    ap.add_argument("--workload", default="slice2048_100k",
                    choices=["slice2048_100k", "batch64", "powerlaw16", "serving", "image2048", "volume256",
                             "build"],
                    help="default: the single 100k-region slice, followed by the 64-slice batched leg; "
                         "the others print their own JSON line")
    ap.add_argument("--requests", type=int, default=128, help="serving: number of requests")
    ap.add_argument("--launch", default=None,
                    help="pin the launch shape 'mode,waves_per_block,blocks_per_cu' instead of autotuning "
                         "(for profiles of one shape)")
    ap.add_argument("--workers", type=int, default=0,
                    help="processes drawing the batch inputs (0: the cores available, at most 16; 1 draws in "
                         "this process with a progress line per graph, as profiler runs need)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (scale for the HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the EM path of one graph runs on one device and the library "
              "has no multi-GPU path (independent graphs would go whole to separate GPUs; one huge graph "
              "would be split by cliques with a label halo). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    from paper_1809_05018_amd import synth

    workers = args.workers if args.workers > 0 else max(1, min(16, host_cpu()["cores_available"]))
    progress = (lambda i, k: log(f"  drew {i}/{k}")) if workers == 1 else None
    # inputs are drawn before the GPU is touched (worker processes are forked)
    graphs = None
    if args.workload == "slice2048_100k":
        log("generating the 2048x2048 / 100k-region slice")
        g = synth.workload_large()
        if not args.no_batch:
            log("generating 64 slices (sides log-uniform in [512, 2560])")
            graphs = synth.workload_batch(64, 3, workers=workers, progress=progress)
    elif args.workload == "batch64":
        log("generating 64 slices (sides log-uniform in [512, 2560])")
        graphs = synth.workload_batch(64, 3, workers=workers, progress=progress)
    elif args.workload == "powerlaw16":
        log("generating 16 power-law graphs of 500k vertices")
        graphs = synth.workload_skewed(16, 500_000, 4, workers=workers, progress=progress)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        return copy_calibration(dev)
    if args.workload in ("batch64", "powerlaw16"):
        out = batched_leg(args, dev, args.workload, graphs)
        print(json.dumps(out), flush=True)
        return
    if args.workload == "serving":
        return bench_serving(args, dev)
    if args.workload in ("image2048", "volume256"):
        return bench_image(args, dev)
    if args.workload == "build":
        return bench_build(args, dev)
    result = bench_slice(args, dev, g)
    if graphs is not None:
        leg = batched_leg(args, dev, "batch64", graphs)
        result["batched_over_plain"] = leg["batched_over_plain"]
        result["bitwise_equal_plain_batched"] = leg["bitwise_equal_plain_batched"]
        result["batch64"] = leg
    print(json.dumps(result), flush=True)


def bench_slice(args, dev, g):
    """The 100k-region slice: 30 EM iterations per step (the headline figure)."""
    import numpy as np
    import torch

    from paper_1809_05018_amd import pmrf, synth

    L, beta, iters = 2, 0.5, args.iters
    x0 = synth.threshold_labels(g.y, L)
    prob = pmrf.Problem(g.n, g.row_ptr, g.col_idx, g.y, L, dev)
    info = prob.hoods.info
    log(f"n={info.n} H={info.H} M={info.M} A={info.A} max_hood={info.max_hood} tiles={info.tiles}")

    # starting parameters: the parameter update of the threshold labels, on the device
    prob.set_state(x0, np.zeros(L), np.ones(L))
    prob.run(pmrf.pmrf_em_params(L=L, beta=beta, max_iters=0, init_from_labels=True))
    torch.cuda.synchronize()
    state0 = prob.state.clone()  # starting labels and parameters
    params = pmrf.pmrf_em_params(L=L, beta=beta, max_iters=iters)
    prob.prepare(params)

    def step():
        prob.state.copy_(state0)
        prob.run(params)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region 1: throughput (default launch mode, no timing events)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    out = prob.results(params)
    assert out["status"] == 0, out["status"]
    # per-step times (each step synchronised on its own), for the median
    per_step = []
    for _ in range(10):
        t = time.perf_counter()
        step()
        torch.cuda.synchronize()
        per_step.append(time.perf_counter() - t)
    # timed region 2: the same steps with HIP events around every EM-iteration
    # kernel on its stream (the library then launches directly, without a graph)
    pmrf.pmrf_profile_begin()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed_ev = time.perf_counter() - t1
    ev_ms, launches = pmrf.pmrf_profile_end()
    out_ev = prob.results(params)
    assert np.array_equal(out_ev["x"], out["x"]) and np.array_equal(out_ev["mu"], out["mu"])
    evals_per_step = info.M * L * iters
    value = evals_per_step * args.steps / elapsed
    ms_step = elapsed / args.steps * 1e3
    avg_launch_s = ev_ms * 1e-3 / max(1, launches)
    b_launch = alg_bytes(info)
    achieved = b_launch / avg_launch_s / 1e9
    log(f"{ms_step:.3f} ms/step, {value:.4g} evals/s, k_iter avg {avg_launch_s * 1e6:.2f} us over {launches} launches "
        f"({elapsed_ev / args.steps * 1e3:.3f} ms/step with timing events)")

    result = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "slice2048_100k", "image": "2048x2048 two-phase, seed 2", "regions": info.n,
                   "neighbourhoods": info.H, "elements": info.M, "labels": L, "beta": beta, "em_iters": iters,
                   "mode": "HIP graph, one iteration kernel per EM iteration"},
        "step_ms_median": float(np.median(per_step)) * 1e3,
        "per_iteration": {"alg_bytes": b_launch, "us": ms_step * 1e3 / iters,
                          "frac": b_launch * iters / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "note": "algorithmic bytes of all iterations of a step over the whole step's wall time"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "k_iter<2>", "alg_bytes_per_launch": b_launch,
                     "avg_launch_us": avg_launch_s * 1e6, "launches_timed": launches,
                     "timing": "HIP events stamped with each EM iteration's kernel dispatch begin and end (hipExtLaunchKernel), second timed region of the same steps"},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        log("timing the serial oracle on the same workload")
        ref, cpu = cpu_baseline(g, L, beta, iters, x0, info.M)
        result["cpu_baseline"] = cpu
        result["parity"] = parity_block([out], [ref])
        result["speedup_vs_oracle"] = value / cpu["value"]
    return result


def build_all(graphs, workers=8):
    """Neighbourhoods of many graphs on host threads (the builder releases the GIL)."""
    import concurrent.futures as cf

    from paper_1809_05018_amd import pmrf

    with cf.ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda g: pmrf.pmrf_build_neighborhoods(g.n, g.row_ptr, g.col_idx), graphs))


def batched_leg(args, dev, workload, graphs):
    """Many graphs: one pmrf_em_run per graph in sequence ("plain") against one
    pmrf_em_batch over all of them ("batched"), same starting state, same
    iterations; results must be bitwise equal.  The oracle runs the first 16
    graphs (all iterations of the slices; all 40 iterations of two power-law
    graphs) for the CPU baseline and the parity block."""
    import numpy as np
    import torch

    from paper_1809_05018_amd import pmrf, synth

    if workload == "batch64":
        L, beta, iters = 2, 0.5, 30
        cfg = {"workload": "batch64", "slices": len(graphs), "sides": "log-uniform 512..2560, seed 3",
               "regions_per_slice": "side^2/26.2", "labels": L, "beta": beta, "em_iters": iters}
    else:
        L, beta, iters = 4, 0.8, 40
        cfg = {"workload": "powerlaw16", "graphs": len(graphs), "vertices": 500_000,
               "degrees": "P(d)~d^-2.5 on [3,30]", "labels": L, "beta": beta, "em_iters": iters}
    t0 = time.perf_counter()
    hoods = build_all(graphs)
    log(f"neighbourhoods built in {time.perf_counter() - t0:.1f} s")
    probs, starts = [], []
    for g, h in zip(graphs, hoods):
        prob = pmrf.Problem(g.n, g.row_ptr, g.col_idx, g.y, L, dev, hoods=h)
        x0 = synth.threshold_labels(g.y, L)
        prob.set_state(x0, np.zeros(L), np.ones(L))
        prob.run(pmrf.pmrf_em_params(L=L, beta=beta, max_iters=0, init_from_labels=True))
        starts.append((prob.labels.clone(), prob.mu.clone(), prob.sigma.clone()))
        probs.append(prob)
    torch.cuda.synchronize()
    params = pmrf.pmrf_em_params(L=L, beta=beta, max_iters=iters)
    for p in probs:
        p.prepare(params)
    M = sum(h.M for h in hoods)
    b_iter = sum(alg_bytes(h.info) for h in hoods)
    evals = M * L * iters
    log(f"graphs={len(graphs)} n={sum(h.n for h in hoods)} M={M} alg bytes/iter={b_iter / 1e9:.3f} GB")

    def reset():
        for p, (x, mu, sg) in zip(probs, starts):
            p.labels.copy_(x)
            p.mu.copy_(mu)
            p.sigma.copy_(sg)

    def plain():
        reset()
        for p in probs:
            p.run(params)

    items = [p.item(params) for p in probs]
    ws = torch.empty(pmrf.pmrf_em_batch_workspace_bytes(items), dtype=torch.uint8, device=dev)

    def batched():
        reset()
        pmrf.pmrf_em_batch(items, ws)

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    steps = max(1, min(args.steps, 5))
    # each path runs with the launch shape the autotuner finds fastest for it
    # (results are independent of the shape), unless a shape is pinned
    saved = pmrf.pmrf_get_launch()
    if args.launch:
        mode, waves, bpc = (int(v) for v in args.launch.split(","))
        shape_plain = shape_batch = (mode, waves, 0, bpc)
        pmrf.pmrf_set_launch(*shape_plain)
        tune = {}
    else:
        shape_plain, _ = pmrf.autotune_launch(plain, reps=1)
    t_plain = timed(plain, steps)
    res_plain = [p.results(params) for p in probs]
    if not args.launch:
        shape_batch, tune = pmrf.autotune_launch(batched, reps=2)
    t_batch = timed(batched, steps)
    res_batch = [p.results(params) for p in probs]
    log(f"launch shapes: plain {shape_plain}, batched {shape_batch} "
        f"({', '.join(f'{k}: {v * 1e3:.2f} ms' for k, v in tune.items())})")
    same = all(np.array_equal(a[k], b[k]) for a, b in zip(res_plain, res_batch) for k in ("x", "mu", "sigma", "trace"))
    pmrf.pmrf_profile_begin()
    batched()
    torch.cuda.synchronize()
    ev_ms, launches = pmrf.pmrf_profile_end()
    pmrf.pmrf_set_launch(**saved)
    avg = ev_ms * 1e-3 / max(1, launches)
    achieved = b_iter / avg / 1e9
    log(f"plain {t_plain * 1e3:.2f} ms/step, batched {t_batch * 1e3:.2f} ms/step, ratio {t_plain / t_batch:.2f}, "
        f"iteration kernels {avg * 1e6:.1f} us")
    out = {"metric": METRIC, "value": evals / t_batch, "unit": "evals/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": t_batch * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": cfg,
           "plain": {"value": evals / t_plain, "ms_per_step": t_plain * 1e3},
           "batched_over_plain": t_plain / t_batch, "bitwise_equal_plain_batched": same,
           "launch_shape": {"plain": list(shape_plain), "batched": list(shape_batch),
                            "fields": "mode, waves_per_block, tiles_per_wave, blocks_per_cu"},
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS,
                        "traffic": measured_traffic(BATCH_COUNTERS_FILE if workload == "batch64"
                                                    else POWERLAW_COUNTERS_FILE),
                        "kernel": (f"k_iter<{4 if L > 2 else 2}> batched" +
                                   (" (the superchunks of neighbourhoods above 64 members in the same launch)"
                                    if L > 2 else " (+ k_iter_packets where a graph has neighbourhoods above 64 "
                                    "members)")),
                        "alg_bytes_per_launch": b_iter, "avg_launch_us": avg * 1e6, "launches_timed": launches,
                        "timing": "HIP events around each EM iteration's work kernels, one batched run"},
           "cpu_baseline": None}
    if not args.no_cpu_baseline:
        threads = max(1, min(16, host_cpu()["cores_available"], len(graphs)))
        # a bounded sample: all iterations of 16 slices; all 40 iterations of
        # two of the large power-law graphs
        sample = threads if workload == "batch64" else min(2, len(graphs))
        log(f"timing the oracle on {sample} graphs in parallel ({iters} iterations each)")
        cpu, refs = cpu_baseline_parallel(graphs, L, beta, iters, sample)
        out["cpu_baseline"] = cpu
        out["speedup_vs_oracle"] = out["value"] / cpu["value"]
        out["parity"] = parity_block(res_batch[: len(refs)], refs)
    return out


def bench_image(args, dev):
    """Image in, graph out: the region adjacency graph and region means of the
    2048 x 2048 slice with its 100k-region oversegmentation (inputs resident
    on the device), then the labels painted back and the confusion counts
    against the generating phases."""
    import numpy as np
    import torch

    from paper_1809_05018_amd import pmrf, synth

    if args.workload == "volume256":
        # 256 slices of 256 x 256, each oversegmented on its own (ids offset per
        # slice), so regions meet across slices as well as within them
        log("generating a 256^3 volume (256 slices, 2,500 regions each)")
        labs, imgs, phs, off = [], [], [], 0
        for z in range(256):
            im, lb, p_ = synth.image_slice(6000 + z, 256, 2500)
            labs.append(lb + off)
            imgs.append(im)
            phs.append(p_)
            off += int(lb.max()) + 1
        lab, img, ph = np.stack(labs).astype(np.int32), np.stack(imgs), np.stack(phs)
    else:
        log("generating the 2048x2048 image and its 100k-region oversegmentation")
        img, lab, ph = synth.image_slice(2, 2048, 100_000)
    n = int(lab.max()) + 1
    h, w = lab.shape[-2:]
    npix = lab.size
    r = torch.from_numpy(lab).to(dev)
    p = torch.from_numpy(img).to(dev)
    truth = torch.from_numpy(ph.astype(np.uint8)).to(dev)
    ws = torch.empty(pmrf.pmrf_volume_graph_workspace_bytes(w, h, npix // (h * w), n), dtype=torch.uint8, device=dev)
    labels = torch.from_numpy(synth.threshold_labels(np.zeros(n), 2)).to(dev)

    def step():
        row_ptr, col_idx, means = pmrf.image_graph(r, p, n, ws)
        seg = pmrf.labels_to_pixels(r, labels, n)
        counts = pmrf.confusion(seg, truth, 2)
        return row_ptr, col_idx, means, counts

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    steps = max(1, args.steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    row_ptr, col_idx, means, _ = out
    nnz = int(col_idx.numel())
    # algorithmic bytes of the graph call: region ids and pixels read once,
    # the CSR and the means written once
    b_alg = 5 * npix + 4 * (n + 1) + 4 * nnz + 8 * n
    achieved = b_alg / dt / 1e9
    log(f"{dt * 1e3:.3f} ms per {args.workload} (graph, means, paint, confusion), nnz={nnz}")
    result = {
        "metric": "image-to-graph pixels/s (region adjacency graph + region means + paint + confusion)",
        "value": npix / dt, "unit": "pixels/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32/u8 in, f64 means", "data": "synthetic",
        "config": {"workload": args.workload,
                   "image": "2048x2048 two-phase, seed 2" if args.workload == "image2048"
                   else "256 slices of 256x256 two-phase, seeds 6000+z, 6-connected",
                   "regions": n, "adjacency": nnz},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "whole graph call",
                     "alg_bytes_per_launch": b_alg,
                     "note": "wall time of the whole step, which waits for the host once (entry count, id check)"},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        from oracle import image as oi

        t1 = time.perf_counter()
        ref_ptr, ref_col = oi.region_graph(lab, n)
        ref_means = oi.region_means(lab, img, n)
        cpu = time.perf_counter() - t1
        result["cpu_baseline"] = {"value": npix / cpu, "unit": "pixels/s", "cores": 1, "kind": "oracle",
                                  "sample": f"graph and means of the full {args.workload}, once (NumPy oracle)"}
        result["parity"] = {"graph_equal": bool(np.array_equal(row_ptr.cpu().numpy(), ref_ptr)
                                                and np.array_equal(col_idx.cpu().numpy(), ref_col)),
                            "means_equal": bool(np.array_equal(means.cpu().numpy(), ref_means))}
    print(json.dumps(result), flush=True)


def bench_build(args, dev):
    """Neighbourhood construction (maximal cliques, 1-neighbourhoods, owners,
    packed device layout) on the device against the host builder, for the
    100k-region slice and one 500k-vertex power-law graph; the device build
    starts from the CSR resident in device memory and ends with the layout
    there, the host build from the CSR in host memory."""
    import numpy as np
    import torch

    from paper_1809_05018_amd import pmrf, synth

    log("generating the 100k-region slice and a 500k-vertex power-law graph")
    graphs = {"slice2048_100k": synth.workload_large(), "powerlaw_500k": synth.powerlaw_graph(4, 500_000)}
    steps = max(1, args.steps)
    rows = {}
    for name, g in graphs.items():
        rp = torch.from_numpy(np.asarray(g.row_ptr, np.int32)).to(dev)
        ci = torch.from_numpy(np.asarray(g.col_idx, np.int32)).to(dev)
        for _ in range(max(1, args.warmup)):
            d = pmrf.pmrf_build_neighborhoods_device(g.n, rp, ci)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            d = pmrf.pmrf_build_neighborhoods_device(g.n, rp, ci)
        dev_s = (time.perf_counter() - t0) / steps
        host_runs = max(1, min(3, steps))
        t0 = time.perf_counter()
        for _ in range(host_runs):
            h = pmrf.pmrf_build_neighborhoods(g.n, g.row_ptr, g.col_idx)
        host_s = (time.perf_counter() - t0) / host_runs
        a, b = d.upload(dev), h.upload(dev)
        same = (d.device_bytes == h.device_bytes and bool(torch.equal(a[: h.device_bytes], b[: h.device_bytes])))
        rows[name] = {"n": g.n, "nnz": int(g.row_ptr[-1]), "H": d.H, "M": d.M, "max_hood": d.max_hood,
                      "device_ms": dev_s * 1e3, "host_ms": host_s * 1e3, "host_over_device": host_s / dev_s,
                      "layout_equal_to_host_builder": same}
        log(f"{name}: device {dev_s * 1e3:.2f} ms, host {host_s * 1e3:.1f} ms, layout equal {same}")
    first = rows["slice2048_100k"]
    result = {"metric": "neighbourhood construction time (device builder)", "value": first["device_ms"],
              "unit": "ms", "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": first["device_ms"],
              "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
              "data": "synthetic", "config": {"workload": "build", "graphs": list(rows)}, "graphs": rows,
              "roofline": None,
              "roofline_note": "a chain of short passes with host waits between them (level counts, sizes): "
                               "latency bound, not bandwidth bound",
              "cpu_baseline": None}
    print(json.dumps(result), flush=True)


def bench_serving(args, dev):
    """Continuous batching: requests (slices with 1k..1M regions, log-uniform,
    L in {2,3,4}, beta 0.5, 30 iterations) arrive as a Poisson process at 70 %
    of the capacity measured with all requests queued at time 0."""
    import numpy as np

    from paper_1809_05018_amd import pmrf, serve, synth

    rng = np.random.default_rng(5)
    pool_n = 24
    log(f"generating a pool of {pool_n} slices (regions log-uniform in [1k, 1M])")
    desc = synth.serving_requests(pool_n, 5)
    pool = [synth.image_graph(d["seed"], d["side"], d["regions"], 2) for d in desc]
    reqs_spec = [(int(rng.integers(0, pool_n)), int(rng.integers(2, 5))) for _ in range(args.requests)]

    def make(arrivals):
        return [serve.Request(rid=j, n=pool[k].n, row_ptr=pool[k].row_ptr, col_idx=pool[k].col_idx, y=pool[k].y,
                              L=L, beta=0.5, iters=30, arrival=float(a))
                for j, ((k, L), a) in enumerate(zip(reqs_spec, arrivals))]

    ex = serve.GpuExecutor(dev)
    budget = 64 << 30
    warm = serve.Server(ex, budget, iters_per_step=10)
    warm.run(make(np.zeros(min(8, args.requests))))
    closed = serve.Server(ex, budget, iters_per_step=10)
    cap = closed.run(make(np.zeros(args.requests)))
    lam = 0.7 * cap.throughput_rps
    log(f"capacity {cap.throughput_rps:.1f} req/s ({cap.evals_per_s:.3g} evals/s); arrivals at {lam:.1f} req/s")
    arr = synth.poisson_arrivals(args.requests, lam, 5)
    srv = serve.Server(ex, budget, iters_per_step=10)
    ls0 = pmrf.pmrf_launch_stats()
    st = srv.run(make(arr))
    ls1 = pmrf.pmrf_launch_stats()
    launches = {k: ls1[k] - ls0[k] for k in ls0}
    log(f"serving: p50 {st.p50_s:.3f} s, p99 {st.p99_s:.3f} s, {st.throughput_rps:.1f} req/s, {st.steps} steps, "
        f"launch modes {launches}")
    out = {"metric": "serving latency p50/p99 and throughput", "value": st.evals_per_s, "unit": "evals/s",
           "n_gpus": 1, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "serving", "requests": args.requests, "pool": pool_n,
                      "regions": "log-uniform 1k..1M", "labels": "uniform {2,3,4}", "beta": 0.5, "em_iters": 30,
                      "iters_per_step": 10, "arrival_rate_rps": lam, "hbm_budget_bytes": budget},
           "p50_s": st.p50_s, "p99_s": st.p99_s, "mean_s": st.mean_s, "throughput_rps": st.throughput_rps,
           "capacity_rps": cap.throughput_rps, "max_active": st.max_active, "steps": st.steps,
           "builder": "device", "build_s_mean": st.build_s_mean, "wall_s": st.wall_s,
           "launches": dict(launches, note="batched calls during the timed run: HIP graphs captured, replayed, and "
                                         "calls launched directly (an argument set seen once runs directly)")}
    # the same arrivals with the neighbourhoods built on the host
    hst = serve.Server(serve.GpuExecutor(dev, builder="host"), budget, iters_per_step=10).run(make(arr))
    log(f"host builder at the same rate: p50 {hst.p50_s:.3f} s, p99 {hst.p99_s:.3f} s, build {hst.build_s_mean:.3f} s")
    out["host_builder_same_arrivals"] = {"p50_s": hst.p50_s, "p99_s": hst.p99_s, "mean_s": hst.mean_s,
                                         "throughput_rps": hst.throughput_rps, "build_s_mean": hst.build_s_mean}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
