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
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_iter_slice2048_100k_counters.json")
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


def measured_traffic(per_launch_units: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source; else None."""
    try:
        d = json.load(open(COUNTERS_FILE))
    except (OSError, ValueError):
        return None
    if d.get("kernel_sha") != kernel_sha():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(g, L, beta, iters, x0, M):
    import numpy as np

    import oracle

    og = oracle.OracleGraph(g.n, g.row_ptr, g.col_idx)
    t0 = time.perf_counter()
    ref = og.em_run(g.y, L, beta, x0, np.zeros(L), np.ones(L), iters, init_from_labels=True)
    dt = time.perf_counter() - t0
    return ref, {"value": M * L * iters / dt, "unit": "evals/s", "cores": 1, "kind": "oracle",
                 "sample": f"full workload, {iters} EM iterations, serial C oracle (-O2), EM loop only, {dt:.2f} s",
                 "seconds": round(dt, 3), "cpu": platform.processor() or platform.machine()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--iters", type=int, default=30, help="EM iterations per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the EM path of one graph runs on one device and this build "
              "has no multi-GPU path (see DESIGN.md for how it would shard). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1809_05018_amd import pmrf, synth

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    L, beta, iters = 2, 0.5, args.iters
    log("generating the 2048x2048 / 100k-region slice")
    g = synth.workload_large()
    x0 = synth.threshold_labels(g.y, L)
    prob = pmrf.Problem(g.n, g.row_ptr, g.col_idx, g.y, L, dev)
    info = prob.hoods.info
    log(f"n={info.n} H={info.H} M={info.M} A={info.A} max_hood={info.max_hood} tiles={info.tiles}")

    # starting parameters: the parameter update of the threshold labels, on the device
    prob.set_state(x0, np.zeros(L), np.ones(L))
    prob.run(pmrf.pmrf_em_params(L=L, beta=beta, max_iters=0, init_from_labels=True))
    torch.cuda.synchronize()
    x0_dev = prob.labels.clone()
    mu0, s0 = prob.mu.clone(), prob.sigma.clone()
    params = pmrf.pmrf_em_params(L=L, beta=beta, max_iters=iters)
    prob.prepare(params)

    def step():
        prob.labels.copy_(x0_dev)
        prob.mu.copy_(mu0)
        prob.sigma.copy_(s0)
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
                   "mode": "HIP graph of two kernels per EM iteration"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("bytes"),
                     "kernel": "k_iter<2>", "alg_bytes_per_launch": b_launch,
                     "avg_launch_us": avg_launch_s * 1e6, "launches_timed": launches,
                     "timing": "HIP events around each EM-iteration launch, second timed region of the same steps"},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        log("timing the serial oracle on the same workload")
        ref, cpu = cpu_baseline(g, L, beta, iters, x0, info.M)
        result["cpu_baseline"] = cpu
        labels_equal = bool(np.array_equal(out["x"], ref["x"]))
        rel = lambda a, b: float(np.max(np.abs(np.asarray(a) - np.asarray(b)) / np.abs(np.asarray(b))))
        result["parity"] = {"labels_bit_exact": labels_equal, "near_ties": ref["total_near_ties"],
                            "mu_rel": rel(out["mu"], ref["mu"]), "sigma_rel": rel(out["sigma"], ref["sigma"]),
                            "trace_rel": rel(out["trace"], ref["trace"])}
        result["speedup_vs_oracle"] = value / cpu["value"]
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
