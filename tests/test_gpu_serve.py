"""Serving on the GPU: requests arriving while others run are batched together;
each result equals the same request run alone (needs the GPU)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1809_05018_amd import pmrf, serve, synth
from tests.gpu_helpers import compare_runs

pytestmark = pytest.mark.gpu


def test_serving_mix_equals_solo():
    rng = np.random.default_rng(17)
    count = 16
    arrivals = np.cumsum(rng.exponential(0.003, size=count))
    reqs = []
    for j in range(count):
        regions = int(np.exp(rng.uniform(np.log(300), np.log(20000))))
        side = int(round(np.sqrt(26.2 * regions)))
        g = synth.image_graph(800 + j, side, regions, 2)
        reqs.append(serve.Request(rid=j, n=g.n, row_ptr=g.row_ptr, col_idx=g.col_idx, y=g.y,
                                  L=int(rng.integers(2, 5)), beta=0.5, iters=30, arrival=float(arrivals[j])))
    ex = serve.GpuExecutor("cuda")
    sizes = [ex.footprint(r, ex.build(r)) for r in reqs]
    srv = serve.Server(ex, hbm_budget=int(sum(sizes) * 0.5), iters_per_step=10)
    before = pmrf.pmrf_launch_stats()
    stats = srv.run(reqs)
    after = pmrf.pmrf_launch_stats()
    assert after["captures"] == before["captures"] and after["replays"] == before["replays"]  # no graph per step
    assert after["direct"] - before["direct"] == stats.steps
    assert stats.requests == count and max(srv.footprint_log) <= srv.budget
    assert stats.max_active > 1  # work really overlapped
    for r in reqs:
        solo = pmrf.solve(r.n, r.row_ptr, r.col_idx, r.y, serve.threshold_start(r.y, r.L), np.zeros(r.L),
                          np.ones(r.L), pmrf.pmrf_em_params(L=r.L, beta=r.beta, max_iters=r.iters,
                                                            init_from_labels=True))
        for k in ("x", "mu", "sigma", "S", "trace"):
            assert np.array_equal(np.asarray(r.result[k]), np.asarray(solo[k])), (r.rid, k)
    # the served results against the oracle: the smallest requests whose
    # oracle run has no near tie (so every label is decided), all their
    # iterations from the same start
    compared = 0
    for r in sorted(reqs, key=lambda q: q.n):
        og = oracle.OracleGraph(r.n, r.row_ptr, r.col_idx)
        ref = og.em_run(r.y, r.L, r.beta, serve.threshold_start(r.y, r.L), np.zeros(r.L), np.ones(r.L), r.iters,
                        init_from_labels=True)
        if ref["total_near_ties"]:
            continue
        got = dict(r.result, status=0, iters=r.done_iters)
        # the per-call bookkeeping restarts in each batched call, so only the
        # quantities of the whole run are compared
        for key in ("near_ties", "nonconv", "map_conv_iter", "em_conv_iter", "total_near_ties"):
            got[key] = ref[key]
        compare_runs(got, ref, f"served request {r.rid} (n={r.n}, L={r.L})")
        compared += 1
        if compared == 3:
            break
    assert compared == 3


def solo_schedule(r, k):
    """The request run alone in the calls the server makes: min(k, remaining)
    iterations per call, early exit on, until a call stops early."""
    prob = pmrf.Problem(r.n, r.row_ptr, r.col_idx, r.y, r.L)
    prob.set_state(serve.threshold_start(r.y, r.L), np.zeros(r.L), np.ones(r.L))
    done, first, trace = 0, True, []
    while done < r.iters:
        todo = min(k, r.iters - done)
        params = pmrf.pmrf_em_params(L=r.L, beta=r.beta, max_iters=todo, init_from_labels=first, early_exit=True)
        prob.run(params)
        out = prob.results(params)
        assert out["status"] == 0
        trace += out["trace"][: out["iters"]].tolist()
        done += out["iters"]
        first = False
        if out["iters"] < todo:
            break
    return done, out, np.array(trace)


def test_serving_early_exit_retires_converged_requests():
    rng = np.random.default_rng(23)
    reqs = []
    for j in range(10):
        regions = int(np.exp(rng.uniform(np.log(300), np.log(8000))))
        side = int(round(np.sqrt(26.2 * regions)))
        g = synth.image_graph(900 + j, side, regions, 2)
        early = j % 2 == 0
        reqs.append(serve.Request(rid=j, n=g.n, row_ptr=g.row_ptr, col_idx=g.col_idx, y=g.y, L=2,
                                  beta=0.0 if early else 0.5, iters=40 if early else 12,
                                  arrival=0.002 * j, early_exit=early))
    srv = serve.Server(serve.GpuExecutor("cuda"), hbm_budget=1 << 34, iters_per_step=6)
    stats = srv.run(reqs)
    assert stats.requests == len(reqs)
    early = [r for r in reqs if r.early_exit]
    assert any(r.done_iters < r.iters for r in early)
    for r in early:
        done, out, trace = solo_schedule(r, 6)
        assert r.done_iters == done, (r.rid, r.done_iters, done)
        for key in ("x", "mu", "sigma"):
            assert np.array_equal(np.asarray(r.result[key]), np.asarray(out[key])), (r.rid, key)
        assert np.array_equal(np.asarray(r.result["trace"]), trace), r.rid
    assert all(r.done_iters == r.iters for r in reqs if not r.early_exit)
