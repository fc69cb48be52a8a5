"""The serving loop's scheduling on the CPU, with an executor that runs the
oracle instead of the GPU and a virtual clock: admission by footprint,
retirement, latency bookkeeping, and results equal to one uninterrupted run."""
import numpy as np
import pytest

import oracle
from paper_1809_05018_amd import serve, synth


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class OracleExecutor:
    """Same methods as serve.GpuExecutor; each step costs 1 ms of virtual time.
    It keeps its own account of what it holds (each open request's buffers and
    a workspace sized for each step) and the peak of that account."""

    def __init__(self, clock):
        self.clock = clock
        self.live = 0
        self.ws = 0
        self.peak = 0

    def build(self, req):
        return oracle.OracleGraph(req.n, req.row_ptr, req.col_idx)

    def footprint(self, req, og):
        return 1000 + 40 * og.M + 16 * req.n

    def workspace_need(self, entries, k):
        # grows with the iterations of the step, like the library's history buffer
        return sum(300 + 24 * og.H + 4 * r.n + 8 * min(k, r.iters - r.done_iters) for r, og in entries)

    def open(self, req, og):
        x0 = serve.threshold_start(req.y, req.L)
        self.live += self.footprint(req, og)
        self.peak = max(self.peak, self.live + self.ws)
        return {"og": og, "x": x0, "mu": np.zeros(req.L), "sigma": np.ones(req.L), "first": True, "trace": [],
                "fp": self.footprint(req, og)}

    def step(self, active, k):
        self.clock.t += 1e-3
        self.ws = self.workspace_need([(r, s["og"]) for r, s in active], k)
        self.peak = max(self.peak, self.live + self.ws)
        out = []
        for req, slot in active:
            todo = min(k, req.iters - req.done_iters)
            r = slot["og"].em_run(req.y, req.L, req.beta, slot["x"], slot["mu"], slot["sigma"], todo,
                                  init_from_labels=slot["first"], early_exit=req.early_exit)
            slot.update(x=r["x"], mu=r["mu"], sigma=r["sigma"], first=False, S=r["S"])
            slot["trace"].extend(r["trace"].tolist())
            out.append(r["iters"])
        return out

    def close(self, req, slot):
        self.live -= slot["fp"]
        return {"x": slot["x"], "mu": slot["mu"], "sigma": slot["sigma"], "S": slot["S"],
                "trace": np.array(slot["trace"]), "evals": slot["og"].M * req.L * req.done_iters}


def make_requests(count=12, seed=9):
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(0.002, size=count))
    reqs = []
    for j in range(count):
        side = int(rng.integers(48, 160))
        g = synth.image_graph(700 + j, side, max(20, side * side // 30), 2)
        L = int(rng.integers(2, 5))
        reqs.append(serve.Request(rid=j, n=g.n, row_ptr=g.row_ptr, col_idx=g.col_idx, y=g.y, L=L, beta=0.5,
                                  iters=int(rng.integers(5, 16)), arrival=float(arrivals[j])))
    return reqs


@pytest.mark.parametrize("budget_scale,k", [(100.0, 4), (1.2, 3), (3.0, 7)])
def test_server_results_and_admission(budget_scale, k):
    clock = VirtualClock()
    ex = OracleExecutor(clock)
    reqs = make_requests()
    biggest = max(ex.footprint(r, og) + ex.workspace_need([(r, og)], k) for r in reqs for og in [ex.build(r)])
    srv = serve.Server(ex, hbm_budget=int(biggest * budget_scale), iters_per_step=k, clock=clock, sleep=clock.sleep)
    stats = srv.run(reqs)
    assert stats.requests == len(reqs) and stats.rejected == 0
    assert max(srv.footprint_log) <= srv.budget
    assert ex.peak <= srv.budget  # what the executor really held, workspace included
    if budget_scale < 2:
        assert stats.max_active < len(reqs)  # admission held requests back
        assert any(r.admitted > r.arrival for r in reqs)
    for r in reqs:
        og = oracle.OracleGraph(r.n, r.row_ptr, r.col_idx)
        x0 = serve.threshold_start(r.y, r.L)
        ref = og.em_run(r.y, r.L, r.beta, x0, np.zeros(r.L), np.ones(r.L), r.iters, init_from_labels=True)
        assert np.array_equal(r.result["x"], ref["x"])
        assert np.array_equal(r.result["mu"], ref["mu"]) and np.array_equal(r.result["sigma"], ref["sigma"])
        assert np.array_equal(r.result["trace"], ref["trace"]) and np.array_equal(r.result["S"], ref["S"])
        assert r.finished >= r.admitted >= r.arrival
    assert stats.p99_s >= stats.p50_s > 0


def test_request_above_budget_is_refused_alone():
    """A request that cannot fit even alone is refused on its own; every other
    request still completes, with the same result as an uninterrupted run."""
    clock = VirtualClock()
    ex = OracleExecutor(clock)
    reqs = make_requests(count=6)
    need = {r.rid: ex.footprint(r, og) + ex.workspace_need([(r, og)], 4) for r in reqs for og in [ex.build(r)]}
    big = max(need, key=need.get)
    budget = max(v for k, v in need.items() if k != big)
    assert need[big] > budget
    srv = serve.Server(ex, hbm_budget=budget, iters_per_step=4, clock=clock, sleep=clock.sleep)
    stats = srv.run(reqs)
    assert stats.rejected == 1 and stats.requests == len(reqs) - 1
    for r in reqs:
        if r.rid == big:
            assert r.result is None and "budget" in r.error
        else:
            assert r.error is None and r.done_iters == r.iters
            og = oracle.OracleGraph(r.n, r.row_ptr, r.col_idx)
            ref = og.em_run(r.y, r.L, r.beta, serve.threshold_start(r.y, r.L), np.zeros(r.L), np.ones(r.L),
                            r.iters, init_from_labels=True)
            assert np.array_equal(r.result["x"], ref["x"])
    assert ex.peak <= budget
    # nothing fits: every request is refused and the loop still ends
    srv = serve.Server(OracleExecutor(clock), hbm_budget=100, clock=clock, sleep=clock.sleep)
    stats = srv.run(make_requests(count=2))
    assert stats.requests == 0 and stats.rejected == 2


def schedule_reference(req, k):
    """The oracle run in the calls the server makes for an early-exit request:
    min(k, remaining) iterations per call until a call stops early."""
    og = oracle.OracleGraph(req.n, req.row_ptr, req.col_idx)
    x, mu, sigma = serve.threshold_start(req.y, req.L), np.zeros(req.L), np.ones(req.L)
    done, first, trace = 0, True, []
    while done < req.iters:
        todo = min(k, req.iters - done)
        r = og.em_run(req.y, req.L, req.beta, x, mu, sigma, todo, init_from_labels=first, early_exit=True)
        x, mu, sigma, first = r["x"], r["mu"], r["sigma"], False
        trace += r["trace"].tolist()
        done += r["iters"]
        if r["iters"] < todo:
            break
    return done, x, mu, sigma, np.array(trace)


def test_early_exit_requests_retire_when_converged():
    clock = VirtualClock()
    ex = OracleExecutor(clock)
    reqs = make_requests(count=8, seed=21)
    for r in reqs[::2]:  # beta = 0 converges within a few iterations
        r.beta, r.iters, r.early_exit = 0.0, 40, True
    srv = serve.Server(ex, hbm_budget=10**12, iters_per_step=6, clock=clock, sleep=clock.sleep)
    stats = srv.run(reqs)
    assert stats.requests == len(reqs)
    early = [r for r in reqs if r.early_exit]
    assert any(r.done_iters < r.iters for r in early)  # some stopped before their budget
    for r in early:
        done, x, mu, sigma, trace = schedule_reference(r, 6)
        assert r.done_iters == done
        assert np.array_equal(r.result["x"], x)
        assert np.array_equal(r.result["mu"], mu) and np.array_equal(r.result["sigma"], sigma)
        assert np.array_equal(r.result["trace"], trace)
    for r in reqs:
        if not r.early_exit:
            assert r.done_iters == r.iters
