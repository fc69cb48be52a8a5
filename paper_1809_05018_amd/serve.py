"""Continuous-batching request loop over pmrf_em_batch.

Requests (one slice each: region graph, intensities, L, beta, iterations)
arrive over time.  The loop keeps a set of active requests whose graph and
label state stay resident on the device, and advances all of them together,
``iters_per_step`` EM iterations per batched call.  Between steps it retires
finished requests (freeing their memory) and admits arrived ones while the
device footprint stays within ``hbm_budget`` bytes: the requests' own buffers
plus the exact workspace of the next batched call over the active set and the
candidate (``pmrf_em_batch_workspace_bytes``).  A request that could not fit
even alone is refused on its own (``Request.error``) and the others go on.
Neighbourhoods of arriving requests are built on host worker threads while the
device steps.  (The device builder's temporaries come from the library's own
memory pool, which keeps up to 1 GiB of freed blocks per device; that reserve
is outside ``hbm_budget``.)

Splitting a request's iterations over several batched calls gives the same
labels, parameters, energy trace and neighbourhood sums as one call with all
iterations (every step starts from the previous step's labels and parameters,
and batching does not change any result).  The convergence bookkeeping
(per-iteration non-converged counts, first converged iteration) restarts at
each call and is reported per step.

A request with ``early_exit`` stops as soon as every neighbourhood sum has
converged (the window test of the EM loop): the device stops iterating that
graph inside the batched call, the call reports fewer iterations than it was
given, and the loop retires the request at once, freeing its memory for
waiting requests.  Because the bookkeeping restarts at each call, the test can
fire from the (W+1)-th iteration of a call on (W = 3), so ``iters_per_step``
should be at least W + 1 for it to fire at all.

The executor does the device work; ``GpuExecutor`` drives the HIP library.  A
test executor with the same methods can stand in for it.
"""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import threading
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    y: np.ndarray
    L: int
    beta: float
    iters: int
    arrival: float = 0.0  # seconds after the start of the run
    x0: np.ndarray | None = None  # starting labels (default: threshold labelling)
    early_exit: bool = False  # stop (and retire) once the neighbourhood sums have converged
    # filled in by the server
    admitted: float | None = None
    finished: float | None = None
    build_s: float = 0.0
    done_iters: int = 0
    result: dict | None = None
    error: str | None = None  # set when the request was refused


def threshold_start(y, L):
    return np.minimum(L - 1, np.floor(np.asarray(y) * L / 256.0)).astype(np.int32)


class GpuExecutor:
    """Device side of the server: one pmrf.Problem per active request, one
    batch workspace sized exactly for each step."""

    def __init__(self, device="cuda", builder="device"):
        import torch

        from . import pmrf

        self.torch, self.pmrf = torch, pmrf
        self.device = torch.device(device)
        self.ws = None
        if builder not in ("device", "host"):
            raise ValueError("builder is 'device' or 'host'")
        self.builder = builder
        self._local = threading.local()

    def build(self, req: Request):
        """Neighbourhood construction (thread safe).  On the device each build
        thread has a stream of its own, so builds overlap the running steps."""
        pm, torch = self.pmrf, self.torch
        if self.builder == "host":
            return pm.pmrf_build_neighborhoods(req.n, req.row_ptr, req.col_idx)
        s = getattr(self._local, "stream", None)
        if s is None:
            s = self._local.stream = torch.cuda.Stream(self.device)
        with torch.cuda.stream(s):
            return pm.pmrf_build_neighborhoods_device(req.n, req.row_ptr, req.col_idx, stream=s)

    def open(self, req: Request, hoods):
        pm = self.pmrf
        prob = pm.Problem(req.n, req.row_ptr, req.col_idx, req.y, req.L, self.device, hoods=hoods)
        x0 = req.x0 if req.x0 is not None else threshold_start(req.y, req.L)
        prob.set_state(x0, np.zeros(req.L), np.ones(req.L))
        full = pm.pmrf_em_params(L=req.L, beta=req.beta, max_iters=req.iters)
        prob.prepare(full, workspace=False)  # trace and statistics buffers for the whole request
        prob.trace.zero_()
        prob.iter_stats.zero_()
        return {"prob": prob, "first": True, "hoods": hoods}

    def footprint(self, req: Request, hoods) -> int:
        """Exact device bytes of one request's own buffers while it is active
        (the batch workspace is counted separately, by ``workspace_need``)."""
        pm = self.pmrf
        n1, H1, T = max(1, req.n), max(1, hoods.H), max(1, req.iters)

        def t(nbytes):  # torch allocations are rounded to 512 bytes
            return (nbytes + 511) // 512 * 512

        return (t(max(256, hoods.device_bytes)) + t(8 * n1) + t(4 * n1) + 2 * t(8 * req.L) + t(8 * H1)
                + t(8 * pm.NCOUNTERS) + t(8 * T) + t(16 * T) + hoods.device_held()[1])

    def _params(self, req: Request, k: int, first: bool):
        todo = min(k, req.iters - req.done_iters)
        return self.pmrf.pmrf_em_params(L=req.L, beta=req.beta, max_iters=todo, init_from_labels=first,
                                        early_exit=req.early_exit)

    def workspace_need(self, entries: list, k: int) -> int:
        """Exact bytes of the workspace of the next batched call over
        ``entries`` = [(request, hoods)] (the library's own sizing)."""
        if not entries:
            return 0
        pm = self.pmrf
        items = [pm.EmItem(h.handle.value, 0, 0, 0, 0, 0, 0, 0, 0, 0, self._params(r, k, False)) for r, h in entries]
        return (pm.pmrf_em_batch_workspace_bytes(items) + 511) // 512 * 512

    def step(self, active: list, k: int):
        """Advance every active request by min(k, remaining) iterations in one
        batched call; returns the iterations done per request."""
        pm, torch = self.pmrf, self.torch
        items = []
        for req, slot in active:
            prob = slot["prob"]
            it = prob.item(self._params(req, k, slot["first"]))
            it.d_trace = prob.trace.data_ptr() + 8 * req.done_iters
            it.d_iter_stats = prob.iter_stats.data_ptr() + 16 * req.done_iters
            items.append(it)
            slot["first"] = False
        need = pm.pmrf_em_batch_workspace_bytes(items)
        if self.ws is None or self.ws.numel() != need:
            self.ws = None  # release before allocating: the footprint is the exact need
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        # the active set, its trace offsets and its starting flags change from
        # step to step, so a HIP graph of one step would rarely be replayed:
        # steps launch their kernels directly (launch mode 3)
        prev = pm.pmrf_get_launch()
        pm.pmrf_set_launch(**dict(prev, mode=3))
        try:
            pm.pmrf_em_batch(items, self.ws)
        finally:
            pm.pmrf_set_launch(**prev)
        # one copy back for every request's counters (it waits for the batch)
        c = torch.stack([slot["prob"].counters for _, slot in active]).cpu().numpy()
        out = []
        for (req, slot), row in zip(active, c):
            if row[pm.CTR_STATUS] != 0:
                raise pm.PmrfError(int(row[pm.CTR_STATUS]), f"request {req.rid}: device-reported error")
            out.append(int(row[pm.CTR_ITERS]))
        return out

    def close(self, req: Request, slot) -> dict:
        prob = slot["prob"]
        it = req.done_iters
        res = {"x": prob.labels[: req.n].cpu().numpy(), "mu": prob.mu.cpu().numpy(),
               "sigma": prob.sigma.cpu().numpy(), "S": prob.hood_energy[: prob.hoods.H].cpu().numpy(),
               "trace": prob.trace[:it].cpu().numpy(), "evals": prob.hoods.M * req.L * it}
        slot["prob"] = None
        return res

    def workspace_bytes(self) -> int:
        return 0 if self.ws is None else self.ws.numel()


@dataclasses.dataclass
class ServeStats:
    requests: int
    wall_s: float
    p50_s: float
    p99_s: float
    mean_s: float
    throughput_rps: float
    evals_per_s: float
    max_active: int
    max_footprint: int
    steps: int
    build_s_mean: float
    rejected: int = 0


class Server:
    def __init__(self, executor, hbm_budget: int, iters_per_step: int = 10, max_active: int = 256,
                 build_workers: int = 4, clock=time.perf_counter, sleep=time.sleep):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.k = int(iters_per_step)
        self.max_active = int(max_active)
        self.pool = cf.ThreadPoolExecutor(max_workers=build_workers)
        self.clock, self.sleep = clock, sleep
        self.footprint_log: list[int] = []

    def run(self, requests: list[Request]) -> ServeStats:
        pending = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock()
        now = lambda: self.clock() - t0
        builds: dict[int, cf.Future] = {}
        queue: list[Request] = []  # arrived, waiting for admission
        active: list[tuple[Request, dict, int]] = []  # (request, slot, own footprint)
        done: list[Request] = []
        self.rejected: list[Request] = []
        evals = 0
        steps = 0
        max_active = 0
        i = 0

        def build(req):
            b0 = time.perf_counter()
            h = self.ex.build(req)
            return h, time.perf_counter() - b0

        while len(done) + len(self.rejected) < len(pending):
            t = now()
            while i < len(pending) and pending[i].arrival <= t:
                req = pending[i]
                builds[req.rid] = self.pool.submit(build, req)
                queue.append(req)
                i += 1
            # admission, in arrival order, while the requests' own buffers and
            # the next call's workspace fit
            own = sum(fp for _, _, fp in active)
            entries = [(r, s["hoods"]) for r, s, _ in active]
            still = []
            for req in queue:
                fut = builds[req.rid]
                if not fut.done() or len(active) >= self.max_active:
                    still.append(req)
                    continue
                hoods, req.build_s = fut.result()
                fp = self.ex.footprint(req, hoods)
                if fp + self.ex.workspace_need([(req, hoods)], self.k) > self.budget:
                    req.error = f"request {req.rid} needs more than the budget of {self.budget} bytes alone"
                    req.finished = now()
                    self.rejected.append(req)
                    del builds[req.rid]
                    continue
                if own + fp + self.ex.workspace_need(entries + [(req, hoods)], self.k) > self.budget:
                    still.append(req)
                    continue
                slot = self.ex.open(req, hoods)
                slot.setdefault("hoods", hoods)
                req.admitted = now()
                active.append((req, slot, fp))
                entries.append((req, hoods))
                own += fp
                del builds[req.rid]
            queue = still
            max_active = max(max_active, len(active))
            if not active:
                # idle: wait for the next arrival or build
                if queue:
                    next(iter(cf.as_completed([builds[r.rid] for r in queue])))
                elif i < len(pending):
                    self.sleep(max(0.0, pending[i].arrival - now()))
                continue
            self.footprint_log.append(own + self.ex.workspace_need(entries, self.k))
            did = self.ex.step([(r, s) for r, s, _ in active], self.k)
            steps += 1
            keep = []
            for (req, slot, fp), d in zip(active, did):
                req.done_iters += d
                if req.done_iters >= req.iters or d < min(self.k, req.iters - (req.done_iters - d)):
                    req.result = self.ex.close(req, slot)
                    req.finished = now()
                    evals += req.result["evals"]
                    done.append(req)
                else:
                    keep.append((req, slot, fp))
            active = keep
        wall = now()
        lat = np.array([r.finished - r.arrival for r in done]) if done else np.zeros(1)
        return ServeStats(requests=len(done), wall_s=wall, p50_s=float(np.percentile(lat, 50)),
                          p99_s=float(np.percentile(lat, 99)), mean_s=float(lat.mean()),
                          throughput_rps=len(done) / wall if wall > 0 else 0.0, evals_per_s=evals / wall if wall > 0 else 0.0,
                          max_active=max_active,
                          max_footprint=max(self.footprint_log) if self.footprint_log else 0, steps=steps,
                          build_s_mean=float(np.mean([r.build_s for r in done])) if done else 0.0,
                          rejected=len(self.rejected))
