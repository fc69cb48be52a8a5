"""HIP path against the oracle, through the C ABI (needs the GPU)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1809_05018_amd import pmrf, synth
from tests import pins
from tests.gpu_helpers import (TIE, assert_close, compare_runs, end_to_end, gpu_run, init_state, lockstep,
                               vertex_energies)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def device():
    assert torch.cuda.is_available(), "gpu tests need a HIP device"
    return "cuda"


def test_lockstep_small():
    g = synth.workload_small()
    lockstep(g, 2, 0.5, 20, "slice256_1k")


def test_lockstep_multilabel_powerlaw():
    g = synth.powerlaw_graph(4242, 6000, phases=4, dmax=45)
    lockstep(g, 4, 0.8, 6, "powerlaw6k_L4")


def test_end_to_end_small():
    end_to_end(synth.workload_small(), 2, 0.5, 20, "slice256_1k")


def test_end_to_end_large():
    gpu, ref = end_to_end(synth.workload_large(), 2, 0.5, 30, "slice2048_100k")
    assert gpu["evals"] == 30 * 2 * pmrf.pmrf_build_neighborhoods(
        synth.workload_large().n, synth.workload_large().row_ptr, synth.workload_large().col_idx).M


def test_end_to_end_three_phase():
    end_to_end(synth.image_graph(77, 512, 5000, 3), 3, 0.5, 15, "slice512_5k_L3")


def test_end_to_end_large_hoods():
    # degrees up to 80 give neighbourhoods above 64 members (multi-chunk packets)
    g = synth.powerlaw_graph(99, 20000, phases=4, dmax=80, exponent=2.0)
    h = pmrf.pmrf_build_neighborhoods(g.n, g.row_ptr, g.col_idx)
    assert h.max_hood > 64
    end_to_end(g, 4, 0.8, 8, "powerlaw20k_dmax80")


@pytest.mark.parametrize("L", [5, 8, 16])
def test_end_to_end_many_labels(L):
    g = synth.image_graph(31 + L, 256, 1500, 4)
    end_to_end(g, L, 0.3, 6, f"slice256_L{L}")


def test_beta_zero_and_early_exit():
    g = synth.workload_small()
    end_to_end(g, 2, 0.0, 20, "beta0")
    gpu, ref = end_to_end(g, 2, 0.0, 20, "beta0_early", early_exit=True)
    assert ref["iters"] < 20


def test_init_from_labels():
    g = synth.workload_small()
    x0 = synth.threshold_labels(g.y, 2)
    og = oracle.OracleGraph(g.n, g.row_ptr, g.col_idx)
    ref = og.em_run(g.y, 2, 0.5, x0, [1.0, 2.0], [3.0, 4.0], 5, init_from_labels=True)
    prob = pmrf.Problem(g.n, g.row_ptr, g.col_idx, g.y, 2)
    gpu = gpu_run(prob, x0, [1.0, 2.0], [3.0, 4.0], beta=0.5, max_iters=5, init_from_labels=True)
    compare_runs(gpu, ref, "init_from_labels")
    # zero iterations: only the starting update runs
    ref0 = og.em_run(g.y, 2, 0.5, x0, [1.0, 2.0], [3.0, 4.0], 0, init_from_labels=True)
    gpu0 = gpu_run(prob, x0, [1.0, 2.0], [3.0, 4.0], beta=0.5, max_iters=0, init_from_labels=True)
    assert gpu0["iters"] == 0 and np.array_equal(gpu0["x"], x0)
    assert_close(gpu0["mu"], ref0["mu"], "init mu")
    assert_close(gpu0["sigma"], ref0["sigma"], "init sigma")


@pytest.mark.parametrize("case", ["single", "isolated", "clique40", "star101", "path", "empty"])
def test_edge_graphs(case):
    rng = np.random.default_rng(5)
    if case == "single":
        n, (rp, ci) = 1, pins.csr(1, [])
    elif case == "isolated":
        n, (rp, ci) = 7, pins.csr(7, [])
    elif case == "clique40":
        n, (rp, ci) = 40, pins.csr(40, [(a, b) for a in range(40) for b in range(a + 1, 40)])
    elif case == "star101":
        n, (rp, ci) = 101, pins.csr(101, [(0, i) for i in range(1, 101)])
    elif case == "path":
        n, (rp, ci) = 300, pins.csr(300, [(i, i + 1) for i in range(299)])
    else:
        n, (rp, ci) = 0, (np.zeros(1, np.int32), np.zeros(0, np.int32))
    y = rng.uniform(0, 255, n)
    g = synth.GraphInput(n=n, row_ptr=rp, col_idx=ci, y=y, name=case)
    if n == 0:
        prob = pmrf.Problem(0, rp, ci, y, 2)
        out = gpu_run(prob, np.zeros(0, np.int32), [50.0, 150.0], [20.0, 20.0], beta=0.5, max_iters=3)
        assert out["status"] == 0 and out["iters"] == 3 and out["trace"].tolist() == [0.0, 0.0, 0.0]
        return
    end_to_end(g, 2, 0.7, 6, case)


def test_device_reported_errors():
    g = synth.workload_small()
    prob = pmrf.Problem(g.n, g.row_ptr, g.col_idx, g.y, 2)
    x = synth.threshold_labels(g.y, 2)
    x[17] = 2
    out = gpu_run(prob, x, [80.0, 170.0], [20.0, 20.0], max_iters=3)
    assert out["status"] == pmrf.PMRF_EBADLABEL and out["iters"] == 0
    x[17] = 0
    out = gpu_run(prob, x, [80.0, 170.0], [20.0, 0.0], max_iters=3)
    assert out["status"] == pmrf.PMRF_EBADPARAM
    out = gpu_run(prob, x, [80.0, 170.0], [20.0, 20.0], max_iters=3)  # the same buffers recover
    assert out["status"] == 0 and out["iters"] == 3


def test_determinism_and_launch_shape_invariance():
    g = synth.image_graph(8, 1024, 25000, 2)
    x0, mu0, s0 = init_state(g, 2)
    prob = pmrf.Problem(g.n, g.row_ptr, g.col_idx, g.y, 2)
    old = pmrf.pmrf_get_launch()
    outs = []
    try:
        for shape in [(3, 0, 0, 0), (1, 0, 0, 0), (1, 1, 0, 0), (3, 16, 0, 0), (2, 8, 0, 1), (2, 4, 0, 3),
                      (3, 2, 0, 0)]:
            pmrf.pmrf_set_launch(*shape)
            outs.append(gpu_run(prob, x0, mu0, s0, beta=0.5, max_iters=12))
    finally:
        pmrf.pmrf_set_launch(**old)
    for o in outs[1:]:
        for k in ("x", "mu", "sigma", "S", "trace", "near_ties", "nonconv"):
            assert np.array_equal(o[k], outs[0][k]), k


def test_resume_equals_uninterrupted():
    g = synth.workload_small()
    x0, mu0, s0 = init_state(g, 2)
    prob = pmrf.Problem(g.n, g.row_ptr, g.col_idx, g.y, 2)
    full = gpu_run(prob, x0, mu0, s0, beta=0.5, max_iters=30)
    a = gpu_run(prob, x0, mu0, s0, beta=0.5, max_iters=15)
    b = gpu_run(prob, a["x"], a["mu"], a["sigma"], beta=0.5, max_iters=15)
    assert np.array_equal(b["x"], full["x"])
    assert np.array_equal(b["mu"], full["mu"]) and np.array_equal(b["sigma"], full["sigma"])
    assert np.array_equal(np.concatenate([a["trace"], b["trace"]]), full["trace"])
    assert np.array_equal(b["S"], full["S"])


def test_graph_replays_match_direct_launches():
    """The cached HIP graph, replayed several times with eager device work and
    synchronisation between replays, gives the direct-launch result every time."""
    g = synth.image_graph(21, 512, 6000, 2)
    x0, mu0, s0 = init_state(g, 2)
    prob = pmrf.Problem(g.n, g.row_ptr, g.col_idx, g.y, 2)
    old = pmrf.pmrf_get_launch()
    try:
        pmrf.pmrf_set_launch(3, 0, 0, 0)
        eager = gpu_run(prob, x0, mu0, s0, beta=0.5, max_iters=10)
        pmrf.pmrf_set_launch(1, 0, 0, 0)
        for rep in range(4):
            scratch = torch.randn(1 << 20, device="cuda", dtype=torch.float64)  # eager work between replays
            scratch.mul_(2.0).sum().item()
            out = gpu_run(prob, x0, mu0, s0, beta=0.5, max_iters=10)
            for k in ("x", "mu", "sigma", "S", "trace", "near_ties", "nonconv"):
                assert np.array_equal(out[k], eager[k]), (rep, k)
    finally:
        pmrf.pmrf_set_launch(**old)


@pytest.mark.parametrize("W", [1, 6])
def test_convergence_window_lengths(W):
    # W = 6 exceeds the slot path's prefetched window, so every superchunk of
    # the graph takes the packet kernel; W = 1 is the shortest window
    g = synth.workload_small()
    x0, mu0, s0 = init_state(g, 2)
    og = oracle.OracleGraph(g.n, g.row_ptr, g.col_idx)
    ref = og.em_run(g.y, 2, 0.5, x0, mu0, s0, 12, window=W)
    prob = pmrf.Problem(g.n, g.row_ptr, g.col_idx, g.y, 2)
    gpu = gpu_run(prob, x0, mu0, s0, beta=0.5, max_iters=12, conv_window=W)
    compare_runs(gpu, ref, f"window{W}")


def test_profile_events_time_each_iteration():
    """Profiling mode stamps one event pair per EM iteration (around the slot
    kernel, or the slot and packet kernels together) and changes no result;
    an empty graph still runs one (empty) block per iteration, which is timed."""
    cases = [(synth.workload_small(), 2, 9),
             (synth.powerlaw_graph(99, 20000, phases=4, dmax=80, exponent=2.0), 4, 5)]
    for g, L, iters in cases:
        x0, mu0, s0 = init_state(g, L)
        prob = pmrf.Problem(g.n, g.row_ptr, g.col_idx, g.y, L)
        plain = gpu_run(prob, x0, mu0, s0, beta=0.5, max_iters=iters)
        pmrf.pmrf_profile_begin()
        timed = gpu_run(prob, x0, mu0, s0, beta=0.5, max_iters=iters)
        ms, launches = pmrf.pmrf_profile_end()
        assert launches == iters and ms > 0.0, (g.name, launches, ms)
        for k in ("x", "mu", "sigma", "S", "trace", "near_ties", "nonconv"):
            assert np.array_equal(timed[k], plain[k]), (g.name, k)
    rp, ci = np.zeros(1, np.int32), np.zeros(0, np.int32)
    prob = pmrf.Problem(0, rp, ci, np.zeros(0), 2)
    pmrf.pmrf_profile_begin()
    gpu_run(prob, np.zeros(0, np.int32), [50.0, 150.0], [20.0, 20.0], beta=0.5, max_iters=3)
    ms, launches = pmrf.pmrf_profile_end()
    assert launches == 3 and ms > 0.0


# ------------------------------------------------------------------ ties
def one_step_both(g, L, beta, x, mu, sigma):
    og = oracle.OracleGraph(g.n, g.row_ptr, g.col_idx)
    ref = og.em_step(g.y, L, beta, x, mu, sigma, per_element=True)
    prob = pmrf.Problem(g.n, g.row_ptr, g.col_idx, g.y, L)
    gpu = gpu_run(prob, x, mu, sigma, beta=beta, max_iters=1)
    assert gpu["status"] == 0
    return og, ref, gpu


def test_exact_tie_takes_the_lowest_label():
    """y halfway between two means with equal sigma: both energies are exactly
    12.5 on both sides, so both take label 0 and count two near ties; the
    Potts count breaks the same tie towards the neighbours' label."""
    rp, ci = pins.csr(2, [(0, 1)])
    g = synth.GraphInput(n=2, row_ptr=rp, col_idx=ci, y=np.array([5.0, 5.0]), name="edge_tie")
    for beta, x, want, ties in ((0.0, [1, 1], [0, 0], 2), (0.5, [1, 1], [1, 1], 0), (0.5, [0, 1], [1, 0], 0)):
        _, ref, gpu = one_step_both(g, 2, beta, np.array(x, np.int32), [0.0, 10.0], [1.0, 1.0])
        assert list(ref["x"]) == want and ref["near_ties"] == ties
        assert list(gpu["x"]) == want and gpu["near_ties"][0] == ties, (beta, x, gpu["x"], gpu["near_ties"])
        assert gpu["trace"][0] == ref["T"]


def test_exact_ties_general_labels():
    """Four labels, the tie between labels 1 and 3 only (general-L kernel):
    lowest tied label on both sides, on a grid where a third of the vertices
    sit exactly on the tie."""
    side = 24
    edges = [(r * side + c, r * side + c + 1) for r in range(side) for c in range(side - 1)]
    edges += [(r * side + c, (r + 1) * side + c) for r in range(side - 1) for c in range(side)]
    rp, ci = pins.csr(side * side, edges)
    rng = np.random.default_rng(41)
    y = rng.uniform(0, 255, side * side)
    y[::3] = 5.0
    g = synth.GraphInput(n=side * side, row_ptr=rp, col_idx=ci, y=y, name="grid_tie_L4")
    mu, sigma = [100.0, 0.0, 50.0, 10.0], [1.0, 1.0, 1.0, 1.0]
    x = rng.integers(0, 4, g.n).astype(np.int32)
    _, ref, gpu = one_step_both(g, 4, 0.0, x, mu, sigma)
    assert np.all(ref["x"][::3] == 1) and ref["near_ties"] >= g.n // 3
    assert np.array_equal(gpu["x"], ref["x"]) and gpu["near_ties"][0] == ref["near_ties"]
    assert_close(gpu["S"], ref["S"], "S_h")


@pytest.mark.parametrize("beta", [0.0, 0.5])
def test_constructed_near_ties(beta):
    """Intensities a few units in the last place from the midpoint of two
    means: gaps of 1e-14 or less, which the two sides may round either way.
    Near-tie counts must agree, labels must agree at every vertex with a clear
    gap, and at a near tie the device's label must be a minimiser within 1e-9."""
    rng = np.random.default_rng(43)
    gi = synth.image_graph(44, 256, 1000, 2)
    y = gi.y.copy()
    tied = rng.random(gi.n) < 0.3
    y[tied] = 125.0 + rng.integers(-4, 5, tied.sum()) * 2.0 ** -45
    g = synth.GraphInput(n=gi.n, row_ptr=gi.row_ptr, col_idx=gi.col_idx, y=y, name="near_ties")
    mu, sigma = [80.0, 170.0], [25.0, 25.0]
    x = synth.threshold_labels(y, 2)
    og, ref, gpu = one_step_both(g, 2, beta, x, mu, sigma)
    gaps = ref["gap"][og.owner()]
    clear = gaps >= TIE
    assert beta > 0 or (~clear).sum() > 0
    assert gpu["near_ties"][0] == ref["near_ties"] == int((~clear).sum())
    assert np.array_equal(gpu["x"][clear], ref["x"][clear])
    idx = np.flatnonzero(~clear)
    E = vertex_energies(og, g, 2, beta, x, mu, sigma, idx)
    assert np.all(E[np.arange(idx.size), gpu["x"][idx]] - E.min(axis=1) < TIE)
    assert_close(gpu["S"], ref["S"], "S_h")
    # and over several iterations (the near-tie protocol of end_to_end)
    end_to_end(g, 2, beta, 8, f"near_ties_beta{beta}", start=(x, np.array(mu), np.array(sigma)))


# ------------------------------------------------------- random starting state
@pytest.mark.parametrize("which,L", [("slice256_1k", 2), ("slice256_1k", 4), ("slice2048_100k", 2),
                                     ("slice2048_100k", 4)])
def test_random_start(which, L):
    """The paper's initialisation: random labels, mu and sigma drawn uniformly
    from [0, 255] (sigma from [1, 255] so that it is positive)."""
    g = synth.workload_small() if which == "slice256_1k" else synth.workload_large()
    x0, mu0, s0 = synth.random_init(900 + L, g.n, L)
    end_to_end(g, L, 0.5, 20 if which == "slice256_1k" else 30, f"{which}_random_L{L}", start=(x0, mu0, s0))
