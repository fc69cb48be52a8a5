"""Checks that pin the oracle to facts outside itself.

Each ``check_*`` raises ``AssertionError`` on a mismatch.  They take the oracle
library handle, so the planted-mistake test can run the same checks against
deliberately broken builds of the oracle and show that each mistake is caught.

What pins what:
  worked example (golden, Sec. 3.2.2)     replication layout and the gathers
  brute force over all vertex subsets     maximal cliques, canonical order
  closed forms on K_n, paths, stars,      neighbourhoods = clique + 1-ring
  cycles, empty graphs
  reachability by adjacency-matrix        k-neighbourhoods (k = 2, 3) and their
  powers, paths and stars at k = 2        in-neighbourhood adjacency
  serial Scatter simulation, argmin over  the scatter rules of the label update
  occurrences, a hand-worked path, beta=0 (owner, last neighbourhood, minimum)
  adjacency-matrix recomputation          in-hood adjacency, owner rule
  scipy.stats.norm.logpdf                 the Gaussian data term
  per-vertex synchronous ICM on the CSR   label update through neighbourhoods
  exhaustive labellings (n <= 8)          argmin, Potts count, tie rule
  numpy mean / std(ddof=0)                parameter update
  classification EM on y (beta = 0)       the whole loop without smoothness
  constructed sequences                   convergence test
"""
from __future__ import annotations

import itertools
import math
import os

import numpy as np
from scipy.stats import norm

import oracle
from paper_1809_05018_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
HALF_LOG_2PI = 0.5 * math.log(2.0 * math.pi)


def read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split("=", 1)
            out[k.strip()] = np.array([float(t) for t in v.split()])
    return out


# --------------------------------------------------------------- graphs

def adj_matrix(n, rp, ci):
    A = np.zeros((n, n), dtype=bool)
    for v in range(n):
        A[v, ci[rp[v]:rp[v + 1]]] = True
    return A


def csr(n, edges):
    e = np.array(edges, dtype=np.int64).reshape(-1, 2)
    return synth.csr_from_edges(n, e[:, 0], e[:, 1])


def brute_cliques(n, rp, ci):
    A = adj_matrix(n, rp, ci)
    out = []
    for mask in range(1, 1 << n):
        S = [v for v in range(n) if (mask >> v) & 1]
        if not all(A[a, b] for a, b in itertools.combinations(S, 2)):
            continue
        if any(all(A[u, s] for s in S) for u in range(n) if not (mask >> u) & 1):
            continue
        out.append(tuple(S))
    return sorted(out)


def oracle_lists(og):
    cp, cv = og.cliques()
    hp, hv = og.hoods()
    cl = [tuple(int(t) for t in cv[cp[h]:cp[h + 1]]) for h in range(og.H)]
    hl = [tuple(int(t) for t in hv[hp[h]:hp[h + 1]]) for h in range(og.H)]
    return cl, hl


def random_small_graphs(count=60, nmax=8):
    for s in range(count):
        n = 1 + s % nmax
        p = (0.2, 0.5, 0.8)[s % 3]
        rp, ci = synth.small_random_graph(100 + s, n, p)
        yield n, rp, ci


def data_energy(y, mu, sigma):
    """Gaussian negative log density without the 1/2 ln(2 pi) constant, via scipy."""
    return -norm.logpdf(np.asarray(y)[:, None], np.asarray(mu)[None, :], np.asarray(sigma)[None, :]) - HALF_LOG_2PI


# --------------------------------------------------------------- checks

def check_worked_example(lib):
    g = read_golden("replicate_worked_example.txt")
    hp = g["hood_ptr"].astype(np.int64)
    L = int(g["L"][0])
    tl, oi, hi = oracle.replicate(hp, L, lib=lib)
    assert np.array_equal(tl, g["testLabel"].astype(int)), tl
    assert np.array_equal(oi, g["oldIndex"].astype(int)), oi
    assert np.array_equal(hi, g["hoodId"].astype(int)), hi
    vl, vm = oracle.gather(oi, g["hoods"].astype(int), g["x"].astype(int), g["y"], lib=lib)
    assert np.array_equal(vl, g["vertLabel"].astype(int)), vl
    assert np.array_equal(vm, g["vertMu"]), vm


def check_cliques_bruteforce(lib):
    for n, rp, ci in random_small_graphs():
        og = oracle.OracleGraph(n, rp, ci, lib=lib)
        cl, _ = oracle_lists(og)
        assert cl == brute_cliques(n, rp, ci), (n, cl)


def check_closed_forms(lib):
    cases = []
    for n in range(1, 8):  # complete graph: one clique, one neighbourhood = V
        rp, ci = csr(n, list(itertools.combinations(range(n), 2)))
        cases.append((n, rp, ci, [tuple(range(n))], [tuple(range(n))]))
    for n in range(2, 9):  # path: cliques are edges, hood = {i-1 .. i+2}
        rp, ci = csr(n, [(i, i + 1) for i in range(n - 1)])
        cl = [(i, i + 1) for i in range(n - 1)]
        hl = [tuple(range(max(0, i - 1), min(n - 1, i + 2) + 1)) for i in range(n - 1)]
        cases.append((n, rp, ci, cl, hl))
    for k in range(1, 7):  # star: cliques are spokes, every hood = V
        rp, ci = csr(k + 1, [(0, i) for i in range(1, k + 1)])
        cases.append((k + 1, rp, ci, [(0, i) for i in range(1, k + 1)], [tuple(range(k + 1))] * k))
    for n in range(4, 9):  # cycle: cliques are edges, hood = {i-1, i, i+1, i+2} mod n
        edges = [(i, (i + 1) % n) for i in range(n)]
        rp, ci = csr(n, edges)
        cl = sorted(tuple(sorted(e)) for e in edges)
        hl = [tuple(sorted({(c[0] - 1) % n, c[0], c[1], (c[1] + 1) % n} if c != (0, n - 1)
                           else {n - 2, n - 1, 0, 1})) for c in cl]
        cases.append((n, rp, ci, cl, hl))
    for n in range(1, 6):  # no edges: singletons
        rp, ci = csr(n, [])
        cases.append((n, rp, ci, [(v,) for v in range(n)], [(v,) for v in range(n)]))
    rp, ci = csr(6, [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5)])  # two triangles
    cases.append((6, rp, ci, [(0, 1, 2), (3, 4, 5)], [(0, 1, 2), (3, 4, 5)]))
    for n, rp, ci, cl_want, hl_want in cases:
        og = oracle.OracleGraph(n, rp, ci, lib=lib)
        cl, hl = oracle_lists(og)
        assert cl == cl_want, (n, cl, cl_want)
        assert hl == hl_want, (n, hl, hl_want)


def check_hoods_adjacency_owner(lib):
    graphs = list(random_small_graphs())
    g1 = synth.workload_small()
    graphs.append((g1.n, g1.row_ptr, g1.col_idx))
    for n, rp, ci in graphs:
        og = oracle.OracleGraph(n, rp, ci, lib=lib)
        cl, hl = oracle_lists(og)
        hp, hv = og.hoods()
        ap, aloc = og.adjacency()
        owner = og.owner()
        nbrs = [set(ci[rp[v]:rp[v + 1]].tolist()) for v in range(n)]
        for h, (c, hood) in enumerate(zip(cl, hl)):
            want = set(c)
            for v in c:
                want |= nbrs[v]
            assert hood == tuple(sorted(want)), (h, hood)
            for j, v in enumerate(hood):
                e = hp[h] + j
                got = aloc[ap[e]:ap[e + 1]].tolist()
                assert got == [jj for jj, u in enumerate(hood) if u in nbrs[v]], (h, j)
        for v in range(n):
            h0 = min(h for h, c in enumerate(cl) if v in c)
            assert owner[v] == hp[h0] + hl[h0].index(v), v
            assert nbrs[v] <= set(hl[h0])  # the owner's hood holds all of N(v)
        if n > 100:
            assert max(len(c) for c in cl) <= 4  # planar region graph


def _random_theta(rng, L):
    mu = np.sort(rng.uniform(20, 230, size=L))
    sigma = rng.uniform(5, 40, size=L)
    return mu, sigma


def check_data_term(lib):
    g = synth.workload_small()
    og = oracle.OracleGraph(g.n, g.row_ptr, g.col_idx, lib=lib)
    rng = np.random.default_rng(7)
    hp, hv = og.hoods()
    for L in (2, 3, 5):
        mu, sigma = _random_theta(rng, L)
        x = rng.integers(0, L, g.n).astype(np.int32)
        out = og.em_step(g.y, L, 0.0, x, mu, sigma, per_element=True)
        D = data_energy(g.y, mu, sigma)
        want_m = D.min(axis=1)[hv]
        assert np.allclose(out["m"], want_m, rtol=1e-12, atol=1e-12)
        S_want = np.add.reduceat(want_m, hp[:-1]) if og.H else np.zeros(0)
        assert np.allclose(out["S"], S_want, rtol=1e-12, atol=1e-10)
        assert abs(out["T"] - S_want.sum()) <= 1e-12 * abs(S_want.sum())
        srt = np.sort(D, axis=1)
        clear = (srt[:, 1] - srt[:, 0])[hv] > 1e-9
        assert np.array_equal(out["a"][clear], D.argmin(axis=1)[hv][clear])


def icm_step(n, rp, ci, y, L, beta, x, mu, sigma):
    """Synchronous iterated conditional modes directly on the CSR graph."""
    D = data_energy(y, mu, sigma)
    E = D.copy()
    for v in range(n):
        nb = x[ci[rp[v]:rp[v + 1]]]
        for l in range(L):
            E[v, l] += beta * np.count_nonzero(nb != l)
    srt = np.sort(E, axis=1)
    return E.argmin(axis=1), srt[:, 1] - srt[:, 0]


def check_sync_icm(lib):
    rng = np.random.default_rng(11)
    gs = [synth.workload_small(), synth.powerlaw_graph(17, 3000, phases=3)]
    for g in gs:
        og = oracle.OracleGraph(g.n, g.row_ptr, g.col_idx, lib=lib)
        for L, beta in ((2, 0.5), (3, 0.8), (4, 2.0)):
            mu, sigma = _random_theta(rng, L)
            x = rng.integers(0, L, g.n).astype(np.int32)
            out = og.em_step(g.y, L, beta, x, mu, sigma)
            want, gap = icm_step(g.n, g.row_ptr, g.col_idx, g.y, L, beta, x, mu, sigma)
            clear = gap > 1e-9
            assert clear.mean() > 0.99
            assert np.array_equal(out["x"][clear], want[clear])
            assert out["x"].min() >= 0 and out["x"].max() < L


def check_tie_rule(lib):
    # exact tie by symmetry: y halfway between two means with equal sigma
    rp, ci = csr(2, [(0, 1)])
    og = oracle.OracleGraph(2, rp, ci, lib=lib)
    y = np.array([5.0, 5.0])
    out = og.em_step(y, 2, 0.0, np.array([1, 1]), [0.0, 10.0], [1.0, 1.0], per_element=True)
    assert list(out["x"]) == [0, 0] and out["near_ties"] == 2
    # the Potts count breaks the same tie towards the neighbours' label
    out = og.em_step(y, 2, 0.5, np.array([1, 1]), [0.0, 10.0], [1.0, 1.0])
    assert list(out["x"]) == [1, 1] and out["near_ties"] == 0
    out = og.em_step(y, 2, 0.5, np.array([0, 1]), [0.0, 10.0], [1.0, 1.0])
    assert list(out["x"]) == [1, 0]  # each takes the other's label (synchronous update)


def global_energy(n, edges, D, beta, x):
    U = D[np.arange(n), x].sum()
    for a, b in edges:
        U += beta * (x[a] != x[b])
    return U


def check_exhaustive(lib):
    rng = np.random.default_rng(23)
    # 24 mixed cases (n = 3..7, L = 2..4), then every 8-vertex case at L = 2 and 3
    sizes = []
    for s in range(24):
        n = 3 + s % 5
        L = 2 + s % 3
        if L ** n > 20000:
            n = 5
        sizes.append((n, L))
    sizes += [(8, 2), (8, 2), (8, 3), (8, 3)]
    for s, (n, L) in enumerate(sizes):
        rp, ci = synth.small_random_graph(500 + s, n, 0.5)
        edges = [(v, u) for v in range(n) for u in ci[rp[v]:rp[v + 1]] if u > v]
        og = oracle.OracleGraph(n, rp, ci, lib=lib)
        y = rng.uniform(0, 255, n)
        mu, sigma = _random_theta(rng, L)
        beta = float(rng.uniform(0.2, 30.0))
        D = data_energy(y, mu, sigma)
        best, xbest = None, None
        for xs in itertools.product(range(L), repeat=n):
            x = np.array(xs)
            U = global_energy(n, edges, D, beta, x)
            if best is None or U < best:
                best, xbest = U, x
        # a global minimiser with clear conditional minima is a fixed point
        _, gap = icm_step(n, rp, ci, y, L, beta, xbest, mu, sigma)
        if (gap > 1e-9).all():
            out = og.em_step(y, L, beta, xbest.astype(np.int32), mu, sigma)
            assert np.array_equal(out["x"], xbest), (s, out["x"], xbest)
        # beta = 0: one step from any labelling reaches the global minimiser
        x0 = rng.integers(0, L, n).astype(np.int32)
        out0 = og.em_step(y, L, 0.0, x0, mu, sigma)
        srt = np.sort(D, axis=1)
        if ((srt[:, 1] - srt[:, 0]) > 1e-9).all():
            assert np.array_equal(out0["x"], D.argmin(axis=1))
        # hood energy after the argmin never exceeds the energy at the incoming labels
        x1 = rng.integers(0, L, n).astype(np.int32)
        out1 = og.em_step(y, L, beta, x1, mu, sigma)
        A = adj_matrix(n, rp, ci)
        _, hl = oracle_lists(og)
        for h, hood in enumerate(hl):
            hood = list(hood)
            e_in = sum(D[v, x1[v]] + beta * sum(1 for u in hood if A[v, u] and x1[u] != x1[v]) for v in hood)
            assert out1["S"][h] <= e_in + 1e-9 * abs(e_in), (s, h)


def check_mstep(lib):
    rng = np.random.default_rng(31)
    y = rng.uniform(0, 255, 5000)
    for L in (2, 3, 6):
        x = rng.integers(0, L - 1, y.size).astype(np.int32)  # label L-1 stays empty
        mu_in = rng.uniform(0, 255, L)
        s_in = rng.uniform(1, 50, L)
        mu, sg = oracle.mstep(y, L, x, mu_in, s_in, 1e-3, lib=lib)
        for l in range(L - 1):
            sel = y[x == l]
            assert abs(mu[l] - sel.mean()) <= 1e-13 * abs(sel.mean())
            assert abs(sg[l] - sel.std(ddof=0)) <= 1e-12 * sel.std(ddof=0)
            # maximum likelihood: nearby parameters do not fit better
            nll = lambda m, s: -norm.logpdf(sel, m, s).sum()
            base = nll(mu[l], sg[l])
            for d in (1e-3, 1e-1):
                assert nll(mu[l] + d, sg[l]) >= base and nll(mu[l] - d, sg[l]) >= base
                assert nll(mu[l], sg[l] * (1 + d)) >= base and nll(mu[l], sg[l] * (1 - d)) >= base
        assert mu[L - 1] == mu_in[L - 1] and sg[L - 1] == s_in[L - 1]  # empty label keeps
    # constant intensities: sigma floors at sigma_min
    mu, sg = oracle.mstep(np.full(10, 42.0), 2, np.zeros(10, np.int32), [0.0, 0.0], [1.0, 1.0], 0.25, lib=lib)
    assert mu[0] == 42.0 and sg[0] == 0.25


def cem_beta0(y, L, x, iters, sigma_min):
    """Classification EM for a 1-D Gaussian mixture (no smoothness term)."""
    mu = np.array([y[x == l].mean() if (x == l).any() else 0.0 for l in range(L)])
    sg = np.array([max(y[x == l].std(ddof=0), sigma_min) if (x == l).any() else 1.0 for l in range(L)])
    for _ in range(iters):
        x = data_energy(y, mu, sg).argmin(axis=1)
        for l in range(L):
            sel = y[x == l]
            if sel.size:
                mu[l] = sel.mean()
                sg[l] = max(sel.std(ddof=0), sigma_min)
    return x, mu, sg


def check_cem(lib):
    for g, L in ((synth.workload_small(), 2), (synth.image_graph(9, 200, 700, 3), 3)):
        og = oracle.OracleGraph(g.n, g.row_ptr, g.col_idx, lib=lib)
        x0 = synth.threshold_labels(g.y, L)
        out = og.em_run(g.y, L, 0.0, x0, np.zeros(L), np.ones(L), 12, init_from_labels=True)
        xw, muw, sgw = cem_beta0(g.y, L, x0.copy(), 12, 1e-3)
        assert np.array_equal(out["x"], xw)
        assert np.allclose(out["mu"], muw, rtol=1e-12) and np.allclose(out["sigma"], sgw, rtol=1e-11)


def check_udata_monotone(lib):
    g = synth.image_graph(13, 256, 900, 2)
    og = oracle.OracleGraph(g.n, g.row_ptr, g.col_idx, lib=lib)
    rng = np.random.default_rng(3)
    x = rng.integers(0, 2, g.n).astype(np.int32)
    mu, sigma = np.array([60.0, 200.0]), np.array([30.0, 30.0])
    prev = None
    for _ in range(8):
        u = data_energy(g.y, mu, sigma)[np.arange(g.n), x].sum()
        assert prev is None or u <= prev + 1e-9 * abs(prev)
        prev = u
        out = og.em_step(g.y, 2, 0.0, x, mu, sigma)
        # the E-step alone also lowers it: new labels under the old parameters
        assert data_energy(g.y, mu, sigma)[np.arange(g.n), out["x"]].sum() <= u + 1e-9 * abs(u)
        x, mu, sigma = out["x"], out["mu"], out["sigma"]


def check_convergence(lib):
    hc = lambda h, tol=1e-4: oracle.hood_converged(np.array(h, dtype=float), tol, lib=lib)
    assert hc([5.0, 5.0, 5.0, 5.0])
    assert hc([5.0, 5.0 + 9e-5, 5.0 - 9e-5 + 9e-5, 5.0])
    assert not hc([5.0 + 2e-4, 5.0, 5.0, 5.0])  # oldest of the three differs
    assert not hc([5.0, 5.0, 5.0 + 2e-4, 5.0])  # newest previous differs
    assert not hc([5.0, 5.0, 5.0, 5.0 + 1e-4 * 1.5])
    assert not hc([1.0, 1.0, 1.0, 1.0 + 0.5], tol=0.5)  # strict inequality
    assert hc([1.0, 1.0], tol=1e-4) and not hc([1.0, 2.0], tol=0.5)  # window of one
    # the loop: beta = 0 classification EM becomes stationary; the first
    # all-converged iteration is the first t >= 3 whose sums equal the previous three
    g = synth.workload_small()
    og = oracle.OracleGraph(g.n, g.row_ptr, g.col_idx, lib=lib)
    x0 = synth.threshold_labels(g.y, 2)
    run = og.em_run(g.y, 2, 0.0, x0, np.zeros(2), np.ones(2), 20, init_from_labels=True)
    x, (mu, sg) = x0.copy(), oracle.mstep(g.y, 2, x0, np.zeros(2), np.ones(2), lib=lib)
    hist = []
    for t in range(20):
        out = og.em_step(g.y, 2, 0.0, x, mu, sg)
        hist.append(out["S"])
        assert run["trace"][t] == out["T"]
        x, mu, sg = out["x"], out["mu"], out["sigma"]
    want = next((t for t in range(3, 20) if all(np.all(np.abs(hist[t] - hist[t - w]) < 1e-4) for w in (1, 2, 3))), -1)
    assert want > 0 and run["map_conv_iter"] == want
    assert (run["nonconv"][:3] == og.H).all()
    early = og.em_run(g.y, 2, 0.0, x0, np.zeros(2), np.ones(2), 20, early_exit=True, init_from_labels=True)
    assert early["iters"] == want + 1 and np.array_equal(early["x"], run["x"])


def check_k_hoods(lib):
    """k-neighbourhoods (Sec. 3.1): clique plus every vertex within k edges of a
    member, by reachability through powers of (I + A); closed forms on paths
    and stars; the owner rule still sees every neighbour, so at k = 2 the labels
    equal synchronous ICM on the graph."""
    graphs = list(random_small_graphs(40))
    for k in (2, 3):
        for n, rp, ci in graphs:
            og = oracle.OracleGraph(n, rp, ci, lib=lib, k=k)
            og1 = oracle.OracleGraph(n, rp, ci, lib=lib)
            cl, hl = oracle_lists(og)
            assert cl == oracle_lists(og1)[0]  # the cliques do not depend on k
            A = adj_matrix(n, rp, ci)
            R = np.eye(n, dtype=np.int64)
            step = (np.eye(n, dtype=np.int64) + A.astype(np.int64))
            for _ in range(k):
                R = np.minimum(R @ step, 1)
            hp, hv = og.hoods()
            ap, aloc = og.adjacency()
            for h, (c, hood) in enumerate(zip(cl, hl)):
                want = sorted(set(np.nonzero(R[list(c)].any(axis=0))[0].tolist()))
                assert list(hood) == want, (k, h, hood, want)
                for j, v in enumerate(hood):
                    e = hp[h] + j
                    assert aloc[ap[e]:ap[e + 1]].tolist() == [jj for jj, u in enumerate(hood) if A[v, u]], (k, h, j)
    for n in range(3, 9):  # path, k = 2: hood(edge i, i+1) = {i-2 .. i+3}
        rp, ci = csr(n, [(i, i + 1) for i in range(n - 1)])
        og = oracle.OracleGraph(n, rp, ci, lib=lib, k=2)
        _, hl = oracle_lists(og)
        assert hl == [tuple(range(max(0, i - 2), min(n - 1, i + 3) + 1)) for i in range(n - 1)], (n, hl)
    rp, ci = csr(7, [(0, i) for i in range(1, 7)] + [(1, 2)])  # star with one chord, k = 2: every hood = V
    og = oracle.OracleGraph(7, rp, ci, lib=lib, k=2)
    assert all(h == tuple(range(7)) for h in oracle_lists(og)[1])
    g = synth.workload_small()
    og = oracle.OracleGraph(g.n, g.row_ptr, g.col_idx, lib=lib, k=2)
    rng = np.random.default_rng(13)
    for L, beta in ((2, 0.5), (3, 0.8)):
        mu, sigma = _random_theta(rng, L)
        x = rng.integers(0, L, g.n).astype(np.int32)
        out = og.em_step(g.y, L, beta, x, mu, sigma)
        want, gap = icm_step(g.n, g.row_ptr, g.col_idx, g.y, L, beta, x, mu, sigma)
        clear = gap > 1e-9
        assert np.array_equal(out["x"][clear], want[clear])


def check_scatter_rules(lib):
    """Scatter rules of "Update Output Labels": the last write of a serial
    Scatter over the hood-major array, the minimum over a vertex's
    occurrences (first on ties), and a hand-worked path where the three rules
    part; at beta = 0 all occurrences of a vertex agree, so the rules do."""
    R = oracle
    # hand-worked: path 0-1-2-3, cliques {0,1} {1,2} {2,3}, hoods {0,1,2} {0,1,2,3} {1,2,3}.
    # Vertex 1: the first two hoods hold both its neighbours (energies d_l + beta each,
    # one disagreeing neighbour per label: x_0 = 1, x_2 = 0); the third holds only
    # vertex 2 (energies d_0 and d_1 + beta).  With d_0 - d_1 = 0.1 < beta = 0.5:
    # owner -> label 1; last hood -> 0; minimum (d_0 < d_1 + beta) -> 0.
    rp, ci = csr(4, [(0, 1), (1, 2), (2, 3)])
    og = oracle.OracleGraph(4, rp, ci, lib=lib)
    y = np.array([0.0, 5.01, 10.0, 10.0])
    x = np.array([1, 0, 0, 1], np.int32)
    got = {rule: int(og.em_step(y, 2, 0.5, x, [0.0, 10.0], [1.0, 1.0], rule=rule)["x"][1])
           for rule in (R.RULE_OWNER, R.RULE_LAST, R.RULE_MIN)}
    assert got == {R.RULE_OWNER: 1, R.RULE_LAST: 0, R.RULE_MIN: 0}, got
    # exact tie across occurrences: y_1 = 5.25 gives d_0 = 13.78125, d_1 = 11.28125
    # (exact in binary), beta = 2.5: every occurrence of vertex 1 has minimum
    # 13.78125, the first two at label 1, the third (a tie inside it, lowest
    # label) at label 0; the minimum rule takes the first occurrence
    y = np.array([0.0, 5.25, 10.0, 10.0])
    out = {rule: og.em_step(y, 2, 2.5, x, [0.0, 10.0], [1.0, 1.0], per_element=True, rule=rule)
           for rule in (R.RULE_OWNER, R.RULE_LAST, R.RULE_MIN)}
    hp, hv = og.hoods()
    occ = np.nonzero(hv == 1)[0]
    assert np.all(out[R.RULE_MIN]["m"][occ] == 13.78125) and list(out[R.RULE_MIN]["a"][occ]) == [1, 1, 0]
    assert [int(out[r]["x"][1]) for r in (R.RULE_OWNER, R.RULE_LAST, R.RULE_MIN)] == [1, 0, 1]
    rng = np.random.default_rng(29)
    cases = [(n, rp, ci) for n, rp, ci in random_small_graphs(30)]
    g = synth.workload_small()
    cases.append((g.n, g.row_ptr, g.col_idx))
    for n, rp, ci in cases:
        og = oracle.OracleGraph(n, rp, ci, lib=lib)
        hp, hv = og.hoods()
        yv = rng.uniform(0, 255, n)
        for L, beta in ((2, 0.0), (2, 0.7), (3, 1.5)):
            mu, sigma = _random_theta(rng, L)
            x = rng.integers(0, L, n).astype(np.int32)
            outs = {rule: og.em_step(yv, L, beta, x, mu, sigma, per_element=True, rule=rule)
                    for rule in (R.RULE_OWNER, R.RULE_LAST, R.RULE_MIN)}
            m, a = outs[R.RULE_OWNER]["m"], outs[R.RULE_OWNER]["a"]
            for o in outs.values():  # the rule changes only the label update
                assert np.array_equal(o["m"], m) and np.array_equal(o["S"], outs[R.RULE_OWNER]["S"])
            sim = x.copy()  # a serial Scatter over the hood-major array
            for e in range(len(hv)):
                sim[hv[e]] = a[e]
            assert np.array_equal(outs[R.RULE_LAST]["x"], sim)
            owner = og.owner()
            for v in range(n):
                occ = np.nonzero(hv == v)[0]
                best = occ[np.argmin(m[occ])]
                assert outs[R.RULE_MIN]["x"][v] == a[best], (v, occ)
                assert m[best] <= m[owner[v]] and m[best] <= m[occ[-1]]
            if beta == 0.0:
                for rule in (R.RULE_LAST, R.RULE_MIN):
                    assert np.array_equal(outs[rule]["x"], outs[R.RULE_OWNER]["x"])
                    assert outs[rule]["near_ties"] == outs[R.RULE_OWNER]["near_ties"]
    # minimum rule, near tie between occurrences: vertex 1 at gap 0.1 in every
    # hood, but its minimum differs by 1e-12 between the two kinds of hoods with
    # different labels (d_0 - d_1 = beta - 1e-12)
    d = 0.5 - 1e-12
    y1 = (d + 50.0) / 10.0  # (y^2 - (y - 10)^2) / 2 = 10 y - 50 = d
    out = oracle.OracleGraph(4, *csr(4, [(0, 1), (1, 2), (2, 3)]), lib=lib).em_step(
        np.array([0.0, y1, 10.0, 10.0]), 2, 0.5, np.array([1, 0, 0, 1], np.int32), [0.0, 10.0], [1.0, 1.0],
        rule=R.RULE_MIN)
    assert out["near_ties"] >= 1


ALL_CHECKS = [
    check_worked_example,
    check_cliques_bruteforce,
    check_closed_forms,
    check_hoods_adjacency_owner,
    check_data_term,
    check_sync_icm,
    check_tie_rule,
    check_exhaustive,
    check_mstep,
    check_cem,
    check_udata_monotone,
    check_convergence,
    check_k_hoods,
    check_scatter_rules,
]
