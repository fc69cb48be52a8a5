"""Seeded synthetic inputs for the PMRF EM path.

This module only draws inputs: two-phase images, their jittered-grid Voronoi
oversegmentation, the region-adjacency graph (CSR), region mean intensities,
power-law stress graphs, and a threshold labelling used as the initial labels.
It holds none of the method's arithmetic (no energies, no argmin, no parameter
estimation), so both the oracle and the HIP path can be fed from it.

The paper evaluates on a noisy porous-media benchmark stack and on beamline
slices (Section 4.1, "Datasets"); neither is available here.  The generators
below stand in for their shape: 2D 8-bit slices with two (or more) Gaussian
phases, oversegmented into irregular regions whose adjacency graph is the
optimisation input (Section 3.1, graph construction).

Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64), drawn in
the order documented per function.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class GraphInput:
    """One optimisation problem: a CSR region graph plus per-region intensity."""

    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col_idx: np.ndarray  # int32[nnz], sorted per row, symmetric, no self loops
    y: np.ndarray  # float64[n] region mean intensity
    truth: np.ndarray | None = None  # int32[n] generating phase per region (majority)
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


PHASE_MEANS = {2: (80.0, 170.0), 3: (60.0, 128.0, 196.0), 4: (40.0, 100.0, 160.0, 220.0)}
PHASE_SD = {2: 25.0, 3: 22.0, 4: 20.0}


def phase_field(rng: np.random.Generator, side: int, phases: int, smooth: float = 8.0) -> np.ndarray:
    """White N(0,1) noise, Gaussian-smoothed with periodic wrap, cut at quantiles."""
    from scipy.ndimage import gaussian_filter

    noise = rng.standard_normal((side, side))
    field = gaussian_filter(noise, sigma=smooth, mode="wrap")
    cuts = np.quantile(field, [k / phases for k in range(1, phases)])
    return np.searchsorted(cuts, field, side="right").astype(np.int32)


def two_phase_image(rng: np.random.Generator, side: int, phases: int = 2):
    """uint8 image: per-pixel N(mean[phase], sd) rounded and clipped to [0, 255]."""
    ph = phase_field(rng, side, phases)
    means = np.asarray(PHASE_MEANS[phases])
    pix = rng.normal(means[ph], PHASE_SD[phases])
    img = np.clip(np.rint(pix), 0, 255).astype(np.uint8)
    return img, ph


def jittered_voronoi(rng: np.random.Generator, side: int, regions: int) -> np.ndarray:
    """Region id per pixel: one seed uniform in each cell of a g x g grid, pixel
    centres go to the nearest seed, empty regions dropped, ids compacted in
    row-major cell order."""
    from scipy.spatial import cKDTree

    g = max(1, int(round(side / math.sqrt(side * side / regions))))
    cell = side / g
    gi, gj = np.meshgrid(np.arange(g), np.arange(g), indexing="ij")
    sy = (gi.ravel() + rng.random(g * g)) * cell
    sx = (gj.ravel() + rng.random(g * g)) * cell
    tree = cKDTree(np.stack([sy, sx], axis=1))
    py, px = np.meshgrid(np.arange(side) + 0.5, np.arange(side) + 0.5, indexing="ij")
    _, idx = tree.query(np.stack([py.ravel(), px.ravel()], axis=1), workers=-1)
    used = np.zeros(g * g, dtype=bool)
    used[idx] = True
    remap = np.cumsum(used) - 1
    return remap[idx].reshape(side, side).astype(np.int32)


def rag_csr(lab: np.ndarray):
    """4-connected region adjacency graph as a symmetric, row-sorted CSR."""
    n = int(lab.max()) + 1
    a = np.concatenate([lab[:, :-1].ravel(), lab[:-1, :].ravel()])
    b = np.concatenate([lab[:, 1:].ravel(), lab[1:, :].ravel()])
    keep = a != b
    return csr_from_edges(n, a[keep], b[keep])


def csr_from_edges(n: int, a: np.ndarray, b: np.ndarray):
    """Symmetric CSR from an undirected edge list; drops self loops and repeats."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    keep = a != b
    a, b = a[keep], b[keep]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = np.unique(lo * n + hi)
    lo, hi = key // n, key % n
    src = np.concatenate([lo, hi])
    dst = np.concatenate([hi, lo])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr.astype(np.int32), dst.astype(np.int32)


def image_slice(seed: int, side: int, regions: int, phases: int = 2):
    """The inputs of an image slice: the uint8 image, its oversegmentation
    (int32 region id per pixel) and the generating phase per pixel.

    Draw order from ``default_rng(seed)``: smoothing noise (side^2 normals),
    pixel noise (side^2 normals), seed jitter (2 g^2 uniforms)."""
    rng = np.random.default_rng(seed)
    img, ph = two_phase_image(rng, side, phases)
    lab = jittered_voronoi(rng, side, regions)
    return img, lab, ph


def image_graph(seed: int, side: int, regions: int, phases: int = 2, name: str = "") -> GraphInput:
    """Image slice -> oversegmentation -> RAG with region-mean intensities
    (the draws of ``image_slice``)."""
    img, lab, ph = image_slice(seed, side, regions, phases)
    row_ptr, col_idx = rag_csr(lab)
    n = row_ptr.size - 1
    cnt = np.bincount(lab.ravel(), minlength=n).astype(np.float64)
    y = np.bincount(lab.ravel(), weights=img.ravel().astype(np.float64), minlength=n) / cnt
    # ground-truth phase per region: the most frequent generating phase
    votes = np.zeros((n, phases), dtype=np.int64)
    np.add.at(votes, (lab.ravel(), ph.ravel()), 1)
    truth = votes.argmax(axis=1).astype(np.int32)
    return GraphInput(n=n, row_ptr=row_ptr, col_idx=col_idx, y=y, truth=truth,
                      name=name or f"image{side}_r{regions}_s{seed}",
                      meta={"side": side, "regions": regions, "phases": phases, "seed": seed,
                            "pixels_per_region": float(side * side) / n})


def powerlaw_graph(seed: int, n: int, phases: int = 4, dmin: int = 3, dmax: int = 30,
                   exponent: float = 2.5, sd: float = 20.0, name: str = "") -> GraphInput:
    """Degree-skewed stress graph (not an image).

    Degrees from P(d) ~ d^-exponent on [dmin, dmax]; configuration model with
    self loops and repeated edges dropped.  Phases uniform in [0, phases), then
    three synchronous neighbour-majority rounds (a vertex keeps its phase unless
    one phase has a strict majority count among its neighbours).  Intensity
    y = clip(N(mean[phase], sd), 0, 255) in float64.

    Draw order: n degree uniforms, one stub permutation, n phase integers,
    n intensity normals."""
    rng = np.random.default_rng(seed)
    d = np.arange(dmin, dmax + 1)
    p = d.astype(np.float64) ** (-exponent)
    p /= p.sum()
    deg = d[np.searchsorted(np.cumsum(p), rng.random(n), side="right").clip(0, d.size - 1)]
    if deg.sum() % 2:
        deg[0] += 1
    stubs = np.repeat(np.arange(n), deg)
    stubs = stubs[rng.permutation(stubs.size)]
    row_ptr, col_idx = csr_from_edges(n, stubs[0::2], stubs[1::2])
    ph = rng.integers(0, phases, size=n).astype(np.int32)
    src = np.repeat(np.arange(n), np.diff(row_ptr))
    for _ in range(3):
        votes = np.zeros((n, phases), dtype=np.int64)
        np.add.at(votes, (src, ph[col_idx]), 1)
        top = votes.max(axis=1)
        unique_top = (votes == top[:, None]).sum(axis=1) == 1
        ph = np.where(unique_top & (top > 0), votes.argmax(axis=1), ph).astype(np.int32)
    means = np.asarray(PHASE_MEANS[phases])
    y = np.clip(rng.normal(means[ph], sd), 0.0, 255.0)
    return GraphInput(n=n, row_ptr=row_ptr, col_idx=col_idx, y=y, truth=ph,
                      name=name or f"powerlaw_n{n}_s{seed}",
                      meta={"n": n, "seed": seed, "phases": phases})


def threshold_labels(y: np.ndarray, L: int) -> np.ndarray:
    """Simple-threshold labelling: label = min(L-1, floor(y * L / 256))."""
    return np.minimum(L - 1, np.floor(np.asarray(y) * L / 256.0)).astype(np.int32)


def random_init(seed: int, n: int, L: int):
    """Random labels in [0, L) and per-label mu, sigma uniform in [0, 255]
    (Section 3.2.2 initialisation); sigma is kept away from 0 by drawing from
    [1, 255]."""
    rng = np.random.default_rng(seed)
    x = rng.integers(0, L, size=n).astype(np.int32)
    mu = rng.uniform(0.0, 255.0, size=L)
    sigma = rng.uniform(1.0, 255.0, size=L)
    return x, mu, sigma


def small_random_graph(seed: int, n: int, p: float) -> tuple[np.ndarray, np.ndarray]:
    """Erdos-Renyi G(n, p) as CSR (for exhaustive tests on tiny graphs)."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    return csr_from_edges(n, iu[keep], ju[keep])


# ---------------------------------------------------------------------------
# Named workloads (sizes of the five evaluation configurations)
# ---------------------------------------------------------------------------

def workload_small(seed: int = 1) -> GraphInput:
    """256 x 256 two-phase slice, ~1,000 regions."""
    return image_graph(seed, 256, 1000, 2, name="slice256_1k")


def workload_large(seed: int = 2) -> GraphInput:
    """2048 x 2048 two-phase slice, ~100k regions."""
    return image_graph(seed, 2048, 100_000, 2, name="slice2048_100k")


def batch_sides(count: int = 64, seed: int = 3, lo: int = 512, hi: int = 2560):
    """Slice sides log-uniform in [lo, hi]; regions = round(side^2 / 26.2)."""
    rng = np.random.default_rng(seed)
    sides = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(int)
    return [(int(s), int(round(s * s / 26.2))) for s in sides]


def _draw_all(fn, args, workers: int, progress=None):
    """fn(*a) for every a in args, in order; with workers > 1 in forked worker
    processes (each draw has its own seed, so the result is the same).
    ``progress(i, count)`` is called after each serial draw."""
    if workers <= 1 or len(args) <= 1:
        out = []
        for i, a in enumerate(args):
            out.append(fn(*a))
            if progress:
                progress(i + 1, len(args))
        return out
    import multiprocessing as mp

    with mp.get_context("fork").Pool(min(workers, len(args))) as pool:
        return pool.starmap(fn, args, chunksize=1)


def workload_batch(count: int = 64, seed: int = 3, scale: float = 1.0, workers: int = 1, progress=None):
    """Uneven slices for the batched path (``scale`` shrinks sides for tests).
    ``workers`` > 1 draws the slices in forked processes: call it before the
    process touches a GPU."""
    args = []
    for i, (s, r) in enumerate(batch_sides(count, seed)):
        s2 = max(32, int(round(s * scale)))
        r2 = max(16, int(round(s2 * s2 / 26.2)))
        args.append((seed * 1000 + i, s2, r2, 2, f"batch{i}_{s2}"))
    return _draw_all(image_graph, args, workers, progress)


def workload_skewed(count: int = 16, n: int = 500_000, seed: int = 4, workers: int = 1, progress=None):
    """Power-law graphs, L=4 phases (``workers`` as for ``workload_batch``)."""
    args = [(seed * 1000 + i, n, 4, 3, 30, 2.5, 20.0, f"powerlaw{i}") for i in range(count)]
    return _draw_all(powerlaw_graph, args, workers, progress)


def serving_requests(count: int = 256, seed: int = 5, rmin: int = 1000, rmax: int = 1_000_000):
    """Request descriptors: (request seed, side, regions, L); graphs are drawn
    lazily with ``image_graph``.  Regions log-uniform, L uniform in {2, 3, 4}."""
    rng = np.random.default_rng(seed)
    regions = np.rint(np.exp(rng.uniform(math.log(rmin), math.log(rmax), size=count))).astype(int)
    labels = rng.integers(2, 5, size=count)
    reqs = []
    for j in range(count):
        side = int(round(math.sqrt(26.2 * regions[j])))
        reqs.append({"seed": seed * 1000 + j, "side": side, "regions": int(regions[j]), "L": int(labels[j])})
    return reqs


def poisson_arrivals(count: int, rate: float, seed: int = 5) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed + 7919)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
