"""Oracle of the image-in / segmentation-out steps, written from their
definitions: the region adjacency graph and region means of an oversegmented
image (the graph the optimisation takes, Sec. 5; the input of Alg. 2), the
labels painted back onto the pixels (its output), and the confusion counts
and verification metrics of Sec. 4.2.1.

TEST INFRASTRUCTURE ONLY (imported by ``tests/`` and ``bench.py``'s CPU leg;
the product path never imports it, and it imports nothing from the product).
Plain NumPy: each step is its definition written out; a sort (``np.unique``)
is the only library primitive.
"""
from __future__ import annotations

import numpy as np


def adjacent_pairs(regions: np.ndarray) -> np.ndarray:
    """Unordered pairs (u, v), u < v, of regions that touch: a pixel (voxel) of
    u and one of v are neighbours along one axis (4-connectivity in an image,
    6-connectivity in a volume).  Returns int64[m, 2] in ascending
    lexicographic order."""
    reg = np.asarray(regions, dtype=np.int64)
    a_parts, b_parts = [], []
    for axis in range(reg.ndim):  # a pixel and its next neighbour along the axis
        lo = [slice(None)] * reg.ndim
        hi = [slice(None)] * reg.ndim
        lo[axis] = slice(None, -1)
        hi[axis] = slice(1, None)
        a_parts.append(reg[tuple(lo)].ravel())
        b_parts.append(reg[tuple(hi)].ravel())
    a = np.concatenate(a_parts)
    b = np.concatenate(b_parts)
    differ = a != b
    lo = np.minimum(a[differ], b[differ])
    hi = np.maximum(a[differ], b[differ])
    if lo.size == 0:
        return np.zeros((0, 2), dtype=np.int64)
    return np.unique(np.stack([lo, hi], axis=1), axis=0)


def region_graph(regions: np.ndarray, n: int):
    """Symmetric CSR (row_ptr int32[n+1], col_idx int32[nnz]) of the region
    adjacency graph, every row ascending."""
    pairs = adjacent_pairs(regions)
    rows = [[] for _ in range(n)]
    for u, v in pairs.tolist():
        rows[u].append(v)
        rows[v].append(u)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    for u in range(n):
        rows[u].sort()
        row_ptr[u + 1] = row_ptr[u] + len(rows[u])
    col_idx = np.array([v for r in rows for v in r], dtype=np.int64)
    return row_ptr.astype(np.int32), col_idx.astype(np.int32)


def region_means(regions: np.ndarray, pixels: np.ndarray, n: int) -> np.ndarray:
    """Mean pixel value of each region: the integer sum over the pixel count,
    in FP64 (0 for a region without pixels)."""
    reg = np.asarray(regions, dtype=np.int64).ravel()
    pix = np.asarray(pixels, dtype=np.int64).ravel()
    sums = np.zeros(n, dtype=np.int64)
    counts = np.zeros(n, dtype=np.int64)
    np.add.at(sums, reg, pix)
    np.add.at(counts, reg, 1)
    out = np.zeros(n, dtype=np.float64)
    has = counts > 0
    out[has] = sums[has].astype(np.float64) / counts[has].astype(np.float64)
    return out


def labels_to_pixels(regions: np.ndarray, labels: np.ndarray, n: int) -> np.ndarray:
    """Each pixel takes its region's label (255 for an id outside [0, n) or a
    label outside [0, 255))."""
    reg = np.asarray(regions, dtype=np.int64)
    lab = np.asarray(labels, dtype=np.int64)
    out = np.full(reg.shape, 255, dtype=np.uint8)
    ok = (reg >= 0) & (reg < n)
    vals = lab[reg[ok]]
    good = (vals >= 0) & (vals < 255)
    sub = out[ok]
    sub[good] = vals[good].astype(np.uint8)
    out[ok] = sub
    return out


def confusion(a: np.ndarray, b: np.ndarray, k: int) -> np.ndarray:
    """counts[i, j] = number of pixels with a = i and b = j (i, j < k)."""
    a = np.asarray(a, dtype=np.int64).ravel()
    b = np.asarray(b, dtype=np.int64).ravel()
    keep = (a < k) & (b < k)
    counts = np.zeros((k, k), dtype=np.int64)
    np.add.at(counts, (a[keep], b[keep]), 1)
    return counts


def scores(counts: np.ndarray, positive: int = 1, void: int = 0) -> dict:
    """Sec. 4.2.1: precision TP/(TP+FP), recall TP/(TP+FN), accuracy
    (TP+TN)/(TP+TN+FP+FN) for the positive label (rows: segmentation, columns:
    ground truth), and porosity = void volume / total volume of the
    segmentation."""
    c = np.asarray(counts, dtype=np.int64)
    tp = c[positive, positive]
    fp = c[positive, :].sum() - tp
    fn = c[:, positive].sum() - tp
    tn = c.sum() - tp - fp - fn
    return {"precision": tp / (tp + fp), "recall": tp / (tp + fn),
            "accuracy": (tp + tn) / (tp + tn + fp + fn), "porosity": c[void, :].sum() / c.sum()}
