"""Pins of the image-in / segmentation-out oracle (CPU): a hand-worked example,
closed forms (stripes, block grids, one region per pixel), an independent
construction (the input generator's graph and means), and the paper's metric
formulas on counts worked by hand."""
import os

import numpy as np
import pytest

from oracle import image as oi
from paper_1809_05018_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "image_graph_example.txt")


def read_golden():
    sections, cur = {}, None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.isalpha():
            cur = sections.setdefault(line, [])
        else:
            cur.append(line)
    regions = np.array([[int(v) for v in r.split()] for r in sections["regions"]], dtype=np.int32)
    pixels = np.array([[int(v) for v in r.split()] for r in sections["pixels"]], dtype=np.uint8)
    nbrs = {int(k): [int(v) for v in rest.split()] for k, rest in (r.split(":") for r in sections["neighbours"])}
    sums = {int(k): tuple(int(v) for v in rest.split()) for k, rest in (r.split(":") for r in sections["sums"])}
    return regions, pixels, nbrs, sums


def test_worked_example():
    regions, pixels, nbrs, sums = read_golden()
    n = len(nbrs)
    row_ptr, col_idx = oi.region_graph(regions, n)
    for u in range(n):
        assert col_idx[row_ptr[u]:row_ptr[u + 1]].tolist() == nbrs[u]
    means = oi.region_means(regions, pixels, n)
    for u, (s, c) in sums.items():
        assert means[u] == s / c


@pytest.mark.parametrize("height,width,stripe", [(7, 30, 3), (1, 12, 1), (5, 9, 9)])
def test_vertical_stripes_form_a_path(height, width, stripe):
    regions = np.tile(np.arange(width, dtype=np.int32) // stripe, (height, 1))
    n = int(regions.max()) + 1
    row_ptr, col_idx = oi.region_graph(regions, n)
    for u in range(n):
        assert col_idx[row_ptr[u]:row_ptr[u + 1]].tolist() == [v for v in (u - 1, u + 1) if 0 <= v < n]


@pytest.mark.parametrize("by,bx,size", [(3, 4, 5), (1, 6, 2), (4, 1, 3), (2, 2, 1)])
def test_block_grid_is_the_grid_graph(by, bx, size):
    rr, cc = np.meshgrid(np.arange(by * size), np.arange(bx * size), indexing="ij")
    regions = ((rr // size) * bx + cc // size).astype(np.int32)
    n = by * bx
    row_ptr, col_idx = oi.region_graph(regions, n)
    for i in range(by):
        for j in range(bx):
            u = i * bx + j
            want = sorted([a * bx + b for a, b in ((i - 1, j), (i + 1, j), (i, j - 1), (i, j + 1))
                           if 0 <= a < by and 0 <= b < bx])
            assert col_idx[row_ptr[u]:row_ptr[u + 1]].tolist() == want


def test_one_region_per_pixel_and_one_region():
    rng = np.random.default_rng(4)
    h, w = 6, 7
    pixels = rng.integers(0, 256, size=(h, w), dtype=np.uint8)
    regions = np.arange(h * w, dtype=np.int32).reshape(h, w)
    means = oi.region_means(regions, pixels, h * w)
    assert np.array_equal(means, pixels.ravel().astype(np.float64))
    row_ptr, _ = oi.region_graph(regions, h * w)
    assert row_ptr[-1] == 2 * (h * (w - 1) + (h - 1) * w)  # every pixel pair is an edge
    one = np.zeros((h, w), dtype=np.int32)
    row_ptr, col_idx = oi.region_graph(one, 1)
    assert row_ptr.tolist() == [0, 0] and col_idx.size == 0
    assert oi.region_means(one, pixels, 1)[0] == pixels.astype(np.int64).sum() / (h * w)
    # a region id with no pixel keeps mean 0 and no neighbours
    row_ptr, _ = oi.region_graph(one, 3)
    assert row_ptr.tolist() == [0, 0, 0, 0] and oi.region_means(one, pixels, 3)[1:].tolist() == [0.0, 0.0]


@pytest.mark.parametrize("seed,side,regions", [(5, 64, 120), (6, 100, 400)])
def test_agrees_with_the_input_generator(seed, side, regions):
    img, lab, _ = synth.image_slice(seed, side, regions)
    g = synth.image_graph(seed, side, regions)
    row_ptr, col_idx = oi.region_graph(lab, g.n)
    assert np.array_equal(row_ptr, g.row_ptr) and np.array_equal(col_idx, g.col_idx)
    assert np.allclose(oi.region_means(lab, img, g.n), g.y, rtol=0, atol=1e-12)


def test_paint_confusion_and_scores():
    regions = np.array([[0, 0, 1], [2, 1, 1], [5, 2, 0]], dtype=np.int32)
    labels = np.array([1, 0, 1], dtype=np.int32)
    painted = oi.labels_to_pixels(regions, labels, 3)
    assert painted.tolist() == [[1, 1, 0], [1, 0, 0], [255, 1, 1]]
    truth = np.array([[1, 0, 0], [1, 0, 1], [0, 1, 1]], dtype=np.uint8)
    c = oi.confusion(painted, truth, 2)  # the 255 pixel is not counted
    # pixels (seg, truth): (1,1) (1,0) (0,0) (1,1) (0,0) (0,1) (1,1) (1,1)
    assert c.tolist() == [[2, 1], [1, 4]]
    s = oi.scores(c, positive=1, void=0)
    assert s["precision"] == 4 / 5 and s["recall"] == 4 / 5 and s["accuracy"] == 6 / 8
    assert s["porosity"] == 3 / 8
    same = oi.scores(oi.confusion(truth, truth, 2))
    assert same["precision"] == same["recall"] == same["accuracy"] == 1.0


def test_volume_closed_forms():
    # one region per voxel of a 2 x 2 x 2 volume: the cube graph (degree 3)
    cube = np.arange(8, dtype=np.int32).reshape(2, 2, 2)
    row_ptr, col_idx = oi.region_graph(cube, 8)
    for u in range(8):
        assert col_idx[row_ptr[u]:row_ptr[u + 1]].tolist() == sorted(u ^ bit for bit in (1, 2, 4))
    # blocks of a 3-D grid: the 3-D grid graph
    bz, by, bx, size = 2, 3, 2, 3
    zz, yy, xx = np.meshgrid(np.arange(bz * size), np.arange(by * size), np.arange(bx * size), indexing="ij")
    regions = (((zz // size) * by + yy // size) * bx + xx // size).astype(np.int32)
    row_ptr, col_idx = oi.region_graph(regions, bz * by * bx)
    for k in range(bz):
        for i in range(by):
            for j in range(bx):
                u = (k * by + i) * bx + j
                want = sorted((a * by + b) * bx + c for a, b, c in ((k - 1, i, j), (k + 1, i, j), (k, i - 1, j),
                                                                    (k, i + 1, j), (k, i, j - 1), (k, i, j + 1))
                              if 0 <= a < bz and 0 <= b < by and 0 <= c < bx)
                assert col_idx[row_ptr[u]:row_ptr[u + 1]].tolist() == want
    # regions that run through every slice: the graph of one slice, means over all slices
    img, lab, _ = synth.image_slice(7, 64, 100)
    n = int(lab.max()) + 1
    vol = np.stack([lab] * 3)
    pix = np.stack([img, img // 2, img])
    ref_ptr, ref_col = oi.region_graph(lab, n)
    row_ptr, col_idx = oi.region_graph(vol, n)
    assert np.array_equal(row_ptr, ref_ptr) and np.array_equal(col_idx, ref_col)
    sums = np.zeros(n, np.int64)
    np.add.at(sums, lab.ravel(), 2 * img.ravel().astype(np.int64) + (img // 2).ravel())
    counts = np.bincount(lab.ravel(), minlength=n) * 3
    assert np.array_equal(oi.region_means(vol, pix, n), sums / counts)
