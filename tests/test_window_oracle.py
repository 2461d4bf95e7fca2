"""Pins of the window-graph oracle (Section 2.2's image graph): neighbour
counts of the window, the constant image, one weight by explicit loops,
symmetry, and the Gaussian patch weights."""

import math

import numpy as np
import pytest

from oracle import window_oracle as wo


def test_constant_image_counts():
    h, w, rw = 9, 11, 3
    rp_, col, ww = wo.window_graph(np.full((h, w, 3), 0.4), rw, 2, 0.5)
    deg = np.diff(rp_)
    # neighbours: (min(y+rw, h-1) - max(y-rw, 0) + 1) * (same in x) - 1
    for y in range(h):
        for x in range(w):
            ny = min(y + rw, h - 1) - max(y - rw, 0) + 1
            nx = min(x + rw, w - 1) - max(x - rw, 0) + 1
            assert deg[y * w + x] == ny * nx - 1
    assert np.all(ww == 1.0)          # equal patches: K = exp(0) = 1
    assert deg.max() == (2 * rw + 1) ** 2 - 1


def test_one_weight_by_loops_and_symmetry():
    rng = np.random.default_rng(2)
    img = rng.uniform(0, 1, (10, 12, 3))
    rw, rpatch, sigma = 2, 1, 0.7
    rp_, col, ww = wo.window_graph(img, rw, rpatch, sigma)
    W = np.zeros((120, 120))
    for i in range(120):
        W[i, col[rp_[i]:rp_[i + 1]]] = ww[rp_[i]:rp_[i + 1]]
    np.testing.assert_array_equal(W, W.T)
    for (yi, xi, yj, xj) in [(0, 0, 1, 2), (5, 6, 3, 4), (9, 11, 9, 9), (4, 0, 6, 1)]:
        want = math.exp(-wo.patch_distance(img, yi, xi, yj, xj, rpatch) / sigma ** 2)
        assert W[yi * 12 + xi, yj * 12 + xj] == pytest.approx(want, rel=1e-13)
    # outside the window or self: no edge
    assert W[0, 3] == 0.0 and W[0, 0] == 0.0


def test_patch_alpha_gaussian():
    a = wo.patch_alpha(2)
    assert a.sum() == pytest.approx(1.0, rel=1e-15)
    assert a[2, 3] / a[2, 2] == pytest.approx(math.exp(-1 / 8))
    assert a[0, 0] / a[2, 2] == pytest.approx(math.exp(-8 / 8))
    np.testing.assert_allclose(a, a.T)
    assert wo.patch_alpha(0).tolist() == [[1.0]]


def test_step_edge_closed_form():
    """Grey image, 0 for x <= 4 and 1 for x >= 5, patch radius 1: the pair
    (y, 4)-(y, 5) differs in the centre column of the patch only, so its
    distance is the weight of that column, g(0) / (g(-1) + g(0) + g(1)), with
    g(t) = exp(-t^2 / 2); a pair two columns deep on one side has distance 0;
    the pair (y, 3)-(y, 6) differs in all three columns (distance 1)."""
    img = np.zeros((6, 10))
    img[:, 5:] = 1.0
    sigma = 0.8
    rp_, col, ww = wo.window_graph(img, 3, 1, sigma)

    def weight(i, j):
        row = slice(rp_[i], rp_[i + 1])
        k = np.flatnonzero(col[row] == j)
        assert k.size == 1
        return ww[row][k[0]]

    frac = 1.0 / (1.0 + 2.0 * math.exp(-0.5))
    for y in range(6):
        assert weight(y * 10 + 4, y * 10 + 5) == pytest.approx(math.exp(-frac / sigma ** 2), rel=1e-14)
        assert weight(y * 10 + 1, y * 10 + 2) == 1.0
        assert weight(y * 10 + 3, y * 10 + 6) == pytest.approx(math.exp(-1 / sigma ** 2), rel=1e-14)
    # edge replication: the patch of (0, 4) reaches row -1, a copy of row 0,
    # so the vertical pair (0, 4)-(1, 4) on a vertical edge still has distance 0
    assert weight(4, 14) == 1.0


def test_one_pixel_wide_and_counts():
    # a 1-pixel-wide image is a path-like window graph: pixel y sees rows y +- rw
    rp_, col, ww = wo.window_graph(np.arange(7.0).reshape(7, 1), 2, 0, 1.0)
    assert np.diff(rp_).tolist() == [2, 3, 4, 4, 4, 3, 2]
    # patch radius 0: the weight is exp(-|C_i - C_j|^2 / sigma^2)
    assert ww[rp_[0]:rp_[1]].tolist() == pytest.approx([math.exp(-1.0), math.exp(-4.0)], rel=1e-15)


def test_window_rows_match_full_graph():
    """The per-pixel rows (used at sizes where the full graph is too large)
    agree with the whole graph, including the image border and the crop edge."""
    rng = np.random.default_rng(8)
    img = rng.uniform(0, 1, (17, 23, 3))
    rw, rpatch, sigma = 3, 2, 0.6
    rp_, col, ww = wo.window_graph(img, rw, rpatch, sigma)
    d = np.add.reduceat(ww, rp_[:-1])
    for i, (js, wij, di, dj) in zip([0, 5, 200, 23 * 8 + 11, 390],
                                    wo.window_rows(img, rw, rpatch, sigma, [0, 5, 200, 195, 390])):
        assert js.tolist() == col[rp_[i]:rp_[i + 1]].tolist()
        np.testing.assert_allclose(wij, ww[rp_[i]:rp_[i + 1]], rtol=1e-13)
        assert di == pytest.approx(d[i], rel=1e-13)
        np.testing.assert_allclose(dj, d[js], rtol=1e-13)


@pytest.mark.parametrize("h,w,rw,rp", [(13, 70, 3, 2), (40, 37, 5, 1), (9, 20, 4, 0), (1, 30, 3, 2),
                                        (30, 1, 2, 1)])
def test_c_window_graph_matches_definition(h, w, rw, rp):
    # the plain C window graph (used at 512 x 512 and above) against the
    # numpy one written from the definition: same structure, weights to rounding
    from oracle import c_oracle
    img = np.random.default_rng(h * 1000 + w).uniform(0.0, 255.0, (h, w, 3))
    a = wo.window_graph(img, rw, rp, 40.0)
    b = c_oracle.window_graph(img, rw, rp, 40.0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.abs(a[2] - b[2]).max() <= 1e-13 * a[2].max()
