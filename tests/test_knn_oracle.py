"""Pins of the kNN oracle: closed-form neighbour lists on a line and a
lattice (with exact ties), and agreement with SciPy's k-d tree."""

import math

import numpy as np
import pytest

from oracle import knn_oracle
from oracle import knn_oracle as ko


def test_line_closed_form():
    # points 0, 1, ..., n-1 on a line: neighbours alternate left/right, the
    # left one first on ties (lower index)
    n, k = 12, 4
    idx, d2 = knn_oracle.knn(np.arange(n, dtype=float)[:, None], k)
    for i in range(n):
        cand = sorted((abs(i - j), j) for j in range(n) if j != i)[:k]
        assert list(idx[i]) == [j for _, j in cand]
        assert np.array_equal(d2[i], [float(dd * dd) for dd, _ in cand])
    assert list(idx[5]) == [4, 6, 3, 7]


def test_lattice_ties():
    h, w = 6, 7
    yy, xx = np.mgrid[0:h, 0:w]
    pts = np.stack([yy.ravel(), xx.ravel()], 1).astype(float)
    idx, d2 = knn_oracle.knn(pts, 8)
    i = 2 * w + 3  # interior point
    # 4 edge neighbours (d2 = 1) in index order, then 4 diagonals (d2 = 2)
    assert list(idx[i]) == [i - w, i - 1, i + 1, i + w, i - w - 1, i - w + 1, i + w - 1, i + w + 1]
    assert list(d2[i]) == [1, 1, 1, 1, 2, 2, 2, 2]
    # corner: two at 1, one at 2, then the two at 4
    assert list(idx[0][:5]) == [1, w, w + 1, 2, 2 * w]


def test_matches_kdtree():
    spatial = pytest.importorskip("scipy.spatial")
    rng = np.random.default_rng(3)
    x = rng.standard_normal((700, 5))
    idx, d2 = knn_oracle.knn(x, 9)
    dd, ii = spatial.cKDTree(x).query(x, 10)
    assert np.array_equal(ii[:, 1:], idx)
    assert np.allclose(dd[:, 1:] ** 2, d2, rtol=1e-12, atol=0)


def test_rows_subset_and_self_excluded():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((300, 3))
    full_i, full_d = knn_oracle.knn(x, 5)
    rows = [0, 17, 299]
    sub_i, sub_d = knn_oracle.knn(x, 5, rows=rows)
    assert np.array_equal(full_i[rows], sub_i) and np.array_equal(full_d[rows], sub_d)
    assert not np.any(full_i == np.arange(300)[:, None])


def test_graph_from_knn_line_by_hand():
    """Points 0, 1, 3, 7 on a line, k = 2, bandwidth from the nearest
    neighbour: lists, scales, union and weights worked out by hand."""
    x = np.array([[0.0], [1.0], [3.0], [7.0]])
    idx, d2 = ko.knn(x, 2)
    assert idx.tolist() == [[1, 2], [0, 2], [1, 0], [2, 1]]
    rp, col, w = ko.graph_from_knn(4, idx, d2, scale_rank=1)
    # s = (1, 1, 2, 4)
    want = {(0, 1): math.exp(-1.0), (0, 2): math.exp(-9 / 2), (1, 2): math.exp(-4 / 2),
            (2, 3): math.exp(-16 / 8), (1, 3): math.exp(-36 / 4)}
    assert rp.tolist() == [0, 2, 5, 8, 10]
    assert col.tolist() == [1, 2, 0, 2, 3, 0, 1, 3, 1, 2]
    for i in range(4):
        for p in range(rp[i], rp[i + 1]):
            j = int(col[p])
            assert w[p] == pytest.approx(want[(min(i, j), max(i, j))], rel=1e-15)


def test_graph_from_knn_invariants():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((300, 5))
    idx, d2 = ko.knn(x, 8)
    rp, col, w = ko.graph_from_knn(300, idx, d2, scale_rank=4)
    W = np.zeros((300, 300))
    for i in range(300):
        W[i, col[rp[i]:rp[i + 1]]] = w[rp[i]:rp[i + 1]]
    np.testing.assert_array_equal(W, W.T)          # symmetric
    assert np.all(np.diag(W) == 0)                  # no self-loops
    assert np.all((W == 0) | ((W > 0) & (W <= 1)))  # weights in (0, 1]
    # union: every kNN edge is present, and every edge comes from a kNN list
    E = W > 0
    K = np.zeros_like(E)
    K[np.repeat(np.arange(300), 8), idx.ravel()] = True
    assert np.array_equal(E, K | K.T)
    # the bandwidth: the weight of i's scale_rank-th neighbour j is exp(-s_i / s_j)
    s = np.sqrt(d2[:, 3])
    for i in range(0, 300, 37):
        j = idx[i, 3]
        assert W[i, j] == pytest.approx(math.exp(-s[i] / s[j]), rel=1e-13)


def test_graph_from_knn_duplicates_and_underflow():
    # four identical points: their scales are 0 (floored), mutual weights exp(0) = 1;
    # a far point keeps only edges whose weight does not underflow
    x = np.array([[0.0], [0.0], [0.0], [0.0], [1e3]])
    idx, d2 = ko.knn(x, 2)
    rp, col, w = ko.graph_from_knn(5, idx, d2, scale_rank=1)
    assert np.all(w[:rp[4]] == 1.0)
    assert rp[5] - rp[4] == 0  # the far point's weights underflow: isolated
