"""Pins of the kNN oracle: closed-form neighbour lists on a line and a
lattice (with exact ties), and agreement with SciPy's k-d tree."""

import numpy as np
import pytest

from oracle import knn_oracle


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
