"""Exact k-nearest-neighbour oracle for graph construction.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Section 2.2 builds the
clustering graphs from the k nearest neighbours of each point in Euclidean
distance of its feature vector.  This is that definition written out: the
squared distance from every point to every other point in float64, self
excluded, and a stable sort (equal distances keep the lower index first).
"""

from __future__ import annotations

import numpy as np


def sq_distances(x: np.ndarray, rows=None) -> np.ndarray:
    """Squared Euclidean distances from the points `rows` (default: all) to
    all points, sum over coordinates of (x_ic - x_jc)^2, float64."""
    x = np.asarray(x, dtype=np.float64)
    q = x if rows is None else x[np.asarray(rows)]
    out = np.empty((q.shape[0], x.shape[0]))
    step = max(1, 20_000_000 // max(1, x.shape[0] * x.shape[1]))  # bounded temporaries
    for s in range(0, q.shape[0], step):
        diff = q[s:s + step, None, :] - x[None, :, :]
        out[s:s + step] = (diff * diff).sum(-1)
    return out


def knn(x: np.ndarray, k: int, rows=None):
    """(indices [m, k], squared distances [m, k]) of the k nearest other
    points of each query row, ascending, ties to the lower index."""
    x = np.asarray(x, dtype=np.float64)
    rows = np.arange(x.shape[0]) if rows is None else np.asarray(rows)
    d2 = sq_distances(x, rows)
    d2[np.arange(len(rows)), rows] = np.inf  # a point is not its own neighbour
    idx = np.argsort(d2, axis=1, kind="stable")[:, :k]
    return idx, np.take_along_axis(d2, idx, axis=1)


SCALE_FLOOR = 2.0 ** -256  # s_i of a point with scale_rank duplicates (distance 0)


def graph_from_knn(n: int, idx: np.ndarray, d2: np.ndarray, scale_rank: int = 7):
    """Union-symmetric kNN graph with local-scaling weights, from given kNN
    lists (indices [n, k] ascending by distance, squared distances [n, k]).

    Section 2.2 joins i and j when one is among the other's k nearest
    neighbours (N_c, symmetrised by union) and takes a Gaussian of the
    distance with the adaptive bandwidth of Zelnik-Manor and Perona:
        w_ij = exp(-|x_i - x_j|^2 / (s_i s_j)),  s_i = distance from i to its
        scale_rank-th neighbour (SCALE_FLOOR when that distance is 0).
    Edges whose weight is 0 in float64 are left out.  Returns CSR (row_ptr
    int64, col int32 ascending per row, w float64), written out with a dict
    per row."""
    idx = np.asarray(idx)
    d2 = np.asarray(d2, dtype=np.float64)
    s = np.sqrt(d2[:, scale_rank - 1])
    s = np.where(s > 0, s, SCALE_FLOOR)
    rows = [dict() for _ in range(n)]
    for i in range(n):
        for e in range(idx.shape[1]):
            j = int(idx[i, e])
            wv = float(np.exp(-d2[i, e] / (s[i] * s[j])))
            rows[i][j] = wv
            rows[j][i] = wv
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    cols, ws = [], []
    for i in range(n):
        for j in sorted(rows[i]):
            if rows[i][j] > 0.0:
                cols.append(j)
                ws.append(rows[i][j])
        row_ptr[i + 1] = len(cols)
    return row_ptr, np.asarray(cols, dtype=np.int32), np.asarray(ws)


def self_tuning_graph(x: np.ndarray, k: int, scale_rank: int = 7):
    """The whole recipe from the points: exact kNN in float64, then
    graph_from_knn."""
    idx, d2 = knn(x, k)
    return graph_from_knn(np.asarray(x).shape[0], idx, d2, scale_rank)
