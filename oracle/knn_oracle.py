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
