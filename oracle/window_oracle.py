"""The paper's image graph (Section 2.2), written out from its definition.

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's CPU
baseline, never by the library.  Pixel i at (y_i, x_i)
is joined to every pixel j of its search window, max(|x_i - x_j|,
|y_i - y_j|) <= r_w (the proximity term N_s with dist = r_w + 1), j != i,
with the weight

    w_ij = K(i, j) = exp(- sum_n alpha_n |C(p_i + n) - C(p_j + n)|^2 / sigma^2)

where n runs over the (2 r_p + 1)^2 offsets of the patch and C is the colour
vector.  Readings (the paper leaves them open): alpha_n = g(n_y) g(n_x) with
g(t) = exp(-t^2 / (2 r_p^2)) (the weight falls with the distance from the
patch centre), normalised to sum 1 so that the numerator is a weighted mean
of squared colour differences; pixels outside the image take the colour of
the nearest border pixel (edge replication); sigma is a parameter.  The pixel
itself is not its own neighbour (a full 15 x 15 window gives 224 neighbours).
"""

from __future__ import annotations

import math

import numpy as np


def patch_alpha(rp: int) -> np.ndarray:
    """alpha over the patch offsets, [(2 rp + 1), (2 rp + 1)], summing to 1."""
    t = np.arange(-rp, rp + 1, dtype=np.float64)
    g = np.exp(-t * t / (2.0 * rp * rp)) if rp > 0 else np.ones(1)
    return np.outer(g, g) / g.sum() ** 2


def patch_distance(img, yi, xi, yj, xj, rp, alpha=None):
    """sum_n alpha_n |C(p_i + n) - C(p_j + n)|^2 with edge replication, by
    explicit loops (one pair)."""
    h, w = img.shape[:2]
    alpha = patch_alpha(rp) if alpha is None else alpha
    s = 0.0
    for a in range(-rp, rp + 1):
        for b in range(-rp, rp + 1):
            ci = img[min(max(yi + a, 0), h - 1), min(max(xi + b, 0), w - 1)]
            cj = img[min(max(yj + a, 0), h - 1), min(max(xj + b, 0), w - 1)]
            dd = np.asarray(ci, dtype=np.float64) - np.asarray(cj, dtype=np.float64)
            s += alpha[a + rp, b + rp] * float(dd @ dd)
    return s


def window_graph(img: np.ndarray, rw: int, rp: int, sigma: float):
    """CSR (row_ptr int64, col int32, w float64) of the window graph of an
    h x w x C image, pixels numbered row-major, columns ascending."""
    img = np.asarray(img, dtype=np.float64)
    if img.ndim == 2:
        img = img[:, :, None]
    h, w, _ = img.shape
    alpha = patch_alpha(rp)
    pad = np.pad(img, ((rp, rp), (rp, rp), (0, 0)), mode="edge")
    # patch vectors of every pixel, weighted by sqrt(alpha)
    sa = np.sqrt(alpha)
    P = np.stack([pad[a:a + h, b:b + w, :] * sa[a, b] for a in range(2 * rp + 1)
                  for b in range(2 * rp + 1)], axis=2).reshape(h * w, -1)
    yy, xx = np.divmod(np.arange(h * w), w)
    rows, cols, ws = [], [], []
    for dy in range(-rw, rw + 1):
        for dx in range(-rw, rw + 1):
            if dy == 0 and dx == 0:
                continue
            y2, x2 = yy + dy, xx + dx
            ok = (y2 >= 0) & (y2 < h) & (x2 >= 0) & (x2 < w)
            i = np.flatnonzero(ok)
            j = y2[ok] * w + x2[ok]
            diff = P[i] - P[j]
            rows.append(i)
            cols.append(j)
            ws.append(np.exp(-(diff * diff).sum(1) / (sigma * sigma)))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    ws = np.concatenate(ws)
    order = np.lexsort((cols, rows))
    rows, cols, ws = rows[order], cols[order], ws[order]
    rp_ = np.zeros(h * w + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=h * w), out=rp_[1:])
    return rp_, cols.astype(np.int32), ws


def _patch_vectors(img: np.ndarray, rp: int) -> np.ndarray:
    """sqrt(alpha)-weighted patch vectors of every pixel, [h, w, (2rp+1)^2 C]."""
    h, w, _ = img.shape
    sa = np.sqrt(patch_alpha(rp))
    pad = np.pad(img, ((rp, rp), (rp, rp), (0, 0)), mode="edge")
    return np.concatenate([pad[a:a + h, b:b + w, :] * sa[a, b] for a in range(2 * rp + 1)
                           for b in range(2 * rp + 1)], axis=2)


def window_rows(img: np.ndarray, rw: int, rp: int, sigma: float, pixels):
    """Rows of the window graph for a few pixels of a large image, from the
    definition, without building the whole graph: for each pixel i (row-major
    index) returns (j ascending, w_ij, d_i, d_j)."""
    img = np.asarray(img, dtype=np.float64)
    if img.ndim == 2:
        img = img[:, :, None]
    h, w, _ = img.shape
    out = []
    for i in pixels:
        yi, xi = divmod(int(i), w)
        # every pixel within 2 rw of i (the neighbours' windows), patches from the full image
        y0, y1 = max(yi - 2 * rw, 0), min(yi + 2 * rw, h - 1)
        x0, x1 = max(xi - 2 * rw, 0), min(xi + 2 * rw, w - 1)
        ys0, ys1 = max(y0 - rp, 0), min(y1 + rp, h - 1)
        xs0, xs1 = max(x0 - rp, 0), min(x1 + rp, w - 1)
        # patches of the crop equal the full image's when the crop keeps rp rows
        # and columns beyond the box (or reaches the image border, replicated alike)
        P = _patch_vectors(img[ys0:ys1 + 1, xs0:xs1 + 1], rp)[y0 - ys0:y1 - ys0 + 1,
                                                              x0 - xs0:x1 - xs0 + 1]

        dyx = np.array([(dy, dx) for dy in range(-rw, rw + 1) for dx in range(-rw, rw + 1)
                        if dy or dx])

        def weights_of(yy, xx):
            """(neighbour ids, weights) of box pixel (yy, xx), ascending."""
            gy, gx = yy + y0 + dyx[:, 0], xx + x0 + dyx[:, 1]
            keep = (gy >= 0) & (gy < h) & (gx >= 0) & (gx < w)
            gy, gx = gy[keep], gx[keep]
            diff = P[yy, xx][None, :] - P[gy - y0, gx - x0]
            return gy * w + gx, np.exp(-(diff * diff).sum(1) / (sigma * sigma))

        js, wij = weights_of(yi - y0, xi - x0)
        di = float(wij.sum())
        dj = np.array([weights_of(j // w - y0, j % w - x0)[1].sum() for j in js])
        out.append((js, wij, di, dj))
    return out
