"""Seeded synthetic data and kNN graph construction (input tooling only).

Graph construction follows the paper's weight recipe for data clustering
(Section 2.2): a Gaussian similarity K(i,j) times a kNN proximity N_c(i,j),
with the Zelnik-Manor--Perona local scaling for the bandwidth.  Concretely
w_ij = exp(-||x_i - x_j||^2 / (s_i s_j)) with s_i the distance from x_i to its
7th nearest neighbour (self excluded).  The kNN relation is not symmetric, so
the edge set is symmetrised by union: (i,j) is an edge iff j is among the k
nearest neighbours of i or i among those of j.  Both orientations are stored;
the weight formula is already symmetric.

For images the candidate set of the kNN search is the 15x15 spatial window
around each pixel (the paper's default search window N_s, Section 2.2), so the
graph combines the paper's window proximity with the kNN selection.

All distances and weights are computed in float64.  torch is used only as an
array library here (CPU or GPU), never for the solver.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch


@dataclass
class Graph:
    """Symmetric weighted graph in CSR form (both orientations stored).

    row_ptr: int64 [n+1]; col: int32 [nnz], sorted within each row;
    weight: float64 [nnz], w_ij > 0, no self-loops.
    """

    n: int
    row_ptr: torch.Tensor
    col: torch.Tensor
    weight: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    def to(self, device) -> "Graph":
        return Graph(self.n, self.row_ptr.to(device), self.col.to(device),
                     self.weight.to(device))

    def numpy(self):
        return (self.row_ptr.cpu().numpy(), self.col.cpu().numpy(),
                self.weight.cpu().numpy())


# --------------------------------------------------------------------------
# point clouds and images
# --------------------------------------------------------------------------

def gaussian_mixture(n: int, means: np.ndarray, sigma: float,
                     rng: np.random.Generator, clip_nonneg: bool = False):
    """n points from an equal-weight isotropic Gaussian mixture.

    Component choice is iid uniform.  Returns (points float64 [n, dim],
    component int32 [n]).
    """
    means = np.asarray(means, dtype=np.float64)
    comp = rng.integers(0, means.shape[0], size=n).astype(np.int32)
    x = means[comp] + sigma * rng.standard_normal((n, means.shape[1]))
    if clip_nonneg:
        np.maximum(x, 0.0, out=x)
    return x, comp


def rectangles_image(h: int, w: int, nrect: int, rng: np.random.Generator,
                     side=(32, 160), noise=0.1):
    """Background plus `nrect` axis-aligned rectangles of one foreground colour.

    Colours are uniform in [0,1]^3, the foreground redrawn until it is at
    least 0.3 away from the background.  Gaussian noise is added, unclipped.
    Returns (image float64 [h, w, 3], truth int32 [h, w]; 1 inside a rectangle).
    """
    bg = rng.uniform(0.0, 1.0, 3)
    while True:
        fg = rng.uniform(0.0, 1.0, 3)
        if np.linalg.norm(fg - bg) >= 0.3:
            break
    truth = np.zeros((h, w), dtype=np.int32)
    for _ in range(nrect):
        rh = int(rng.integers(side[0], side[1] + 1))
        rw = int(rng.integers(side[0], side[1] + 1))
        rh, rw = min(rh, h), min(rw, w)
        y0 = int(rng.integers(0, h - rh + 1))
        x0 = int(rng.integers(0, w - rw + 1))
        truth[y0:y0 + rh, x0:x0 + rw] = 1
    img = np.where(truth[..., None] == 1, fg, bg).astype(np.float64)
    img += noise * rng.standard_normal(img.shape)
    return img, truth


def textured_regions_image(h: int, w: int, nregions: int,
                           rng: np.random.Generator, noise=0.05):
    """Voronoi regions of `nregions` seeded points, each with its own texture.

    Per region and channel the value is 0.5 + 0.4 sin(2 pi (fx x + fy y) + phi)
    with fx, fy uniform in [1/64, 1/8] cycles per pixel and phi uniform in
    [0, 2 pi), plus Gaussian noise.  Returns (image [h, w, 3], truth [h, w]).
    """
    seeds = np.stack([rng.uniform(0, h, nregions), rng.uniform(0, w, nregions)], 1)
    fx = rng.uniform(1 / 64, 1 / 8, (nregions, 3))
    fy = rng.uniform(1 / 64, 1 / 8, (nregions, 3))
    ph = rng.uniform(0, 2 * math.pi, (nregions, 3))
    yy, xx = np.meshgrid(np.arange(h, dtype=np.float64),
                         np.arange(w, dtype=np.float64), indexing="ij")
    d2 = (yy[..., None] - seeds[:, 0]) ** 2 + (xx[..., None] - seeds[:, 1]) ** 2
    truth = np.argmin(d2, axis=-1).astype(np.int32)
    del d2
    img = np.empty((h, w, 3), dtype=np.float64)
    for ch in range(3):
        arg = 2 * math.pi * (fx[truth, ch] * xx + fy[truth, ch] * yy) + ph[truth, ch]
        img[..., ch] = 0.5 + 0.4 * np.sin(arg)
    img += noise * rng.standard_normal(img.shape)
    return img, truth


def zorder(h: int, w: int) -> np.ndarray:
    """Z-order (Morton) visit order of an h x w pixel grid, as row-major pixel
    ids: position p of the returned int32 array holds the pixel visited p-th.
    Any aligned 4^j-long run of positions covers a 2^j x 2^j square when h and
    w are powers of two."""
    yy, xx = np.meshgrid(np.arange(h, dtype=np.int64), np.arange(w, dtype=np.int64),
                         indexing="ij")
    code = np.zeros((h, w), dtype=np.int64)
    for bit in range(32):
        code |= ((xx >> bit) & 1) << (2 * bit)
        code |= ((yy >> bit) & 1) << (2 * bit + 1)
    return np.argsort(code.reshape(-1), kind="stable").astype(np.int32)


def patch_features(img: np.ndarray, size: int = 3) -> np.ndarray:
    """Stack the size x size RGB patch around each pixel (edge-replicate pad).

    Returns float64 [h, w, size*size*3] with every patch entry weighted 1.
    """
    r = size // 2
    pad = np.pad(img, ((r, r), (r, r), (0, 0)), mode="edge")
    h, w = img.shape[:2]
    parts = [pad[dy:dy + h, dx:dx + w] for dy in range(size) for dx in range(size)]
    return np.concatenate(parts, axis=-1)


# --------------------------------------------------------------------------
# kNN search
# --------------------------------------------------------------------------

def _exact_d2(x: torch.Tensor, src: torch.Tensor, dst: torch.Tensor,
              chunk: int = 1 << 22) -> torch.Tensor:
    """sum_f (x[src,f] - x[dst,f])^2 in float64, symmetric bit for bit."""
    out = torch.empty(src.numel(), dtype=torch.float64, device=x.device)
    for s in range(0, src.numel(), chunk):
        e = min(src.numel(), s + chunk)
        diff = x[src[s:e]] - x[dst[s:e]]
        out[s:e] = (diff * diff).sum(1)
    return out


def knn_bruteforce(x: torch.Tensor, k: int, chunk: int = 2048,
                   work_dtype=torch.float64) -> torch.Tensor:
    """Indices [n, k] of the k nearest neighbours of every row (self excluded).

    Candidate ranking uses ||a||^2 + ||b||^2 - 2 a.b in `work_dtype`; the
    caller recomputes exact distances for the chosen edges.
    """
    n = x.shape[0]
    xw = x.to(work_dtype)
    sq = (xw * xw).sum(1)
    out = torch.empty((n, k), dtype=torch.int64, device=x.device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        d2 = sq[s:e, None] + sq[None, :] - 2.0 * (xw[s:e] @ xw.T)
        ar = torch.arange(e - s, device=x.device)
        d2[ar, ar + s] = float("inf")
        out[s:e] = torch.topk(d2, k, dim=1, largest=False, sorted=True).indices
        del d2
    return out


def window_knn(feat: torch.Tensor, k: int, radius: int = 7) -> torch.Tensor:
    """kNN restricted to the (2 radius + 1)^2 spatial window of each pixel.

    feat: [h, w, f] float64.  Returns neighbour indices [h*w, k] (row-major
    pixel numbering).  Out-of-image candidates are excluded.
    """
    h, w, _ = feat.shape
    dev = feat.device
    offs = [(dy, dx) for dy in range(-radius, radius + 1)
            for dx in range(-radius, radius + 1) if (dy, dx) != (0, 0)]
    dist = torch.full((h, w, len(offs)), float("inf"), dtype=torch.float64, device=dev)
    for o, (dy, dx) in enumerate(offs):
        y0, y1 = max(0, -dy), min(h, h - dy)
        x0, x1 = max(0, -dx), min(w, w - dx)
        if y0 >= y1 or x0 >= x1:
            continue
        diff = feat[y0:y1, x0:x1] - feat[y0 + dy:y1 + dy, x0 + dx:x1 + dx]
        dist[y0:y1, x0:x1, o] = (diff * diff).sum(-1)
    sel = torch.topk(dist.view(h * w, -1), k, dim=1, largest=False, sorted=True).indices
    del dist
    off_lin = torch.tensor([dy * w + dx for dy, dx in offs], dtype=torch.int64, device=dev)
    return torch.arange(h * w, device=dev, dtype=torch.int64)[:, None] + off_lin[sel]


def self_tuning_graph(x: torch.Tensor, nbr: torch.Tensor, scale_rank: int = 7) -> Graph:
    """Union-symmetrised kNN graph with self-tuning Gaussian weights.

    x: [n, f] float64 features; nbr: [n, k] neighbour indices sorted by
    distance.  s_i = distance to the `scale_rank`-th neighbour.
    """
    n, k = nbr.shape
    dev = x.device
    src = torch.arange(n, device=dev, dtype=torch.int64).repeat_interleave(k)
    dst = nbr.reshape(-1)
    d2 = _exact_d2(x, src, dst)
    d2_sorted = d2.view(n, k)
    s = torch.sqrt(d2_sorted[:, scale_rank - 1])
    s = torch.where(s > 0, s, torch.full_like(s, torch.finfo(torch.float64).tiny ** 0.25))
    w = torch.exp(-d2 / (s[src] * s[dst]))
    rows = torch.cat([src, dst])
    cols = torch.cat([dst, src])
    ww = torch.cat([w, w])
    del src, dst, d2, w
    key = rows * n + cols
    del rows, cols
    ukey, inv = torch.unique(key, sorted=True, return_inverse=True)
    del key
    uw = torch.empty(ukey.numel(), dtype=torch.float64, device=dev)
    uw[inv] = ww
    del inv, ww
    keep = uw > 0
    if not bool(keep.all()):
        ukey, uw = ukey[keep], uw[keep]
    r = ukey // n
    c = (ukey - r * n).to(torch.int32)
    counts = torch.bincount(r, minlength=n)
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    row_ptr[1:] = torch.cumsum(counts, 0)
    if int(counts.min()) == 0:
        raise ValueError("graph has an isolated vertex")
    return Graph(n, row_ptr, c.contiguous(), uw.contiguous())


# --------------------------------------------------------------------------
# labels and initial field
# --------------------------------------------------------------------------

def random_labels(truth: np.ndarray, frac: float, nclass: int,
                  rng: np.random.Generator) -> np.ndarray:
    """Reveal round(frac * n) ground-truth labels, at least one per class.

    Returns int32 [n] with -1 for unlabelled points.
    """
    n = truth.size
    nlab = max(int(round(frac * n)), nclass)
    chosen = []
    for cls in range(nclass):
        members = np.flatnonzero(truth == cls)
        if members.size:
            chosen.append(int(rng.choice(members)))
    rest = np.setdiff1d(np.arange(n), np.asarray(chosen, dtype=np.int64))
    extra = rng.choice(rest, size=nlab - len(chosen), replace=False)
    idx = np.concatenate([np.asarray(chosen, dtype=np.int64), extra])
    lab = np.full(n, -1, dtype=np.int32)
    lab[idx] = truth.reshape(-1)[idx]
    return lab


def scribble_labels(truth: np.ndarray, rng: np.random.Generator, width: int = 3,
                    frac_len: float = 0.25, background_strokes: int = 4) -> np.ndarray:
    """Scribble-style labels on an image's ground truth [h, w] (the paper's
    segmentation inputs mark each object with a few strokes): through the
    centre row of every connected region of class 1, a horizontal stroke
    `width` pixels tall over `frac_len` of the region's bounding-box width; and
    `background_strokes` strokes of the same shape on class-0 pixels at seeded
    random places.  Returns int32 [h * w], -1 unlabelled."""
    from scipy import ndimage
    h, w = truth.shape
    lab = np.full((h, w), -1, dtype=np.int32)
    comps, ncomp = ndimage.label(truth == 1)
    for c in range(1, ncomp + 1):
        ys, xs = np.nonzero(comps == c)
        yc = int(round(ys.mean()))
        x0, x1 = xs.min(), xs.max()
        half = max(1, int(frac_len * (x1 - x0 + 1)) // 2)
        xc = (x0 + x1) // 2
        for y in range(yc - width // 2, yc + width // 2 + 1):
            for x in range(xc - half, xc + half + 1):
                if 0 <= y < h and 0 <= x < w and comps[y, x] == c:
                    lab[y, x] = 1
    bg = truth == 0
    length = max(8, int(frac_len * w / 4))
    placed = 0
    while placed < background_strokes:
        y = int(rng.integers(width, h - width))
        x = int(rng.integers(0, max(1, w - length)))
        box = bg[y - width // 2:y + width // 2 + 1, x:x + length]
        if box.size and box.all():
            lab[y - width // 2:y + width // 2 + 1, x:x + length] = 0
            placed += 1
    return lab.reshape(-1)


def initial_u(labels: np.ndarray, K: int, mode: str = "labels",
              rng: np.random.Generator | None = None) -> np.ndarray:
    """Initial label field u^0 [n, K] float64.

    mode "labels": +1 / -1 one-vs-rest code on labelled rows (K == 1: class 1
    -> +1, class 0 -> -1), 0 on unlabelled rows.  mode "uniform": iid
    uniform[-1, 1] from `rng`.
    """
    n = labels.size
    if mode == "uniform":
        return rng.uniform(-1.0, 1.0, (n, K))
    u = np.zeros((n, K), dtype=np.float64)
    lab = labels >= 0
    if K == 1:
        u[lab, 0] = np.where(labels[lab] == 1, 1.0, -1.0)
    else:
        u[lab, :] = -1.0
        u[np.flatnonzero(lab), labels[lab]] = 1.0
    return u


def tiny_graph(n: int, p: float, rng: np.random.Generator,
               integer_weights: bool = False) -> Graph:
    """Random connected symmetric graph for small tests (a ring plus extras).

    Weights are uniform in (0.1, 1] or, with integer_weights, in {1, 2, 3}.
    """
    a = np.zeros((n, n))
    for i in range(n):
        j = (i + 1) % n
        if i != j:
            a[i, j] = a[j, i] = 1
    extra = rng.uniform(size=(n, n)) < p
    extra = np.triu(extra, 1)
    a = np.maximum(a, extra + extra.T)
    np.fill_diagonal(a, 0)
    if integer_weights:
        wv = rng.integers(1, 4, size=(n, n)).astype(np.float64)
    else:
        wv = rng.uniform(0.1, 1.0, size=(n, n))
    wv = np.triu(wv, 1)
    wv = wv + wv.T
    wmat = a * wv
    return dense_to_graph(wmat)


def dense_to_graph(wmat: np.ndarray) -> Graph:
    """CSR of a dense symmetric weight matrix (zero diagonal)."""
    n = wmat.shape[0]
    rows, cols = np.nonzero(wmat)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    return Graph(n, torch.from_numpy(row_ptr), torch.from_numpy(cols.astype(np.int32)),
                 torch.from_numpy(wmat[rows, cols].astype(np.float64)))
