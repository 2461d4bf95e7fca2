"""The five seeded benchmark workloads and the served request stream.

Each workload is a graph Ginzburg-Landau problem: a symmetric kNN graph, a
label mask, an initial field u^0 and the solver schedule.  Parameter values
that the workload description leaves open follow the paper: the image runs
use eps = 100, c = 11, eta = 100 (Section 5.1.1), the 784-dimensional
clustering run the paper's MNIST values eps = 100, c = 101, eta = 100
(Section 5.2), and the served stream eps = 100, c = 11, eta = 100 (the
paper's other clustering runs).  Workload i draws from numpy SeedSequence(i - 1),
spawned into independent streams for data, labels and u^0; served request j
uses SeedSequence(1000 + j).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

from .graphs import (Graph, gaussian_mixture, knn_bruteforce, window_knn,
                     self_tuning_graph, rectangles_image, textured_regions_image,
                     patch_features, random_labels, scribble_labels, initial_u, zorder)

CONFIG_NAMES = {
    1: "cluster2-n4096-k10",
    2: "image512-rect-k20",
    3: "cluster10-n70000-d784-k10",
    4: "image2048-texture4-k20",
}


@dataclass
class Problem:
    name: str
    graph: Graph
    K: int
    labels: np.ndarray          # int32 [n], -1 = unlabelled
    u0: np.ndarray              # float64 [n, K]
    truth: np.ndarray           # int32 [n] ground-truth class
    eps: float
    c: float
    eta: float
    precond: str                # damped_jacobi | perturbed_jacobi | richardson
    outer: int                  # DCA steps T
    sweeps: int                 # preconditioned sweeps m per DCA step
    store_w: str = "f32"
    store_u: str = "f32"
    delta0: float = 1e-6
    step_k: float = math.inf
    seed: int = 0
    order: np.ndarray | None = None   # int32 processing order of the rows, or None
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.graph.n


def _streams(seed: int):
    ss = np.random.SeedSequence(seed)
    return [np.random.default_rng(s) for s in ss.spawn(3)]


def _dev(device):
    return torch.device(device) if device is not None else torch.device("cpu")


def _mixture_problem(name, n, means, sigma, clip, k, frac, K, seed, device, **kw):
    r_data, r_lab, _ = _streams(seed)
    x, comp = gaussian_mixture(n, means, sigma, r_data, clip_nonneg=clip)
    xt = torch.from_numpy(x).to(_dev(device))
    nbr = knn_bruteforce(xt, k)
    g = self_tuning_graph(xt, nbr)
    del xt, nbr
    nclass = max(K, 2)
    labels = random_labels(comp, frac, nclass, r_lab)
    return Problem(name=name, graph=g, K=K, labels=labels, u0=initial_u(labels, K),
                   truth=comp, seed=seed, **kw)


def _image_problem(name, img, truth, k, frac, K, seed, r_lab, device, **kw):
    feat = torch.from_numpy(patch_features(img, 3)).to(_dev(device))
    h, w, f = feat.shape
    nbr = window_knn(feat, k, radius=7)
    g = self_tuning_graph(feat.view(h * w, f), nbr)
    del feat, nbr
    t = truth.reshape(-1).astype(np.int32)
    labels = random_labels(t, frac, max(K, 2), r_lab)
    return Problem(name=name, graph=g, K=K, labels=labels, u0=initial_u(labels, K),
                   truth=t, seed=seed, order=zorder(h, w), extra={"grid": (h, w)}, **kw)


def make_problem(cfg: int, device="cpu", small: bool = False) -> Problem:
    """Build workload `cfg` (1..4).  small=True shrinks N for CPU-side tests
    while keeping the recipe (same generator, same parameters)."""
    seed = cfg - 1
    if cfg == 1:
        means = np.zeros((2, 10))
        means[0, 0], means[1, 0] = 1.5, -1.5
        return _mixture_problem(CONFIG_NAMES[1], 4096, means, 1.0, False, 10, 0.05, 1,
                                seed, device, eps=1.0, c=3.0, eta=1000.0,
                                precond="damped_jacobi", outer=50, sweeps=4,
                                store_w="f32", store_u="f32")
    if cfg == 2:
        side = 64 if small else 512
        r_data, r_lab, _ = _streams(seed)
        lo, hi = (4, 20) if small else (32, 160)
        img, truth = rectangles_image(side, side, 6, r_data, side=(lo, hi), noise=0.1)
        name = CONFIG_NAMES[2] if not small else "image64-rect-k20"
        return _image_problem(name, img, truth, 20, 0.01, 1, seed, r_lab, device,
                              eps=100.0, c=11.0, eta=100.0, precond="richardson",
                              outer=4, sweeps=8, store_w="f32", store_u="f32")
    if cfg == 3:
        n = 3000 if small else 70000
        r_data, _, _ = _streams(seed)
        means = r_data.standard_normal((10, 784))
        # the mixture draws continue from the same data stream
        x, comp = gaussian_mixture(n, means, 0.8, r_data, clip_nonneg=True)
        _, r_lab, _ = _streams(seed)
        xt = torch.from_numpy(x).to(_dev(device))
        g = self_tuning_graph(xt, knn_bruteforce(xt, 10))
        del xt
        labels = random_labels(comp, 0.03, 10, r_lab)
        name = CONFIG_NAMES[3] if not small else "cluster10-n3000-d784-k10"
        # eps, c, eta: the paper's pDCA values for its MNIST clustering run
        return Problem(name=name, graph=g, K=10, labels=labels, u0=initial_u(labels, 10),
                       truth=comp, seed=seed, eps=100.0, c=101.0, eta=100.0,
                       precond="damped_jacobi", outer=20, sweeps=4,
                       store_w="bf16", store_u="bf16")
    if cfg == 4:
        return texture_problem(128 if small else 2048, device)
    raise ValueError(f"unknown workload {cfg}")


def texture_problem(side: int, device="cpu") -> Problem:
    """Workload 4's recipe on a side x side image (2048 for the workload
    itself): 4 textured Voronoi regions, noise 0.05, 3 x 3 RGB patches, 20-NN
    in the 15 x 15 window, K = 4, 0.5 % labels, 10 x 8 Richardson sweeps,
    bf16 weights and f16 field.  Other sides serve as larger or smaller
    instances of the same workload."""
    seed = 3
    r_data, r_lab, _ = _streams(seed)
    img, truth = textured_regions_image(side, side, 4, r_data, noise=0.05)
    name = CONFIG_NAMES[4] if side == 2048 else f"image{side}-texture4-k20"
    return _image_problem(name, img, truth, 20, 0.005, 4, seed, r_lab, device,
                          eps=100.0, c=11.0, eta=100.0, precond="richardson",
                          outer=10, sweeps=8, store_w="bf16", store_u="f16")


# --------------------------------------------------------------------------
# served stream
# --------------------------------------------------------------------------

@dataclass
class StreamItem:
    index: int
    n: int
    K: int
    knn_k: int
    arrival: float      # seconds after stream start, before rate scaling


def served_stream(count: int = 256, n_range=(1e4, 1e6), seed: int = 4):
    """Sizes, class counts and unit-rate Poisson arrival times of the stream.

    N is log-uniform in n_range, K uniform in {2..10}, kNN k uniform in
    {10..20}; inter-arrival gaps are Exp(1) (scale them by 1/rate).
    """
    rng = np.random.default_rng(seed)
    lo, hi = math.log(n_range[0]), math.log(n_range[1])
    ns = np.exp(rng.uniform(lo, hi, count)).astype(np.int64)
    ks = rng.integers(2, 11, count)
    kk = rng.integers(10, 21, count)
    gaps = rng.exponential(1.0, count)
    t = np.cumsum(gaps) - gaps[0]
    return [StreamItem(i, int(ns[i]), int(ks[i]), int(kk[i]), float(t[i]))
            for i in range(count)]


def served_problem(item: StreamItem, device="cpu", knn=None) -> Problem:
    """Request `item.index`: a K-component mixture in R^10 (means N(0, 9 I),
    unit covariance), self-tuning kNN graph, 2% labels, 20 x 4 damped Jacobi
    with eps = 100, c = 11, eta = 100, bf16 storage.

    `knn(x, k)` may supply the neighbour indices [n, k] (int64 tensor) of the
    float64 points x in place of the brute-force search here."""
    seed = 1000 + item.index
    r_data, r_lab, _ = _streams(seed)
    means = 3.0 * r_data.standard_normal((item.K, 10))
    x, comp = gaussian_mixture(item.n, means, 1.0, r_data)
    xt = torch.from_numpy(x).to(_dev(device))
    nbr = knn(xt, item.knn_k) if knn is not None else knn_bruteforce(xt, item.knn_k)
    g = self_tuning_graph(xt, nbr)
    del xt
    labels = random_labels(comp, 0.02, item.K, r_lab)
    return Problem(name=f"served-{item.index}", graph=g, K=item.K, labels=labels,
                   u0=initial_u(labels, item.K), truth=comp, seed=seed, eps=100.0, c=11.0,
                   eta=100.0, precond="damped_jacobi", outer=20, sweeps=4,
                   store_w="bf16", store_u="bf16")


# --------------------------------------------------------------------------
# the paper's own image graph: search window + patch similarity
# --------------------------------------------------------------------------

@dataclass
class WindowProblem:
    """A segmentation problem on the window graph of Section 2.2, built by the
    library from the image itself (no CSR)."""
    name: str
    image: np.ndarray           # float64 [h, w, 3], 8-bit colour scale
    rw: int                     # window radius: (2 rw + 1)^2 window
    rp: int                     # patch radius: (2 rp + 1)^2 patch
    sigma: float
    K: int
    labels: np.ndarray
    u0: np.ndarray
    truth: np.ndarray
    eps: float = 100.0
    c: float = 11.0
    eta: float = 100.0
    precond: str = "damped_jacobi"
    outer: int = 10
    sweeps: int = 4
    store_w: str = "bf16"
    store_u: str = "f32"
    delta0: float = 1e-6
    step_k: float = math.inf
    seed: int = 0

    @property
    def n(self) -> int:
        return self.image.shape[0] * self.image.shape[1]


def window_problem(h: int = 1024, w: int = 1024, rw: int = 12, rp: int = 2, seed: int = 5,
                   frac: float = 0.01, nrect: int = 6, noise: float = 3.0,
                   scribbles: bool = False, **kw) -> WindowProblem:
    """Binary segmentation on the paper's window graph: `nrect` rectangles of
    one colour over a background (colours uniform on the 8-bit scale [0, 255]^3,
    at least 0.3 * 255 apart), Gaussian noise of `noise` levels, a fraction
    `frac` of pixels labelled with the ground truth, sigma = log(h w) + 1 (the
    order the paper gives for images).  Defaults: a 1024 x 1024 image with the
    25 x 25 window and 5 x 5 patches and eps = 100, c = 11, eta = 100 and four
    sweeps per DCA step (the paper's preconditioner comparison).  scribbles:
    labels from synth.graphs.scribble_labels instead of a random fraction."""
    r_data, r_lab, _ = _streams(seed)
    lo, hi = max(6, min(h, w) // 16), max(8, min(h, w) // 3)
    img, truth = rectangles_image(h, w, nrect, r_data, side=(lo, hi), noise=noise / 255.0)
    img *= 255.0
    t = truth.reshape(-1).astype(np.int32)
    if scribbles:
        labels = scribble_labels(truth, r_lab)
    else:
        labels = random_labels(t, frac, 2, r_lab)
    return WindowProblem(name=f"window{h}x{w}-r{rw}-p{rp}" + ("-scribbles" if scribbles else ""),
                         image=img, rw=rw, rp=rp,
                         sigma=math.log(h * w) + 1.0, K=1, labels=labels,
                         u0=initial_u(labels, 1), truth=t, seed=seed, **kw)
