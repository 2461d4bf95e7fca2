"""GPU parity of the grid layout: a sparse graph on the pixels of an image
whose edges stay within the 15 x 15 window, stored with one-byte
window-relative columns (the kNN image graphs of the benchmark), against the
float64 oracle.  Ragged images cover tiles cut by the right and bottom edges.
"""

import numpy as np
import pytest
import torch

import paper_2303_14495_amd as gl
from oracle import c_oracle, gl_oracle
from synth.graphs import (patch_features, rectangles_image, self_tuning_graph, window_knn)
from tests.gpu_helpers import DEV, label_agreement, make_operator, power_x0, problem, say

pytestmark = pytest.mark.gpu

DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}
_G = {}


class _Img:
    """A kNN-in-window image graph of a ragged size (input tooling of synth/)."""

    def __init__(self, h, w, k=20, seed=3):
        rng = np.random.default_rng(seed)
        img, truth = rectangles_image(h, w, 4, rng, side=(4, 20), noise=0.1)
        feat = torch.from_numpy(patch_features(img, 3))
        nbr = window_knn(feat, k, radius=7)
        self.graph = self_tuning_graph(feat.view(h * w, -1), nbr, scale_rank=min(7, k))
        self.n = h * w
        self.extra = {"grid": (h, w)}
        self.truth = truth.reshape(-1)
        self.name = f"img{h}x{w}"


def _img(h, w):
    if (h, w) not in _G:
        # two-pixel-wide images: an edge pixel has 15 window candidates
        _G[(h, w)] = _Img(h, w, k=20 if min(h, w) >= 4 else 10)
    return _G[(h, w)]


SHAPES = [(37, 70), (8, 64), (13, 200), (2, 150), (150, 2)]


@pytest.mark.parametrize("h,w", SHAPES)
@pytest.mark.parametrize("store", [("f64", "f64"), ("f32", "f32"), ("bf16", "f32"), ("f16", "f16")])
@pytest.mark.parametrize("K", [1, 4])
def test_laplacian_ragged(h, w, store, K):
    p = _img(h, w)
    store_w, store_u = store
    say(f"grid laplacian {h}x{w} store={store} K={K}")
    op = make_operator(p, store_w, layout="grid")
    info = op.info()
    assert info["layout"] == "grid"
    rng = np.random.default_rng(h * w + K)
    X = torch.from_numpy(rng.uniform(-1, 1, (p.n, K))).to(DEV, DT[store_u]).contiguous()
    Y = op.laplacian_apply(X).to(torch.float64).cpu().numpy()
    rp, col, ww = p.graph.numpy()
    ref = gl_oracle.laplacian_apply(p.n, rp, col, ww, X.to(torch.float64).cpu().numpy())
    tol = {("f64", "f64"): 1e-13, ("f32", "f32"): 2e-6, ("bf16", "f32"): 1.5e-2,
           ("f16", "f16"): 3e-3}[store]
    err = np.abs(Y - ref).max()
    say(f"  max err {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("h,w", [(37, 70), (13, 200)])
@pytest.mark.parametrize("store,K", [(("f32", "f32"), 16), (("f64", "f64"), 8), (("f16", "f16"), 16),
                                     (("f32", "f32"), 9)])
def test_laplacian_wide_fields(h, w, store, K):
    # staged tiles above 64 KB (f32 K = 16: 110 KB, f64 K = 8, f32 K = 9) take
    # the 32-bit offset decode; f16 K = 16 (55 KB) the packed one
    p = _img(h, w)
    store_w, store_u = store
    say(f"grid laplacian wide {h}x{w} store={store} K={K}")
    op = make_operator(p, store_w, layout="grid")
    rng = np.random.default_rng(h + w + K)
    X = torch.from_numpy(rng.uniform(-1, 1, (p.n, K))).to(DEV, DT[store_u]).contiguous()
    Y = op.laplacian_apply(X).to(torch.float64).cpu().numpy()
    rp, col, ww = p.graph.numpy()
    ref = gl_oracle.laplacian_apply(p.n, rp, col, ww, X.to(torch.float64).cpu().numpy())
    tol = {"f64": 1e-13, "f32": 2e-6, "f16": 3e-3}[store_u]
    err = np.abs(Y - ref).max()
    say(f"  max err {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("k", [4, 30])
@pytest.mark.parametrize("K", [1, 4])
def test_dense_chunk_rounds(k, K):
    # every pixel's first min(smallest chunk count, 4) chunks are stored by
    # pixel: k = 4 leaves one such round (degrees from 4), k = 30 the most, four
    h, w = 37, 70
    key = (h, w, k)
    if key not in _G:
        _G[key] = _Img(h, w, k=k, seed=7)
    p = _G[key]
    rp, col, ww = p.graph.numpy()
    deg = np.diff(rp)
    rounds = min(int((deg.min() + 7) // 8), 4)
    assert rounds == (1 if k == 4 else 4)
    op = make_operator(p, "f32", layout="grid")
    rng = np.random.default_rng(k + K)
    X = torch.from_numpy(rng.uniform(-1, 1, (p.n, K))).to(DEV, torch.float32).contiguous()
    Y = op.laplacian_apply(X).to(torch.float64).cpu().numpy()
    ref = gl_oracle.laplacian_apply(p.n, rp, col, ww, X.to(torch.float64).cpu().numpy())
    err = np.abs(Y - ref).max()
    say(f"grid dense rounds k={k} K={K}: max err {err:.3e}")
    assert err <= 2e-6


@pytest.mark.parametrize("store", [("f64", "f64"), ("f32", "f32"), ("bf16", "f16")])
def test_unnormalized_laplacian(store):
    p = _img(37, 70)
    store_w, store_u = store
    op = make_operator(p, store_w, layout="grid", laplacian="unnormalized")
    X = torch.from_numpy(np.random.default_rng(5).uniform(-1, 1, (p.n, 3))).to(DEV, DT[store_u])
    Y = op.laplacian_apply(X).to(torch.float64).cpu().numpy()
    rp, col, ww = p.graph.numpy()
    ref = gl_oracle.laplacian_apply(p.n, rp, col, ww, X.to(torch.float64).cpu().numpy(),
                                    laplacian="unnormalized")
    dmax = float(gl_oracle.degrees(p.n, rp, col, ww).max())
    tol = {"f64": 1e-13, "f32": 2e-6}.get(store_u, 3e-2) * max(1.0, dmax)
    assert np.abs(Y - ref).max() <= tol


def test_power_and_eigenpair_vs_oracle():
    p = _img(37, 70)
    rp, col, ww = p.graph.numpy()
    x0 = power_x0(p.n, 7)
    rq_o, _ = c_oracle.power_max_eig(p.n, rp, col, ww, x0, 150)
    op = make_operator(p, "f32", layout="grid")
    rq, lam = op.power_max_eig(torch.from_numpy(x0).to(DEV, torch.float32), 150)
    say(f"grid power: rq {rq:.6f} oracle {rq_o:.6f}")
    assert abs(rq - rq_o) <= 1e-4 * rq_o
    lam_o, _ = gl_oracle.second_eigenpair(p.n, rp, col, ww)
    l2, v, res, _ = op.second_eigenpair(torch.from_numpy(x0).to(DEV, torch.float32), krylov=128,
                                        max_restarts=40, tol=1e-5)
    say(f"grid lambda2 {l2:.6e} oracle {lam_o:.6e} residual {res:.1e}")
    assert res <= 1e-5
    assert l2 == pytest.approx(lam_o, rel=1e-3, abs=1e-6)


@pytest.mark.parametrize("store,tol", [(("f64", "f64"), 1e-10), (("f32", "f32"), 1e-5),
                                       (("bf16", "f16"), 2e-2)])
@pytest.mark.parametrize("K", [1, 4])
def test_solve_ragged(store, tol, K):
    p = _img(37, 70)
    rp, col, ww = p.graph.numpy()
    rng = np.random.default_rng(11)
    lab = np.where(rng.uniform(size=p.n) < 0.05, p.truth % max(K, 2), -1).astype(np.int32)
    u0 = np.zeros((p.n, K))
    if K == 1:
        u0[lab >= 0, 0] = np.where(lab[lab >= 0] == 1, 1.0, -1.0)
    else:
        u0[lab >= 0] = -1.0
        u0[np.flatnonzero(lab >= 0), lab[lab >= 0]] = 1.0
    kw = dict(eps=100.0, c=11.0, eta=100.0, precond="damped_jacobi", outer=5, sweeps=4)
    op = make_operator(p, store[0], layout="grid")
    U = torch.from_numpy(u0).to(DEV, DT[store[1]]).contiguous()
    st = op.solve(torch.from_numpy(lab).to(DEV), U, **kw)
    Ug = U.double().cpu().numpy()
    Uo, eo, _ = c_oracle.dca_solve(p.n, rp, col, ww, lab, u0, **kw)
    e, _, flag = gl.split_stats(st.cpu(), K, kw["outer"], kw["sweeps"])
    err = float(np.abs(Ug - Uo).max())
    say(f"grid solve K={K} store={store}: max|dU| {err:.3e}, agreement {label_agreement(Ug, Uo):.6f}")
    assert flag == 0.0 and err <= tol
    assert np.abs(e.numpy() - eo).max() / np.abs(eo).max() <= (1e-10 if store[1] == "f64" else 2e-2)


def test_grid_matches_tile_on_workload4_small():
    """The same graph in the tile and the grid layout: both GPU solves agree
    to float32 rounding (different summation orders)."""
    p = problem(4, small=True)
    out = []
    for layout in ("tile", "grid"):
        op = make_operator(p, "f32", layout=layout)
        assert op.info()["layout"] == layout
        U = torch.from_numpy(p.u0).to(DEV, torch.float32).contiguous()
        op.solve(torch.from_numpy(p.labels).to(DEV), U, eps=p.eps, c=p.c, eta=p.eta,
                 precond="damped_jacobi", outer=p.outer, sweeps=p.sweeps, stats=False)
        out.append(U.double().cpu().numpy())
    err = float(np.abs(out[0] - out[1]).max())
    say(f"grid vs tile max|dU| {err:.3e}")
    assert err <= 2e-6


def test_grid_rejections():
    p = _img(37, 70)
    g = p.graph
    args = (g.row_ptr.to(DEV), g.col.to(DEV), g.weight.to(DEV))
    with pytest.raises(gl.GLError):  # wrong size
        gl.Operator(*args, layout="grid", grid=(37, 71))
    with pytest.raises(gl.GLError):  # an order with the grid layout
        gl.Operator(*args, layout="grid", grid=(37, 70),
                    order=torch.arange(p.n, dtype=torch.int32, device=DEV))
    with pytest.raises(gl.GLError):  # read as a 70 x 37 image the edges leave the window
        gl.Operator(*args, layout="grid", grid=(70, 37))
    op = gl.Operator(*args, layout="grid", grid=(37, 70), store_w="f64")
    with pytest.raises(gl.GLError, match="LDS"):  # 16 double columns (215 KB) exceed one block's LDS
        op.laplacian_apply(torch.zeros((p.n, 16), dtype=torch.float64, device=DEV))
