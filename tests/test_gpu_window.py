"""GPU parity of the window operator: the paper's image graph (Section 2.2)
built on the device from the image (search window, patch similarity), with
implicit columns, against the float64 oracle's graph from the definition.

Small images span several 64 x 4 tiles with ragged right and bottom edges; the
1024 x 1024 case with the 25 x 25 window is checked on sampled rows, computed
one by one by the oracle, in the launch configuration the benchmark times.
"""

import math

import numpy as np
import pytest
import torch

import paper_2303_14495_amd as gl
from oracle import c_oracle, gl_oracle
from oracle import window_oracle as wo
from synth.configs import window_problem
from tests.gpu_helpers import DEV, label_agreement, say

pytestmark = pytest.mark.gpu

DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}
_CACHE = {}


def _problem(h, w, rw, rp=2, seed=5):
    key = (h, w, rw, rp, seed)
    if key not in _CACHE:
        p = window_problem(h, w, rw, rp, seed=seed)
        _CACHE[key] = (p, wo.window_graph(p.image, rw, rp, p.sigma))
    return _CACHE[key]


def _img(p):
    return torch.from_numpy(p.image).to(DEV, torch.float32)


def _oracle_image(p):
    # both sides see the image as float32
    return p.image.astype(np.float32).astype(np.float64)


def _graph(p):
    key = ("f32img",) + (p.image.shape, p.rw, p.rp, p.seed)
    if key not in _CACHE:
        _CACHE[key] = wo.window_graph(_oracle_image(p), p.rw, p.rp, p.sigma)
    return _CACHE[key]


def _op(p, store_w, laplacian="normalized"):
    return gl.Operator.window(_img(p), p.rw, p.rp, p.sigma, store_w=store_w, laplacian=laplacian)


SHAPES = [(40, 150, 5), (37, 70, 12), (24, 60, 27), (9, 200, 3), (1, 130, 4), (130, 1, 2)]


@pytest.mark.parametrize("h,w,rw", SHAPES)
def test_structure_and_counts(h, w, rw):
    p, _ = _problem(h, w, rw)
    say(f"window structure {h}x{w} r={rw}")
    op = _op(p, "f32")
    rp_, col, ww = _graph(p)
    info = op.info()
    assert info["layout"] == "window"
    assert info["n"] == h * w
    assert info["nnz"] == len(col)
    tiles = math.ceil(w / 64) * math.ceil(h / 4)
    # each pair stored once: the first half of every pixel's window (F32: 4 per vector)
    half = ((2 * rw + 1) ** 2 - 1) // 2
    assert info["stored_entries"] == tiles * 256 * (-(-half // 4) * 4)
    assert info["stream_bytes"] == info["stored_entries"] * 4
    opb = _op(p, "bf16")  # 8 offsets per vector
    assert opb.info()["stored_entries"] == tiles * 256 * (-(-half // 8) * 8)
    opb.close()


@pytest.mark.parametrize("laplacian", ["normalized", "unnormalized"])
def test_weights_f64_column_by_column(laplacian):
    """Unit vectors pull single columns of L out of the operator: every stored
    weight (and degree) against the oracle's graph, F64 storage."""
    p, _ = _problem(13, 70, 3, rp=2, seed=9)
    rp_, col, ww = _graph(p)
    n = p.n
    say(f"window weights column by column, {laplacian}")
    op = _op(p, "f64", laplacian)
    dense = (gl_oracle.dense_normalized_laplacian if laplacian == "normalized"
             else gl_oracle.dense_laplacian)
    L = dense(n, rp_, col, ww)
    # 8 unit vectors per call (8 F64 columns of the halo fit one block's LDS)
    got = np.zeros((n, n))
    for start in range(0, n, 8):
        cols = list(range(start, min(start + 8, n)))
        X = torch.zeros((n, 8), dtype=torch.float64, device=DEV)
        for k, j in enumerate(cols):
            X[j, k] = 1.0
        Y = op.laplacian_apply(X).cpu().numpy()
        got[:, cols] = Y[:, :len(cols)]
    err = np.abs(got - L).max()
    say(f"  max |L_gpu - L_oracle| = {err:.3e}")
    assert err <= 1e-13 * max(1.0, np.abs(L).max())
    np.testing.assert_array_equal(got, got.T)  # stored bit for bit symmetric


@pytest.mark.parametrize("h,w,rw", SHAPES[:4])
@pytest.mark.parametrize("store", [("f64", "f64"), ("f32", "f32"), ("bf16", "f32"), ("f16", "f16")])
@pytest.mark.parametrize("K", [1, 3])
def test_laplacian_apply(h, w, rw, store, K):
    p, _ = _problem(h, w, rw)
    store_w, store_u = store
    if 2 * K * (64 + 2 * rw) * (4 + rw) * (8 if store_u == "f64" else 4) > 147456:
        pytest.skip("K columns exceed the LDS of one block at this radius")
    rp_, col, ww = _graph(p)
    say(f"window laplacian {h}x{w} r={rw} store={store} K={K}")
    op = _op(p, store_w)
    rng = np.random.default_rng(h * w + K)
    X = torch.from_numpy(rng.uniform(-1, 1, (p.n, K))).to(DEV, DT[store_u]).contiguous()
    Y = op.laplacian_apply(X).to(torch.float64).cpu().numpy()
    ref = gl_oracle.laplacian_apply(p.n, rp_, col, ww, X.to(torch.float64).cpu().numpy())
    tol = {("f64", "f64"): 1e-13, ("f32", "f32"): 2e-6, ("bf16", "f32"): 1.5e-2,
           ("f16", "f16"): 3e-3}[store]
    err = np.abs(Y - ref).max()
    say(f"  max err {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("h,w,rw,K", [(37, 70, 12, 13), (24, 60, 27, 5)])
def test_laplacian_at_the_lds_limit(h, w, rw, K):
    """The most columns one call may take: 2 K (64 + 2r)(4 + r) floats of V and
    accumulator fill 146 KB of LDS (r = 12, K = 13; r = 27, K = 5); one more
    column is refused."""
    p, _ = _problem(h, w, rw)
    assert 2 * K * (64 + 2 * rw) * (4 + rw) * 4 <= 147456 < 2 * (K + 1) * (64 + 2 * rw) * (4 + rw) * 4
    rp_, col, ww = _graph(p)
    say(f"window laplacian at the LDS limit {h}x{w} r={rw} K={K}")
    op = _op(p, "f32")
    X = torch.from_numpy(np.random.default_rng(K).uniform(-1, 1, (p.n, K))).to(DEV, torch.float32).contiguous()
    Y = op.laplacian_apply(X).double().cpu().numpy()
    ref = gl_oracle.laplacian_apply(p.n, rp_, col, ww, X.double().cpu().numpy())
    assert np.abs(Y - ref).max() <= 2e-6
    X1 = torch.zeros((p.n, K + 1), dtype=torch.float32, device=DEV)
    with pytest.raises(gl.GLError, match="LDS"):
        op.laplacian_apply(X1)


@pytest.mark.parametrize("h,w,rw", SHAPES[3:])
def test_laplacian_thin_images(h, w, rw):
    p, _ = _problem(h, w, rw)
    rp_, col, ww = _graph(p)
    say(f"window laplacian thin image {h}x{w} r={rw}")
    op = _op(p, "f32")
    X = torch.from_numpy(np.random.default_rng(h + w).uniform(-1, 1, (p.n, 2))).to(DEV, torch.float32)
    Y = op.laplacian_apply(X).double().cpu().numpy()
    ref = gl_oracle.laplacian_apply(p.n, rp_, col, ww, X.double().cpu().numpy())
    assert np.abs(Y - ref).max() <= 2e-6


@pytest.mark.parametrize("store_w", ["f64", "f32"])
def test_unnormalized_laplacian(store_w):
    p, _ = _problem(40, 150, 5)
    rp_, col, ww = _graph(p)
    say(f"window unnormalized laplacian store={store_w}")
    op = _op(p, store_w, "unnormalized")
    X = torch.from_numpy(np.random.default_rng(3).uniform(-1, 1, (p.n, 2))).to(DEV, DT[store_w])
    Y = op.laplacian_apply(X).to(torch.float64).cpu().numpy()
    ref = gl_oracle.laplacian_apply(p.n, rp_, col, ww, X.to(torch.float64).cpu().numpy(),
                                    laplacian="unnormalized")
    dmax = float(np.add.reduceat(ww, rp_[:-1]).max())
    err = np.abs(Y - ref).max()
    say(f"  max err {err:.3e} (dmax {dmax:.1f})")
    assert err <= (1e-13 if store_w == "f64" else 2e-6) * dmax


def _decided_agreement(Ug, Uo, margin):
    """Label agreement on the pixels whose oracle label is decided by more
    than `margin` (K = 1: |u| > margin; K > 1: the top two entries more than
    margin apart).  Pixels of a region that holds no labelled pixel keep u ~ 0
    (the sharp patch weights all but cut the region off), and their label is a
    tie at the working precision: either answer is correct there."""
    if Uo.shape[1] == 1:
        dec = np.abs(Uo[:, 0]) > margin
    else:
        top = np.sort(Uo, axis=1)
        dec = top[:, -1] - top[:, -2] > margin
    agree = float(np.mean(gl_oracle.assign_labels(Ug[dec]) == gl_oracle.assign_labels(Uo[dec])))
    return agree, float(dec.mean())


def _solve_case(p, store_w, store_u, precond="damped_jacobi", laplacian="normalized", K=1,
                outer=None, sweeps=None, step_k=math.inf, lam=2.0):
    rp_, col, ww = _graph(p)
    outer = p.outer if outer is None else outer
    sweeps = p.sweeps if sweeps is None else sweeps
    if K == 1:
        labels, u0 = p.labels, p.u0
    else:
        # K classes: class 0 background, rectangles split by column thirds
        x = np.arange(p.n) % p.image.shape[1]
        truth = np.where(p.truth == 1, 1 + (3 * x // p.image.shape[1]) % (K - 1), 0)
        labels = np.where(p.labels >= 0, truth, -1).astype(np.int32)
        u0 = np.where(labels[:, None] >= 0, -1.0, 0.0) * np.ones((1, K))
        u0[labels >= 0, labels[labels >= 0]] = 1.0
    op = _op(p, store_w, laplacian)
    U = torch.from_numpy(np.ascontiguousarray(u0)).to(DEV, DT[store_u]).contiguous()
    st = op.solve(torch.from_numpy(labels).to(DEV), U, eps=p.eps, c=p.c, eta=p.eta,
                  precond=precond, outer=outer, sweeps=sweeps, delta0=p.delta0,
                  lambda_max=lam, step_k=step_k)
    Ug = U.to(torch.float64).cpu().numpy()
    e, r, flag = gl.split_stats(st.cpu(), K, outer, sweeps)
    Uo, eo, ro = c_oracle.dca_solve(p.n, rp_, col, ww, labels, u0, eps=p.eps, c=p.c, eta=p.eta,
                                    precond=precond, outer=outer, sweeps=sweeps,
                                    delta0=p.delta0, lambda_max=lam, step_k=step_k,
                                    laplacian=laplacian)
    return Ug, Uo, e.numpy(), eo, flag


@pytest.mark.parametrize("h,w,rw", SHAPES[:3])
@pytest.mark.parametrize("store,tol", [(("f64", "f64"), 1e-10), (("f32", "f32"), 1e-5),
                                       (("bf16", "f32"), 2e-2), (("bf16", "bf16"), 2e-2)])
def test_solve_parity(h, w, rw, store, tol):
    p, _ = _problem(h, w, rw)
    say(f"window solve {h}x{w} r={rw} store={store}")
    Ug, Uo, eg, eo, flag = _solve_case(p, *store)
    err = float(np.abs(Ug - Uo).max())
    agree, decided = _decided_agreement(Ug, Uo, tol)
    e_rel = float(np.abs(eg - eo).max() / np.abs(eo).max())
    say(f"  max|dU| {err:.3e}  agreement {agree:.6f} on {decided:.4f} decided  "
        f"(all pixels {label_agreement(Ug, Uo):.6f})  energy rel {e_rel:.2e}")
    assert flag == 0.0
    assert err <= tol
    assert agree >= 0.999 and decided >= 0.5
    assert e_rel <= (1e-10 if store[1] == "f64" else 1e-4 if store == ("f32", "f32") else 2e-2)
    # Theorem 1: the energy does not increase over the DCA steps
    assert np.all(np.diff(eg[:, 0]) <= 1e-6 * np.abs(eg).max())


@pytest.mark.parametrize("store", [("f32", "f32"), ("bf16", "f32"), ("f16", "f16")])
def test_solve_bitwise_repeatable(store):
    """Each stored weight serves both directions of its pair: a tile adds
    w V_j into its own pixel and w V_i into the neighbour's cell of its region,
    and the neighbour's sum gathers the regions of the tiles that cover it.
    The order of all these additions is fixed (the window rows are phases
    separated by barriers, and the regions are summed in tile order), so two
    runs give the same bits.  Ragged 64 x 4 tiles, a window reaching four
    tile rows up and one tile to each side."""
    p, _ = _problem(37, 150, 12)
    say(f"window solve run twice, store={store}")
    op = _op(p, store[0])
    lab = torch.from_numpy(p.labels).to(DEV)
    outs = []
    for _ in range(2):
        U = torch.from_numpy(p.u0).to(DEV, DT[store[1]]).contiguous()
        st = op.solve(lab, U, eps=p.eps, c=p.c, eta=p.eta, precond=p.precond, outer=p.outer,
                      sweeps=p.sweeps, delta0=p.delta0, lambda_max=2.0)
        outs.append((U.cpu().view(torch.uint8).numpy().copy(), st.cpu().numpy().copy()))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])


@pytest.mark.timeout(900)
@pytest.mark.parametrize("store,tol", [(("f32", "f32"), 1e-5), (("bf16", "f32"), 2e-2)])
def test_solve_512_window25(store, tol):
    """A whole solve on a 512 x 512 image with the paper's 25 x 25 window and
    5 x 5 patches (160 M stored edges; the graph of the C oracle, pinned to the
    definition), 10 DCA steps x 4 damped-Jacobi sweeps, against the float64
    oracle."""
    key = ("w512",)
    if key not in _CACHE:
        p = window_problem(512, 512, 12, 2, seed=5)
        _CACHE[key] = (p, c_oracle.window_graph(_oracle_image(p), p.rw, p.rp, p.sigma))
    p, (rp_, col, ww) = _CACHE[key]
    say(f"window solve 512x512 r=12 store={store}: {len(col)} edges")
    op = _op(p, store[0])
    assert op.info()["nnz"] == len(col)
    U = torch.from_numpy(np.ascontiguousarray(p.u0)).to(DEV, DT[store[1]]).contiguous()
    st = op.solve(torch.from_numpy(p.labels).to(DEV), U, eps=p.eps, c=p.c, eta=p.eta,
                  precond=p.precond, outer=p.outer, sweeps=p.sweeps, delta0=p.delta0)
    Ug = U.to(torch.float64).cpu().numpy()
    eg, _, flag = gl.split_stats(st.cpu(), 1, p.outer, p.sweeps)
    key2 = ("w512-oracle",)
    if key2 not in _CACHE:
        _CACHE[key2] = c_oracle.dca_solve(p.n, rp_, col, ww, p.labels, p.u0, eps=p.eps, c=p.c,
                                          eta=p.eta, precond=p.precond, outer=p.outer,
                                          sweeps=p.sweeps, delta0=p.delta0)
    Uo, eo, _ = _CACHE[key2]
    err = float(np.abs(Ug - Uo).max())
    agree, decided = _decided_agreement(Ug, Uo, tol)
    e_rel = float(np.abs(eg.numpy() - eo).max() / np.abs(eo).max())
    say(f"  max|dU| {err:.3e}  agreement {agree:.6f} on {decided:.4f} decided  energy rel {e_rel:.2e}")
    assert flag == 0.0
    assert err <= tol
    assert agree >= 0.999 and decided >= 0.5
    assert e_rel <= (1e-4 if store == ("f32", "f32") else 2e-2)


@pytest.mark.parametrize("precond", ["perturbed_jacobi", "richardson"])
def test_solve_other_preconditioners(precond):
    p, _ = _problem(40, 150, 5)
    rp_, col, ww = _graph(p)
    lam = 2.0
    if precond == "richardson":
        rq, lam = c_oracle.power_max_eig(p.n, rp_, col, ww, np.random.default_rng(1).uniform(-1, 1, p.n))
    say(f"window solve {precond} lambda={lam:.4f}")
    Ug, Uo, _, _, flag = _solve_case(p, "f32", "f32", precond=precond, lam=lam)
    err = float(np.abs(Ug - Uo).max())
    say(f"  max|dU| {err:.3e}")
    assert flag == 0.0 and err <= 1e-5


def test_solve_step_k_and_unnormalized():
    p, _ = _problem(40, 150, 5)
    say("window solve, step k = 0.5, unnormalized L, f32")
    Ug, Uo, _, _, flag = _solve_case(p, "f32", "f32", laplacian="unnormalized", step_k=0.5)
    err = float(np.abs(Ug - Uo).max())
    say(f"  max|dU| {err:.3e}")
    assert flag == 0.0 and err <= 1e-5


@pytest.mark.parametrize("K", [3, 4])
def test_solve_multiclass(K):
    p, _ = _problem(37, 70, 5 if K == 4 else 12)
    say(f"window solve K={K}")
    Ug, Uo, _, _, flag = _solve_case(p, "f32", "f32", K=K)
    err = float(np.abs(Ug - Uo).max())
    agree, decided = _decided_agreement(Ug, Uo, 1e-5)
    say(f"  max|dU| {err:.3e} agreement {agree:.6f} on {decided:.4f} decided")
    assert flag == 0.0 and err <= 1e-5 and agree >= 0.999


def test_power_method_vs_oracle():
    p, _ = _problem(37, 70, 12)
    rp_, col, ww = _graph(p)
    x0 = np.random.default_rng(4).uniform(-1, 1, p.n)
    rq_o, lam_o = c_oracle.power_max_eig(p.n, rp_, col, ww, x0, 150)
    op = _op(p, "f32")
    rq, lam = op.power_max_eig(torch.from_numpy(x0).to(DEV, torch.float32), 150)
    say(f"window power: rq {rq:.6f} oracle {rq_o:.6f}")
    assert abs(rq - rq_o) <= 1e-4 * rq_o
    assert lam == pytest.approx(min(2.0, 1.01 * rq), rel=1e-12)


def test_second_eigenpair_vs_dense_oracle():
    p, _ = _problem(16, 70, 4, seed=11)
    rp_, col, ww = _graph(p)
    lam_o, v_o = gl_oracle.second_eigenpair(p.n, rp_, col, ww)
    op = _op(p, "f32")
    x0 = torch.from_numpy(np.random.default_rng(6).uniform(-1, 1, p.n)).to(DEV, torch.float32)
    lam, v, res, rs = op.second_eigenpair(x0, krylov=128, max_restarts=40, tol=1e-5)
    v = v.cpu().numpy().astype(np.float64)
    say(f"window lambda2 {lam:.6e} oracle {lam_o:.6e} residual {res:.1e} |cos| {abs(v @ v_o):.6f}")
    assert res <= 1e-5
    assert lam == pytest.approx(lam_o, rel=1e-3, abs=1e-6)


def test_window_matches_csr_operator():
    """The same graph through the CSR path (the oracle's weights uploaded) and
    through the window path: the two GPU solves agree."""
    p, _ = _problem(40, 150, 5)
    rp_, col, ww = _graph(p)
    csr = gl.Operator(torch.from_numpy(rp_).to(DEV), torch.from_numpy(col).to(DEV),
                      torch.from_numpy(ww).to(DEV), store_w="f32")
    win = _op(p, "f32")
    lab = torch.from_numpy(p.labels).to(DEV)
    out = []
    for op in (csr, win):
        U = torch.from_numpy(p.u0).to(DEV, torch.float32).contiguous()
        op.solve(lab, U, eps=p.eps, c=p.c, eta=p.eta, precond=p.precond, outer=p.outer,
                 sweeps=p.sweeps, stats=False)
        out.append(U.double().cpu().numpy())
    err = float(np.abs(out[0] - out[1]).max())
    say(f"window vs CSR max|dU| {err:.3e}")
    assert err <= 2e-6


def test_degenerate_and_rejected():
    # one pixel: no neighbour, degree 0
    with pytest.raises(gl.GLError):
        gl.Operator.window(torch.zeros((1, 1, 3), device=DEV), 3, 2, 1.0)
    # every weight underflows: all pixels at least 10 levels apart, tiny sigma
    img = 10.0 * torch.arange(64, dtype=torch.float32, device=DEV).view(8, 8)
    with pytest.raises(gl.GLError):
        gl.Operator.window(img, 1, 0, 0.01)
    # two pixels: one edge of weight exp(-|dC|^2 / sigma^2); L_s = [[1, -1], [-1, 1]]
    op = gl.Operator.window(torch.tensor([[0.0, 1.0]], device=DEV), 1, 0, 2.0, store_w="f64")
    assert op.info()["nnz"] == 2
    Y = op.laplacian_apply(torch.tensor([[1.0], [0.0]], dtype=torch.float64, device=DEV))
    assert Y.cpu().numpy().ravel().tolist() == pytest.approx([1.0, -1.0], abs=1e-15)
    opu = gl.Operator.window(torch.tensor([[0.0, 1.0]], device=DEV), 1, 0, 2.0, store_w="f64",
                             laplacian="unnormalized")
    Y = opu.laplacian_apply(torch.tensor([[1.0], [0.0]], dtype=torch.float64, device=DEV))
    wv = math.exp(-1.0 / 4.0)
    assert Y.cpu().numpy().ravel().tolist() == pytest.approx([wv, -wv], rel=1e-15)
    # the LDS limit: 16 columns of the 55 x 55 window do not fit one block
    p, _ = _problem(24, 60, 27)
    big = _op(p, "f32")
    with pytest.raises(gl.GLError):
        big.laplacian_apply(torch.zeros((p.n, 16), device=DEV))


@pytest.mark.parametrize("store_w,tol", [("f32", 1e-5), ("bf16", 1e-2)])
def test_full_size_sampled_rows(store_w, tol):
    """1024 x 1024 image, 25 x 25 window, 5 x 5 patches (the benchmark's
    workload and launch): sampled rows of L_s X against the oracle's rows
    computed one by one from the definition, including image corners and tile
    borders."""
    p = window_problem()  # defaults: the benchmark workload
    h, w = p.image.shape[:2]
    say(f"window full size {h}x{w} r={p.rw} store={store_w}")
    op = _op(p, store_w)
    X = torch.from_numpy(np.random.default_rng(77).uniform(-1, 1, (p.n, 1))).to(DEV, torch.float32)
    Y = op.laplacian_apply(X).double().cpu().numpy()[:, 0]
    Xn = X.double().cpu().numpy()[:, 0]
    rng = np.random.default_rng(78)
    picks = [0, w - 1, (h - 1) * w, h * w - 1, 63, 64, 3 * w + 63, 4 * w + 64, 511 * w + 512]
    picks += rng.integers(0, p.n, 7).tolist()
    rows = wo.window_rows(_oracle_image(p), p.rw, p.rp, p.sigma, picks)
    worst = 0.0
    for i, (js, wij, di, dj) in zip(picks, rows):
        ref = Xn[i] - float(np.sum(wij / np.sqrt(di * dj) * Xn[js]))
        worst = max(worst, abs(Y[i] - ref))
    say(f"  worst sampled-row error {worst:.3e}")
    assert worst <= tol
