"""GPU parity of gl_second_eigenpair (the unsupervised initialisation of
Section 5.2) against the dense float64 oracle, and of the unsupervised solve
started from the oracle's eigenvector."""

import math

import numpy as np
import pytest
import torch

import paper_2303_14495_amd as gl
from oracle import c_oracle, gl_oracle
from synth.configs import StreamItem, served_problem
from synth.graphs import dense_to_graph
from tests.gpu_helpers import DEV, make_operator, power_x0, problem, say

pytestmark = pytest.mark.gpu


def _path(n):
    W = np.zeros((n, n))
    for i in range(n - 1):
        W[i, i + 1] = W[i + 1, i] = 1.0
    return dense_to_graph(W)


def _gp(g):
    P = type("P", (), {})()
    P.graph = g
    P.n = g.n
    return P


def _x0(n, seed=5):
    return torch.from_numpy(power_x0(n, seed)).to(DEV, torch.float32)


@pytest.mark.parametrize("laplacian", ["normalized", "unnormalized"])
def test_path_closed_form(laplacian):
    n = 64
    g = _path(n)
    op = make_operator(_gp(g), "f32", laplacian=laplacian)
    lam, v, res, rs = op.second_eigenpair(_x0(n), krylov=64, max_restarts=5, tol=1e-6)
    v = v.cpu().numpy().astype(np.float64)
    j = np.arange(n)
    if laplacian == "normalized":
        want_l = 1 - math.cos(math.pi / (n - 1))
        d = np.r_[1.0, np.full(n - 2, 2.0), 1.0]
        want = np.sqrt(d) * np.cos(math.pi * j / (n - 1))
    else:
        want_l = 2 - 2 * math.cos(math.pi / n)
        want = np.cos(math.pi * (j + 0.5) / n)
    want /= np.linalg.norm(want)
    say(f"path {laplacian}: lambda2 {lam:.8e} (want {want_l:.8e}), residual {res:.2e}, restarts {rs}")
    assert lam == pytest.approx(want_l, rel=1e-4)
    assert abs(abs(v @ want) - 1) < 1e-5
    assert v[np.argmax(np.abs(v))] > 0
    assert res <= 1e-5


def _mixture(n=1500, index=7):
    return served_problem(StreamItem(index, n, 2, 10, 0.0), device=DEV)


def test_mixture_vs_dense_oracle():
    p = _mixture()
    rp, col, w = p.graph.numpy()
    lam_o, v_o = gl_oracle.second_eigenpair(p.n, rp, col, w)
    ev = np.linalg.eigvalsh(gl_oracle.dense_normalized_laplacian(p.n, rp, col, w))
    say(f"mixture n={p.n}: lambda2 {lam_o:.6e}, lambda3 {ev[2]:.6e}")
    op = make_operator(p, "f32")
    lam, v, res, rs = op.second_eigenpair(_x0(p.n), krylov=96, max_restarts=30, tol=1e-5)
    v = v.cpu().numpy().astype(np.float64)
    say(f"  gpu lambda2 {lam:.6e}, residual {res:.2e}, restarts {rs}, |cos| {abs(v @ v_o):.8f}")
    assert res <= 1e-5
    assert lam == pytest.approx(lam_o, rel=1e-4, abs=1e-6)
    # eigenvector error bound: |sin angle| <= residual / gap
    gap = ev[2] - lam_o
    assert 1 - abs(v @ v_o) <= max(1e-4, 2 * (res / gap) ** 2)
    assert np.sign(v[np.argmax(np.abs(v))]) > 0


def test_tile_and_direct_agree():
    p = problem(2, small=True)
    a = make_operator(p, "f32", layout="tile")
    b = make_operator(p, "f32", layout="direct", use_order=False)
    x0 = _x0(p.n, 9)
    la, va, ra, _ = a.second_eigenpair(x0, krylov=128, max_restarts=40, tol=1e-5)
    lb, vb, rb, _ = b.second_eigenpair(x0, krylov=128, max_restarts=40, tol=1e-5)
    cosv = abs(float((va.double() @ vb.double()).item()))
    say(f"tile {la:.6e} ({ra:.1e}) direct {lb:.6e} ({rb:.1e}) |cos| {cosv:.8f}")
    assert la == pytest.approx(lb, rel=1e-4)
    assert ra <= 1e-5 and rb <= 1e-5


def test_unsupervised_solve_from_second_eigenvector():
    """The unsupervised run of Section 5.2: no labels, u^0 from the second
    eigenvector (the oracle's, scaled to max |u| = 1), eps = 100, c = 11,
    eta = 100; parity with the oracle and the two clusters recovered."""
    p = _mixture()
    rp, col, w = p.graph.numpy()
    _, v_o = gl_oracle.second_eigenpair(p.n, rp, col, w)
    u0 = gl_oracle.unsupervised_u0(v_o)
    labels = np.full(p.n, -1, dtype=np.int32)
    kw = dict(eps=100.0, c=11.0, eta=100.0, precond="damped_jacobi", outer=20, sweeps=4)
    op = make_operator(p, "f32")
    U = torch.from_numpy(u0).to(DEV, torch.float32).contiguous()
    op.solve(torch.from_numpy(labels).to(DEV), U, stats=False, **kw)
    Ug = U.double().cpu().numpy()
    Uo, _, _ = c_oracle.dca_solve(p.n, rp, col, w, labels, u0, **kw)
    err = float(np.abs(Ug - Uo).max())
    cls = (Ug[:, 0] >= 0).astype(int)
    acc = max(np.mean(cls == p.truth), np.mean(cls != p.truth))
    say(f"unsupervised: max|dU| {err:.2e}, accuracy {acc:.4f}")
    assert err <= 1e-5
    assert acc >= 0.95


def test_rejects_bad_arguments():
    g = _path(16)
    op = make_operator(_gp(g), "f32")
    for kw in [dict(krylov=1), dict(krylov=600), dict(max_restarts=-1), dict(tol=0.0)]:
        with pytest.raises(gl.GLError):
            op.second_eigenpair(_x0(16), **kw)
    with pytest.raises(gl.GLError):
        # a start vector parallel to the null vector D^{1/2} 1
        d = np.r_[1.0, np.full(14, 2.0), 1.0]
        op.second_eigenpair(torch.from_numpy(np.sqrt(d)).to(DEV, torch.float32))
