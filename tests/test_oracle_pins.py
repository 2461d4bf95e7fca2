"""Pins of the float64 oracle to facts the paper and the mathematics fix.

Both oracle implementations (numpy and plain C) are held to:
  * hand-derived exact results on a two-node graph (tests/golden/two_node.json);
  * L_s D^{1/2} 1 = 0, symmetry, positive semidefiniteness and spectrum in
    [0, 2] (Section 2.2, Prop. 3);
  * closed-form largest eigenvalues of L_s for complete graphs, cycles and
    stars (power method, Section 3.1);
  * feasibility G - T > 0 of every preconditioner (Section 3.1);
  * the closed form of m diagonal sweeps and, as m grows, the direct solve
    of T u = b (Section 3, Prop. 1);
  * energy decay F(u^{t+1}) <= F(u^t) and, for one sweep per step, the
    sharper Thm. 1 bound with M_0 = G - T;
  * invariants: sign symmetry, a fixed point, column decoupling, permutation
    equivariance, split-run resume;
  * for the unnormalized Laplacian L = D - W: a hand-derived two-node golden
    (tests/golden/two_node_unnormalized.json), the explicit path Laplacian,
    L 1 = 0, 2D >= L (Prop. 3), L = D^{1/2} L_s D^{1/2}, closed-form largest
    eigenvalues, feasibility and the closed form of the sweeps with the
    D-dependent preconditioners of Section 3.1, energy decay.
"""

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import c_oracle, gl_oracle
from synth.graphs import dense_to_graph, tiny_graph

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ORACLES = [pytest.param(gl_oracle, id="numpy"), pytest.param(c_oracle, id="c")]


def _dense_W(g):
    rp, col, w = g.numpy()
    W = np.zeros((g.n, g.n))
    for i in range(g.n):
        W[i, col[rp[i]:rp[i + 1]]] = w[rp[i]:rp[i + 1]]
    return W


def _dense_Ls(W):
    d = W.sum(1)
    s = 1.0 / np.sqrt(d)
    return np.eye(W.shape[0]) - s[:, None] * W * s[None, :]


def _fid(labels, K):
    n = len(labels)
    lam = np.array([1.0 if l >= 0 else 0.0 for l in labels])
    y = np.zeros((n, K))
    for i, l in enumerate(labels):
        if l < 0:
            continue
        for k in range(K):
            y[i, k] = (1.0 if l == 1 else -1.0) if K == 1 else (1.0 if l == k else -1.0)
    return lam, y


# --------------------------------------------------------------------------
# golden two-node case
# --------------------------------------------------------------------------

@pytest.mark.parametrize("orc", ORACLES)
@pytest.mark.parametrize("golden", ["two_node.json", "two_node_unnormalized.json"])
def test_two_node_golden(orc, golden):
    gd = json.load(open(os.path.join(GOLDEN, golden)))
    lapl = gd.get("laplacian", "normalized")
    rp = np.array(gd["graph"]["row_ptr"], dtype=np.int64)
    col = np.array(gd["graph"]["col"], dtype=np.int32)
    w = np.array(gd["graph"]["weight"])
    lab = np.array(gd["labels"], dtype=np.int32)
    u0 = np.array(gd["u0"])[:, None]
    for case in gd["cases"]:
        k = math.inf if case["step_k"] == "inf" else float(case["step_k"])
        U, en, rs = orc.dca_solve(2, rp, col, w, lab, u0, eps=gd["eps"], c=gd["c"], eta=gd["eta"],
                                  precond=case["precond"], outer=case["outer"],
                                  sweeps=case["sweeps"], delta0=case["delta0"],
                                  lambda_max=case["lambda_max"], step_k=k, laplacian=lapl)
        want = np.array([float(Fraction(x)) for x in case["u"]])
        np.testing.assert_allclose(U[:, 0], want, rtol=0, atol=1e-15, err_msg=case["name"])
        if "residual_sq" in case:
            r = np.array([[float(Fraction(x)) for x in row] for row in case["residual_sq"]])
            np.testing.assert_allclose(rs[:, :, 0], r, rtol=1e-14, err_msg=case["name"])
        if "energies" in case:
            e = np.array([float(Fraction(x)) for x in case["energies"]])
            np.testing.assert_allclose(en[:, 0], e, rtol=1e-14, err_msg=case["name"])


# --------------------------------------------------------------------------
# the normalized Laplacian
# --------------------------------------------------------------------------

def test_path3_normalized_laplacian_explicit():
    # path 0-1-2 with unit weights: d = (1, 2, 1); L_s has off-diagonals -1/sqrt(2)
    g = dense_to_graph(np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]], dtype=float))
    rp, col, w = g.numpy()
    L = gl_oracle.dense_normalized_laplacian(3, rp, col, w)
    h = 1 / math.sqrt(2)
    np.testing.assert_allclose(L, [[1, -h, 0], [-h, 1, -h], [0, -h, 1]], atol=1e-15)
    np.testing.assert_allclose(np.linalg.eigvalsh(L), [0, 1, 2], atol=1e-14)
    for orc in (gl_oracle, c_oracle):
        np.testing.assert_allclose(orc.laplacian_apply(3, rp, col, w, np.eye(3)), L, atol=1e-15)


@pytest.mark.parametrize("orc", ORACLES)
@pytest.mark.parametrize("seed", range(6))
def test_laplacian_properties(orc, seed):
    rng = np.random.default_rng(seed)
    g = tiny_graph(int(rng.integers(3, 24)), 0.3, rng)
    rp, col, w = g.numpy()
    W = _dense_W(g)
    sqrt_d = np.sqrt(W.sum(1))
    # L_s D^{1/2} 1 = 0 (Section 2.2)
    z = orc.laplacian_apply(g.n, rp, col, w, sqrt_d[:, None])
    assert np.abs(z).max() < 1e-13
    L = orc.laplacian_apply(g.n, rp, col, w, np.eye(g.n))
    np.testing.assert_allclose(L, L.T, atol=1e-15)
    ev = np.linalg.eigvalsh(L)
    assert ev.min() > -1e-12 and ev.max() < 2 + 1e-12          # Prop. 3: 0 <= L_s <= 2I
    np.testing.assert_allclose(L, _dense_Ls(W), atol=1e-14)
    # a random block of columns is applied column by column consistently
    X = rng.standard_normal((g.n, 3))
    np.testing.assert_allclose(orc.laplacian_apply(g.n, rp, col, w, X), L @ X, atol=1e-13)


def test_laplacian_scale_invariance():
    # L_s does not change when every weight is scaled by the same factor
    rng = np.random.default_rng(3)
    g = tiny_graph(12, 0.3, rng)
    rp, col, w = g.numpy()
    X = rng.standard_normal((12, 2))
    a = gl_oracle.laplacian_apply(12, rp, col, w, X)
    b = gl_oracle.laplacian_apply(12, rp, col, 7.5 * w, X)
    np.testing.assert_allclose(a, b, atol=1e-14)


# --------------------------------------------------------------------------
# power method: closed-form spectra
# --------------------------------------------------------------------------

def _complete(n):
    return dense_to_graph(np.ones((n, n)) - np.eye(n))


def _cycle(n):
    W = np.zeros((n, n))
    for i in range(n):
        W[i, (i + 1) % n] = W[(i + 1) % n, i] = 1.0
    return dense_to_graph(W)


def _star(n):
    W = np.zeros((n, n))
    W[0, 1:] = W[1:, 0] = 1.0
    return dense_to_graph(W)


@pytest.mark.parametrize("orc", ORACLES)
@pytest.mark.parametrize("name,g,lam", [
    ("K5", _complete(5), 5 / 4),
    ("K9", _complete(9), 9 / 8),
    ("C8", _cycle(8), 2.0),
    ("C10", _cycle(10), 2.0),
    ("C7", _cycle(7), 1 - math.cos(2 * math.pi * 3 / 7)),
    ("C9", _cycle(9), 1 - math.cos(2 * math.pi * 4 / 9)),
    ("S6", _star(6), 2.0),
])
def test_power_method_closed_form(orc, name, g, lam):
    rp, col, w = g.numpy()
    x0 = np.random.default_rng(11).uniform(-1, 1, g.n)
    rq, lhat = orc.power_max_eig(g.n, rp, col, w, x0, iters=150)
    assert abs(rq - lam) < 1e-6 * lam, (name, rq, lam)
    assert lhat == pytest.approx(min(2.0, 1.01 * rq), rel=1e-15)
    assert lhat <= 2.0


# --------------------------------------------------------------------------
# preconditioners: feasibility and the closed form of the sweeps
# --------------------------------------------------------------------------

def _setup(seed, n=None, K=1, p=0.3):
    rng = np.random.default_rng(seed)
    n = n or int(rng.integers(4, 20))
    g = tiny_graph(n, p, rng)
    labels = np.full(n, -1, dtype=np.int32)
    lab_idx = rng.choice(n, size=max(1, n // 4), replace=False)
    labels[lab_idx] = rng.integers(0, max(K, 2), lab_idx.size)
    u0 = rng.uniform(-1, 1, (n, K))
    return g, labels, u0


@pytest.mark.parametrize("kind", gl_oracle.PRECONDS)
@pytest.mark.parametrize("step_k", [math.inf, 0.05, 1.0, 5.0])
def test_preconditioner_feasible(kind, step_k):
    for seed in range(4):
        g, labels, _ = _setup(seed)
        rp, col, w = g.numpy()
        L = _dense_Ls(_dense_W(g))
        lam, _ = _fid(labels, 1)
        eps, c, eta = 1.7, 2.3, 50.0
        lmax = float(np.linalg.eigvalsh(L).max())
        G = np.diag(gl_oracle.precond_diag(kind, lam, eps, c, eta, 1e-3, lmax, step_k))
        T = eps * L + eta * np.diag(lam) + c * np.eye(g.n)
        if not math.isinf(step_k):
            T = np.eye(g.n) + step_k * T
        assert np.linalg.eigvalsh(G - T).min() > 0


def _closed_form_sweeps(L, lam, y, u, eps, c, eta, g, m, step_k):
    n = L.shape[0]
    T = eps * L + eta * np.diag(lam) + c * np.eye(n)
    b = c * u - (u ** 3 - u) / eps + eta * lam[:, None] * y
    if not math.isinf(step_k):
        T, b = np.eye(n) + step_k * T, u + step_k * b
    Ginv = np.diag(1.0 / g)
    Em = np.linalg.matrix_power(np.eye(n) - Ginv @ T, m)
    return u + (np.eye(n) - Em) @ np.linalg.solve(T, b - T @ u), T, b


@pytest.mark.parametrize("orc", ORACLES)
@pytest.mark.parametrize("kind", gl_oracle.PRECONDS)
@pytest.mark.parametrize("m", [1, 3, 8])
@pytest.mark.parametrize("step_k", [math.inf, 0.5])
def test_sweeps_closed_form(orc, kind, m, step_k):
    for seed in range(3):
        g, labels, u0 = _setup(seed, K=1)
        rp, col, w = g.numpy()
        L = _dense_Ls(_dense_W(g))
        lam, y = _fid(labels, 1)
        eps, c, eta = 1.3, 3.0, 20.0
        lmax = float(np.linalg.eigvalsh(L).max())
        gd = gl_oracle.precond_diag(kind, lam, eps, c, eta, 1e-2, lmax, step_k)
        want, _, _ = _closed_form_sweeps(L, lam, y, u0, eps, c, eta, gd, m, step_k)
        U, _, _ = orc.dca_solve(g.n, rp, col, w, labels, u0, eps=eps, c=c, eta=eta, precond=kind,
                                outer=1, sweeps=m, delta0=1e-2, lambda_max=lmax, step_k=step_k)
        np.testing.assert_allclose(U, want, atol=1e-12)


@pytest.mark.parametrize("orc", ORACLES)
def test_many_sweeps_reach_direct_solve(orc):
    # with enough sweeps the inner iteration solves T u^{t+1} = b^t (Section 3)
    g, labels, u0 = _setup(5, n=15, K=2)
    rp, col, w = g.numpy()
    L = _dense_Ls(_dense_W(g))
    lam, y = _fid(labels, 2)
    eps, c, eta = 1.0, 3.0, 10.0
    T = eps * L + eta * np.diag(lam) + c * np.eye(g.n)
    b = c * u0 - (u0 ** 3 - u0) / eps + eta * lam[:, None] * y
    U, _, rs = orc.dca_solve(g.n, rp, col, w, labels, u0, eps=eps, c=c, eta=eta,
                             precond="damped_jacobi", outer=1, sweeps=600)
    np.testing.assert_allclose(U, np.linalg.solve(T, b), atol=1e-11)
    assert rs[0, -1].max() < 1e-20


# --------------------------------------------------------------------------
# energy (Section 2.1) and Thm. 1
# --------------------------------------------------------------------------

def test_energy_double_sum_form():
    # u^T L_s u = 1/2 sum_ij w_ij (u_i/sqrt(d_i) - u_j/sqrt(d_j))^2
    for seed in range(5):
        g, labels, u0 = _setup(seed, K=3)
        rp, col, w = g.numpy()
        W = _dense_W(g)
        d = W.sum(1)
        eps, eta = 0.7, 30.0
        lam, y = _fid(labels, 3)
        F = gl_oracle.energy(g.n, rp, col, w, u0, labels, eps, eta)
        for k in range(3):
            x = u0[:, k] / np.sqrt(d)
            lap = 0.5 * np.sum(W * (x[:, None] - x[None, :]) ** 2)
            want = (eps / 2) * lap + np.sum((u0[:, k] ** 2 - 1) ** 2) / (4 * eps) \
                + (eta / 2) * np.sum(lam * (u0[:, k] - y[:, k]) ** 2)
            assert F[k] == pytest.approx(want, rel=1e-13)


def _convexity_ok(U, eps, c):
    # P2 = (c/2)|u|^2 - W(u)/eps is convex on the iterates iff c >= (3u^2 - 1)/eps
    return np.all(c * eps >= 3 * U ** 2 - 1)


@pytest.mark.parametrize("orc", ORACLES)
@pytest.mark.parametrize("kind", gl_oracle.PRECONDS)
@pytest.mark.parametrize("m", [1, 4])
def test_energy_decreases(orc, kind, m):
    for seed in range(4):
        g, labels, u0 = _setup(seed, n=20, K=2)
        rp, col, w = g.numpy()
        eps, c, eta = 1.0, 3.0, 100.0
        lmax = float(np.linalg.eigvalsh(_dense_Ls(_dense_W(g))).max())
        U, en, _ = orc.dca_solve(g.n, rp, col, w, labels, u0, eps=eps, c=c, eta=eta,
                                 precond=kind, outer=25, sweeps=m, delta0=1e-6,
                                 lambda_max=lmax)
        assert _convexity_ok(U, eps, c)
        assert np.all(np.diff(en, axis=0) <= 1e-12 * np.abs(en[:-1]))


def test_energy_decay_sharp_bound_one_sweep():
    # Thm. 1: F(u+) + 1/2 |u+ - u|^2_{M0} <= F(u), M0 = G - T for one sweep
    for seed in range(5):
        g, labels, u = _setup(seed, n=16, K=1)
        rp, col, w = g.numpy()
        L = _dense_Ls(_dense_W(g))
        lam, _ = _fid(labels, 1)
        eps, c, eta = 1.0, 3.0, 100.0
        T = eps * L + eta * np.diag(lam) + c * np.eye(g.n)
        for kind in gl_oracle.PRECONDS:
            G = np.diag(gl_oracle.precond_diag(kind, lam, eps, c, eta, 1e-6, 2.0))
            M0 = G - T
            U = u.copy()
            for _ in range(10):
                Un, en, _ = gl_oracle.dca_solve(g.n, rp, col, w, labels, U, eps=eps, c=c,
                                                eta=eta, precond=kind, outer=1, sweeps=1)
                assert _convexity_ok(U, eps, c) and _convexity_ok(Un, eps, c)
                dlt = (Un - U)[:, 0]
                assert en[1, 0] + 0.5 * dlt @ M0 @ dlt <= en[0, 0] + 1e-12 * abs(en[0, 0])
                U = Un


# --------------------------------------------------------------------------
# invariants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("orc", ORACLES)
def test_sign_symmetry_bitwise(orc):
    g, labels, u0 = _setup(2, n=18, K=1)
    rp, col, w = g.numpy()
    flipped = np.where(labels >= 0, 1 - labels, -1).astype(np.int32)
    kw = dict(eps=1.0, c=3.0, eta=100.0, precond="damped_jacobi", outer=8, sweeps=3)
    a, _, _ = orc.dca_solve(g.n, rp, col, w, labels, u0, **kw)
    b, _, _ = orc.dca_solve(g.n, rp, col, w, flipped, -u0, **kw)
    assert np.array_equal(a, -b)


@pytest.mark.parametrize("orc", ORACLES)
def test_fixed_point_on_cycle(orc):
    # unweighted cycle: what = 1/2 exactly; u = 1 with every node labelled 1
    # satisfies T u = b, and every sweep leaves it exactly in place
    g = _cycle(12)
    rp, col, w = g.numpy()
    labels = np.ones(12, dtype=np.int32)
    for kind in gl_oracle.PRECONDS:
        U, _, rs = orc.dca_solve(12, rp, col, w, labels, np.ones((12, 1)), eps=1.0, c=3.0,
                                 eta=4.0, precond=kind, outer=5, sweeps=4, delta0=0.25,
                                 lambda_max=2.0)
        assert np.array_equal(U, np.ones((12, 1)))
        assert np.all(rs == 0.0)


@pytest.mark.parametrize("orc", ORACLES)
def test_column_decoupling(orc):
    g, labels, u0 = _setup(4, n=20, K=3)
    rp, col, w = g.numpy()
    kw = dict(eps=1.0, c=3.0, eta=50.0, precond="perturbed_jacobi", outer=6, sweeps=3)
    U, en, rs = orc.dca_solve(g.n, rp, col, w, labels, u0, **kw)
    for k in range(3):
        lk = np.where(labels >= 0, (labels == k).astype(np.int32), -1).astype(np.int32)
        Uk, ek, rk = orc.dca_solve(g.n, rp, col, w, lk, u0[:, k:k + 1], **kw)
        np.testing.assert_allclose(U[:, k], Uk[:, 0], rtol=0, atol=1e-15)
        np.testing.assert_allclose(en[:, k], ek[:, 0], rtol=1e-14)
        np.testing.assert_allclose(rs[:, :, k], rk[:, :, 0], rtol=1e-13)


@pytest.mark.parametrize("orc", ORACLES)
def test_permutation_equivariance(orc):
    g, labels, u0 = _setup(6, n=17, K=2)
    W = _dense_W(g)
    perm = np.random.default_rng(0).permutation(g.n)
    gp = dense_to_graph(W[np.ix_(perm, perm)])
    kw = dict(eps=1.0, c=3.0, eta=50.0, precond="richardson", outer=5, sweeps=4,
              lambda_max=1.9)
    rp, col, w = g.numpy()
    a, ea, _ = orc.dca_solve(g.n, rp, col, w, labels, u0, **kw)
    rp, col, w = gp.numpy()
    b, eb, _ = orc.dca_solve(g.n, rp, col, w, labels[perm], u0[perm], **kw)
    np.testing.assert_allclose(a[perm], b, atol=1e-13)
    np.testing.assert_allclose(ea, eb, rtol=1e-12)


@pytest.mark.parametrize("orc", ORACLES)
def test_split_run_resume(orc):
    # pDCA is memoryless: u^{t+1} depends on u^t only
    g, labels, u0 = _setup(7, n=19, K=2)
    rp, col, w = g.numpy()
    kw = dict(eps=1.0, c=3.0, eta=50.0, precond="damped_jacobi", sweeps=3)
    full, _, _ = orc.dca_solve(g.n, rp, col, w, labels, u0, outer=9, **kw)
    half, _, _ = orc.dca_solve(g.n, rp, col, w, labels, u0, outer=4, **kw)
    rest, _, _ = orc.dca_solve(g.n, rp, col, w, labels, half, outer=5, **kw)
    assert np.array_equal(full, rest)


def test_numpy_and_c_oracles_agree():
    for seed in range(4):
        g, labels, u0 = _setup(seed, n=40, K=3, p=0.15)
        rp, col, w = g.numpy()
        for kind in gl_oracle.PRECONDS:
            kw = dict(eps=1.0, c=3.0, eta=200.0, precond=kind, outer=7, sweeps=4, lambda_max=1.8)
            a, ea, ra = gl_oracle.dca_solve(g.n, rp, col, w, labels, u0, **kw)
            b, eb, rb = c_oracle.dca_solve(g.n, rp, col, w, labels, u0, **kw)
            np.testing.assert_allclose(a, b, atol=1e-14)
            np.testing.assert_allclose(ea, eb, rtol=1e-13)
            np.testing.assert_allclose(ra, rb, rtol=1e-10, atol=1e-20)


def test_labels_rule():
    U = np.array([[0.0], [-1e-300], [0.3]])
    assert list(gl_oracle.assign_labels(U)) == [1, 0, 1]
    V = np.array([[0.2, 0.2, 0.1], [-1, 0.5, 0.5], [0, 0, 1]])
    assert list(gl_oracle.assign_labels(V)) == [0, 1, 2]


# --------------------------------------------------------------------------
# the unnormalized Laplacian L = D - W (Section 2.2) and its preconditioners
# --------------------------------------------------------------------------

def _dense_L(W):
    return np.diag(W.sum(1)) - W


def test_path3_unnormalized_laplacian_explicit():
    # path 0-1-2 with unit weights: the combinatorial Laplacian, eigenvalues 0, 1, 3
    g = dense_to_graph(np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]], dtype=float))
    rp, col, w = g.numpy()
    L = gl_oracle.dense_laplacian(3, rp, col, w)
    np.testing.assert_allclose(L, [[1, -1, 0], [-1, 2, -1], [0, -1, 1]], atol=0)
    np.testing.assert_allclose(np.linalg.eigvalsh(L), [0, 1, 3], atol=1e-14)
    for orc in (gl_oracle, c_oracle):
        got = orc.laplacian_apply(3, rp, col, w, np.eye(3), laplacian="unnormalized")
        np.testing.assert_allclose(got, L, atol=0)


@pytest.mark.parametrize("orc", ORACLES)
@pytest.mark.parametrize("seed", range(6))
def test_unnormalized_laplacian_properties(orc, seed):
    rng = np.random.default_rng(100 + seed)
    g = tiny_graph(int(rng.integers(3, 24)), 0.3, rng)
    rp, col, w = g.numpy()
    W = _dense_W(g)
    d = W.sum(1)
    # L 1 = 0 (Section 2.2)
    z = orc.laplacian_apply(g.n, rp, col, w, np.ones((g.n, 1)), laplacian="unnormalized")
    assert np.abs(z).max() < 1e-13 * d.max()
    L = orc.laplacian_apply(g.n, rp, col, w, np.eye(g.n), laplacian="unnormalized")
    np.testing.assert_allclose(L, L.T, atol=1e-15)
    assert np.linalg.eigvalsh(L).min() > -1e-12 * d.max()
    # Prop. 3: 2D - L = D + W is positive semidefinite
    assert np.linalg.eigvalsh(2 * np.diag(d) - L).min() > -1e-12 * d.max()
    # L = D^{1/2} L_s D^{1/2}
    np.testing.assert_allclose(L, np.sqrt(d)[:, None] * _dense_Ls(W) * np.sqrt(d)[None, :],
                               atol=1e-13 * d.max())
    np.testing.assert_allclose(L, _dense_L(W), atol=1e-14 * d.max())
    # L scales with the weights (L_s does not)
    X = rng.standard_normal((g.n, 2))
    a = orc.laplacian_apply(g.n, rp, col, w, X, laplacian="unnormalized")
    b = orc.laplacian_apply(g.n, rp, col, 4.0 * w, X, laplacian="unnormalized")
    np.testing.assert_allclose(b, 4.0 * a, atol=1e-13 * d.max())


@pytest.mark.parametrize("orc", ORACLES)
@pytest.mark.parametrize("name,g,lam", [
    ("K5", _complete(5), 5.0),           # K_n: eigenvalue n (multiplicity n - 1)
    ("K9", _complete(9), 9.0),
    ("S6", _star(6), 6.0),               # star with m leaves: m + 1
    ("C8", _cycle(8), 4.0),              # cycle: 2 - 2 cos(2 pi j / n)
    ("C7", _cycle(7), 2 - 2 * math.cos(2 * math.pi * 3 / 7)),
])
def test_unnormalized_power_closed_form(orc, name, g, lam):
    rp, col, w = g.numpy()
    x0 = np.random.default_rng(11).uniform(-1, 1, g.n)
    rq, lhat = orc.power_max_eig(g.n, rp, col, w, x0, iters=150, laplacian="unnormalized")
    assert abs(rq - lam) < 1e-6 * lam, (name, rq, lam)
    dmax = float(_dense_W(g).sum(1).max())
    assert lhat == pytest.approx(min(2.0 * dmax, 1.01 * rq), rel=1e-15)
    # the scaled graph scales the eigenvalue
    rq3, _ = orc.power_max_eig(g.n, rp, col, 3.0 * w, x0, iters=150, laplacian="unnormalized")
    assert abs(rq3 - 3 * lam) < 3e-6 * lam


@pytest.mark.parametrize("kind", gl_oracle.PRECONDS)
@pytest.mark.parametrize("step_k", [math.inf, 0.05, 1.0, 5.0])
def test_unnormalized_preconditioner_feasible(kind, step_k):
    for seed in range(4):
        g, labels, _ = _setup(seed)
        W = 2.5 * _dense_W(g)
        d = W.sum(1)
        L = _dense_L(W)
        lam, _ = _fid(labels, 1)
        eps, c, eta = 1.7, 2.3, 50.0
        lmax = float(np.linalg.eigvalsh(L).max())
        G = np.diag(gl_oracle.precond_diag(kind, lam, eps, c, eta, 1e-3, lmax, step_k, d=d))
        T = eps * L + eta * np.diag(lam) + c * np.eye(g.n)
        if not math.isinf(step_k):
            T = np.eye(g.n) + step_k * T
        assert np.linalg.eigvalsh(G - T).min() > 0


@pytest.mark.parametrize("orc", ORACLES)
@pytest.mark.parametrize("kind", gl_oracle.PRECONDS)
@pytest.mark.parametrize("step_k", [math.inf, 0.5])
def test_unnormalized_sweeps_closed_form(orc, kind, step_k):
    for seed in range(3):
        g, labels, u0 = _setup(seed, K=1)
        rp, col, w = g.numpy()
        w = 1.7 * w
        W = 1.7 * _dense_W(g)
        d = W.sum(1)
        L = _dense_L(W)
        lam, y = _fid(labels, 1)
        eps, c, eta = 1.3, 3.0, 20.0
        lmax = float(np.linalg.eigvalsh(L).max())
        # G from its definition (Section 3.1), written here with D explicit
        el = eta * lam
        if math.isinf(step_k):
            gd = {"damped_jacobi": 2 * (eps * d + el + c), "perturbed_jacobi": 2 * eps * d + el + c + 1e-2,
                  "richardson": eps * lmax + el + c + 1e-2}[kind]
        else:
            k = step_k
            gd = {"damped_jacobi": 2 * (1 + k * (eps * d + el + c)),
                  "perturbed_jacobi": 1 + k * (2 * eps * d + el + c) + 1e-2,
                  "richardson": 1 + k * (eps * lmax + el + c) + 1e-2}[kind]
        want, _, _ = _closed_form_sweeps(L, lam, y, u0, eps, c, eta, gd, 3, step_k)
        U, _, _ = orc.dca_solve(g.n, rp, col, w, labels, u0, eps=eps, c=c, eta=eta, precond=kind,
                                outer=1, sweeps=3, delta0=1e-2, lambda_max=lmax, step_k=step_k,
                                laplacian="unnormalized")
        np.testing.assert_allclose(U, want, atol=1e-12)


@pytest.mark.parametrize("orc", ORACLES)
@pytest.mark.parametrize("kind", gl_oracle.PRECONDS)
def test_unnormalized_energy_decreases(orc, kind):
    for seed in range(4):
        g, labels, u0 = _setup(seed, n=20, K=2)
        rp, col, w = g.numpy()
        eps, c, eta = 1.0, 3.0, 100.0
        W = _dense_W(g)
        lmax = float(np.linalg.eigvalsh(_dense_L(W)).max())
        U, en, _ = orc.dca_solve(g.n, rp, col, w, labels, u0, eps=eps, c=c, eta=eta,
                                 precond=kind, outer=25, sweeps=2, delta0=1e-6,
                                 lambda_max=lmax, laplacian="unnormalized")
        assert _convexity_ok(U, eps, c)
        assert np.all(np.diff(en, axis=0) <= 1e-12 * np.abs(en[:-1]))
        # the energy with L written as a double sum: u^T L u = 1/2 sum w_ij (u_i - u_j)^2
        for k in range(2):
            x = U[:, k]
            lap = 0.5 * np.sum(W * (x[:, None] - x[None, :]) ** 2)
            lam, y = _fid(labels, 2)
            want = (eps / 2) * lap + np.sum((x ** 2 - 1) ** 2) / (4 * eps) \
                + (eta / 2) * np.sum(lam * (x - y[:, k]) ** 2)
            assert en[-1, k] == pytest.approx(want, rel=1e-12)


# --------------------------------------------------------------------------
# second eigenpair (unsupervised initialisation, Section 5.2)
# --------------------------------------------------------------------------

def _path(n):
    W = np.zeros((n, n))
    for i in range(n - 1):
        W[i, i + 1] = W[i + 1, i] = 1.0
    return dense_to_graph(W)


@pytest.mark.parametrize("n", [5, 9, 16])
def test_second_eigenpair_path_closed_form(n):
    g = _path(n)
    rp, col, w = g.numpy()
    d = _dense_W(g).sum(1)
    # L_s of the path: lambda_2 = 1 - cos(pi/(n-1)), v_2 ~ D^{1/2} cos(pi j/(n-1))
    lam, v = gl_oracle.second_eigenpair(n, rp, col, w)
    want = np.sqrt(d) * np.cos(np.pi * np.arange(n) / (n - 1))
    want /= np.linalg.norm(want)
    assert lam == pytest.approx(1 - math.cos(math.pi / (n - 1)), abs=1e-13)
    assert abs(abs(v @ want) - 1) < 1e-12
    # L of the path: lambda_2 = 2 - 2 cos(pi/n), v_2 ~ cos(pi (j + 1/2)/n)
    lam, v = gl_oracle.second_eigenpair(n, rp, col, w, laplacian="unnormalized")
    want = np.cos(np.pi * (np.arange(n) + 0.5) / n)
    want /= np.linalg.norm(want)
    assert lam == pytest.approx(2 - 2 * math.cos(math.pi / n), abs=1e-13)
    assert abs(abs(v @ want) - 1) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_second_eigenpair_invariants(seed):
    rng = np.random.default_rng(300 + seed)
    g = tiny_graph(int(rng.integers(6, 30)), 0.3, rng)
    rp, col, w = g.numpy()
    W = _dense_W(g)
    d = W.sum(1)
    lam, v = gl_oracle.second_eigenpair(g.n, rp, col, w)
    assert np.linalg.norm(v) == pytest.approx(1.0, abs=1e-13)
    assert abs(v @ np.sqrt(d)) < 1e-10 * np.linalg.norm(np.sqrt(d))   # v_2 _|_ D^{1/2} 1
    np.testing.assert_allclose(_dense_Ls(W) @ v, lam * v, atol=1e-12)
    assert v[np.argmax(np.abs(v))] > 0
    # the smallest eigenvalue on the complement of the null vector (Courant-Fischer)
    ev = np.linalg.eigvalsh(_dense_Ls(W))
    assert lam == pytest.approx(ev[1], abs=1e-13)
    u0 = gl_oracle.unsupervised_u0(v)
    assert np.abs(u0).max() == pytest.approx(1.0)


def test_second_eigenvector_splits_a_barbell():
    # two 5-cliques joined by one edge: the sign of v_2 separates the cliques
    W = np.zeros((10, 10))
    W[:5, :5] = 1.0
    W[5:, 5:] = 1.0
    np.fill_diagonal(W, 0.0)
    W[4, 5] = W[5, 4] = 1.0
    g = dense_to_graph(W)
    rp, col, w = g.numpy()
    _, v = gl_oracle.second_eigenpair(10, rp, col, w)
    s = np.sign(v)
    assert len(set(s[:5])) == 1 and len(set(s[5:])) == 1 and s[0] != s[9]


def test_second_eigenpair_disconnected_closed_form():
    # two disjoint cliques A (4 nodes) and B (6 nodes): lambda_2 = 0 and v_2 is
    # the null vector orthogonal to D^{1/2} 1: D^{1/2} (vol_B 1_A - vol_A 1_B)
    W = np.zeros((10, 10))
    W[:4, :4] = 1.0
    W[4:, 4:] = 2.0
    np.fill_diagonal(W, 0.0)
    g = dense_to_graph(W)
    rp, col, w = g.numpy()
    d = W.sum(1)
    vol_a, vol_b = d[:4].sum(), d[4:].sum()
    want = np.sqrt(d) * np.r_[np.full(4, vol_b), np.full(6, -vol_a)]
    want /= np.linalg.norm(want)
    lam, v = gl_oracle.second_eigenpair(10, rp, col, w)
    assert abs(lam) < 1e-13
    assert abs(abs(v @ want) - 1) < 1e-12
    # unnormalized: v_2 ~ 6 * 1_A - 4 * 1_B (orthogonal to 1)
    lam, v = gl_oracle.second_eigenpair(10, rp, col, w, laplacian="unnormalized")
    want = np.r_[np.full(4, 6.0), np.full(6, -4.0)]
    want /= np.linalg.norm(want)
    assert abs(lam) < 1e-12
    assert abs(abs(v @ want) - 1) < 1e-12
