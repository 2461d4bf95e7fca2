"""GPU parity of the unnormalized Laplacian L = D - W (Section 2.2) and its
D-dependent preconditioners (Section 3.1) against the float64 oracle.

The operator stores the weights rounded to its storage type and, as its
diagonal, the row sums of the stored weights; the oracle uses the exact
weights and degrees.  Tolerances are those of the normalized path, scaled by
the largest degree where a value scales with the weights.
"""

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import torch

import paper_2303_14495_amd as gl
from oracle import c_oracle, gl_oracle
from synth.graphs import dense_to_graph, tiny_graph
from tests.gpu_helpers import (DEV, gpu_solve, label_agreement, make_operator, oracle_lambda,
                               oracle_solve, power_x0, problem, say)
from tests.test_gpu_parity import _cycle, _lattice

pytestmark = pytest.mark.gpu

UN = "unnormalized"
DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}


def _graph_problem(g):
    P = type("P", (), {})()
    P.graph = g
    P.n = g.n
    return P


def test_two_node_golden_unnormalized_f64():
    gd = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                     "two_node_unnormalized.json")))
    rp = torch.tensor(gd["graph"]["row_ptr"], dtype=torch.int64, device=DEV)
    col = torch.tensor(gd["graph"]["col"], dtype=torch.int32, device=DEV)
    w = torch.tensor(gd["graph"]["weight"], dtype=torch.float64, device=DEV)
    op = gl.Operator(rp, col, w, store_w="f64", laplacian=UN)
    lab = torch.tensor(gd["labels"], dtype=torch.int32, device=DEV)
    for case in gd["cases"]:
        say(f"two-node unnormalized golden case {case['name']}")
        U = torch.tensor(gd["u0"], dtype=torch.float64, device=DEV).view(2, 1).contiguous()
        k = math.inf if case["step_k"] == "inf" else float(case["step_k"])
        st = op.solve(lab, U, eps=gd["eps"], c=gd["c"], eta=gd["eta"], precond=case["precond"],
                      outer=case["outer"], sweeps=case["sweeps"], delta0=case["delta0"],
                      lambda_max=case["lambda_max"], step_k=k)
        want = np.array([float(Fraction(x)) for x in case["u"]])
        np.testing.assert_allclose(U.cpu().numpy()[:, 0], want, rtol=0, atol=4e-15)
        e, r, flag = gl.split_stats(st.cpu(), 1, case["outer"], case["sweeps"])
        if "residual_sq" in case:
            rr = np.array([[float(Fraction(x)) for x in row] for row in case["residual_sq"]])
            np.testing.assert_allclose(r.numpy()[:, :, 0], rr, rtol=1e-14)
        if "energies" in case:
            ee = np.array([float(Fraction(x)) for x in case["energies"]])
            np.testing.assert_allclose(e.numpy()[:, 0], ee, rtol=1e-14)
        assert flag == 0.0


@pytest.mark.parametrize("store", [("f64", "f64"), ("f32", "f32"), ("bf16", "f16")])
@pytest.mark.parametrize("K", [1, 4, 16])
def test_unnormalized_laplacian_ragged(store, K):
    store_w, store_u = store
    rng = np.random.default_rng(50 + K)
    g = tiny_graph(1037, 0.01, rng)
    say(f"unnormalized laplacian n=1037 K={K} store={store}")
    op = make_operator(_graph_problem(g), store_w, laplacian=UN)
    X = torch.from_numpy(rng.uniform(-1, 1, (g.n, K))).to(DEV, torch.float64).to(
        DT[store_u]).contiguous()
    Y = op.laplacian_apply(X).to(torch.float64).cpu().numpy()
    rp, col, w = g.numpy()
    ref = gl_oracle.laplacian_apply(g.n, rp, col, w, X.to(torch.float64).cpu().numpy(),
                                    laplacian=UN)
    dmax = float(gl_oracle.degrees(g.n, rp, col, w).max())
    tol = {"f64": 1e-13, "f32": 2e-6}.get(store_u, 3e-2) * max(1.0, dmax)
    assert np.abs(Y - ref).max() <= tol, np.abs(Y - ref).max()
    # L 1 = 0 up to the rounding of the stored weights' row sums
    ones = torch.ones((g.n, K), dtype=DT[store_u], device=DEV)
    z = op.laplacian_apply(ones).to(torch.float64).abs().max().item()
    assert z <= {"f64": 1e-13, "f32": 1e-5}.get(store_u, 2e-2) * max(1.0, dmax)


@pytest.mark.parametrize("store", [("f64", "f64"), ("f32", "f32"), ("bf16", "f16")])
@pytest.mark.parametrize("K", [1, 4])
def test_unnormalized_laplacian_tile(store, K):
    store_w, store_u = store
    p = _lattice(96, 80, K) if store_w == "f64" else problem(4, small=True)
    say(f"unnormalized tile laplacian n={p.n} K={K} store={store}")
    op = make_operator(p, store_w, layout="tile", laplacian=UN)
    assert op.info()["layout"] == "tile"
    rng = np.random.default_rng(200 + K)
    X = torch.from_numpy(rng.uniform(-1, 1, (p.n, K))).to(DEV, torch.float64).to(
        DT[store_u]).contiguous()
    Y = op.laplacian_apply(X).to(torch.float64).cpu().numpy()
    rp, col, w = p.graph.numpy()
    ref = gl_oracle.laplacian_apply(p.n, rp, col, w, X.to(torch.float64).cpu().numpy(),
                                    laplacian=UN)
    dmax = float(gl_oracle.degrees(p.n, rp, col, w).max())
    tol = {("f64", "f64"): 1e-13, ("f32", "f32"): 2e-6}.get(store, 3e-2) * max(1.0, dmax)
    assert np.abs(Y - ref).max() <= tol, np.abs(Y - ref).max()


@pytest.mark.parametrize("name,g,lam", [
    ("K9", dense_to_graph(np.ones((9, 9)) - np.eye(9)), 9.0),
    ("C8", _cycle(8), 4.0),
    ("C7", _cycle(7), 2 - 2 * math.cos(2 * math.pi * 3 / 7)),
])
def test_unnormalized_power_closed_form(name, g, lam):
    say(f"unnormalized power method {name}")
    op = make_operator(_graph_problem(g), "f32", laplacian=UN)
    x0 = torch.from_numpy(power_x0(g.n, 3)).to(DEV, torch.float32)
    rq, lhat = op.power_max_eig(x0, 150)
    assert abs(rq - lam) <= 1e-5 * lam, (rq, lam)
    dmax = float(np.diff(g.numpy()[0]).max())  # unit weights: the largest row length
    assert lhat == pytest.approx(min(2.0 * dmax, 1.01 * rq), rel=1e-6)


@pytest.mark.parametrize("cfg,layout", [(1, "auto"), (2, "tile")])
def test_unnormalized_power_vs_oracle(cfg, layout):
    p = problem(cfg, small=(cfg == 2))
    say(f"unnormalized power method vs oracle, {p.name}")
    rq_o, lam_o = oracle_lambda(p, laplacian=UN)
    op = make_operator(p, "f32", layout=layout, laplacian=UN)
    rq, lam = op.power_max_eig(torch.from_numpy(power_x0(p.n, p.seed)).to(DEV, torch.float32), 150)
    assert abs(rq - rq_o) <= 1e-4 * rq_o, (rq, rq_o)
    assert abs(lam - lam_o) <= 1e-4 * lam_o


def _check(p, store_w, store_u, tol, precond=None, step_k=None, layout="auto", lam=None):
    precond = precond or p.precond
    if lam is None:
        lam = oracle_lambda(p, laplacian=UN)[1] if precond == "richardson" else 2.0
    say(f"unnormalized solve {p.name} w={store_w} u={store_u} {precond} k={step_k} "
        f"layout={layout} lambda={lam:.4f}")
    op = make_operator(p, store_w, layout=layout, laplacian=UN)
    Ug, eg, rg, flag, _ = gpu_solve(p, store_w, store_u, lambda_max=lam, op=op, precond=precond,
                                    step_k=step_k)
    Uo, eo, ro = oracle_solve(p, lambda_max=lam, laplacian=UN, precond=precond, step_k=step_k)
    err = float(np.abs(Ug - Uo).max())
    agree = label_agreement(Ug, Uo)
    e_rel = float(np.abs(eg - eo).max() / np.abs(eo).max())
    say(f"  max|dU| = {err:.3e}  label agreement = {agree:.6f}  energy rel = {e_rel:.3e}")
    assert flag == 0.0
    assert err <= tol
    assert agree >= 0.999
    assert e_rel <= (1e-10 if store_u == "f64" else 1e-4 if store_u == "f32" else 2e-2)


def test_unnormalized_solve_cfg1_f64():
    _check(problem(1), "f64", "f64", 1e-10)


@pytest.mark.parametrize("precond", ["damped_jacobi", "perturbed_jacobi", "richardson"])
def test_unnormalized_solve_cfg1_f32(precond):
    _check(problem(1), "f32", "f32", 1e-5, precond=precond)


def test_unnormalized_solve_cfg1_step_k():
    _check(problem(1), "f32", "f32", 1e-5, step_k=0.5)


def test_unnormalized_solve_cfg2_tile_f32():
    _check(problem(2, small=True), "f32", "f32", 1e-5, layout="tile")


def test_unnormalized_solve_cfg4_small_bf16():
    _check(problem(4, small=True), "bf16", "f16", 2e-2, layout="tile")


def test_unnormalized_differs_from_normalized():
    # the two Laplacians give different operators on a non-regular graph
    p = problem(1)
    a = make_operator(p, "f32", laplacian=UN)
    b = make_operator(p, "f32")
    X = torch.from_numpy(np.random.default_rng(1).uniform(-1, 1, (p.n, 1))).to(
        DEV, torch.float32)
    assert (a.laplacian_apply(X) - b.laplacian_apply(X)).abs().max().item() > 1e-2
