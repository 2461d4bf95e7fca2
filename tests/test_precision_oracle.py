"""Pins of the reduced-precision emulation (oracle/precision.py), which sets
the floor of the parity tolerances: its rounding against exact tie cases and
library conversions, its arithmetic against the float64 oracle where
rounding cannot matter, and the invariants a correct rounding keeps."""

import math

import numpy as np
import pytest
import torch

from oracle import gl_oracle, precision
from synth.graphs import dense_to_graph


def test_bf16_rounding_ties_and_library():
    one = 1.0
    x = np.array([one + 2.0 ** -8,            # tie between 1 and 1 + 2^-7 -> even (1)
                  one + 3 * 2.0 ** -8,        # tie between 1 + 2^-7 and 1 + 2^-6 -> 1 + 2^-6
                  one + 2.0 ** -8 + 2.0 ** -40,   # just above the tie -> up
                  -(one + 2.0 ** -8 + 2.0 ** -40),
                  3.0e-39])                   # bfloat16 subnormal range
    got = precision.round_to(x, "bf16").astype(np.float64)
    assert got[0] == 1.0
    assert got[1] == 1.0 + 2.0 ** -6
    assert got[2] == 1.0 + 2.0 ** -7 and got[3] == -(1.0 + 2.0 ** -7)
    q = 2.0 ** -133
    assert got[4] == round(3.0e-39 / q) * q
    # float32 inputs: torch's conversion (round to nearest even)
    r = np.random.default_rng(0).standard_normal(4096).astype(np.float32) * 3
    want = torch.from_numpy(r).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(precision.round_to(r, "bf16"), want)
    # float64 inputs exactly representable in float32: the same
    assert np.array_equal(precision.round_to(r.astype(np.float64), "bf16"), want)


def test_f16_rounding_is_single():
    # 1 + 2^-11 is the tie between 1 and 1 + 2^-10; a hair above it must round
    # up even though float32 would first round it onto the tie
    x = np.array([1.0 + 2.0 ** -11 + 2.0 ** -40, 1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11])
    got = precision.round_to(x, "f16").astype(np.float64)
    assert got[0] == 1.0 + 2.0 ** -10
    assert got[1] == 1.0
    assert got[2] == 1.0 + 2.0 ** -9


def _mixture(n=600, seed=3):
    rng = np.random.default_rng(seed)
    from synth.graphs import knn_bruteforce, self_tuning_graph
    x = torch.from_numpy(np.concatenate([rng.standard_normal((n // 2, 5)) + 1.5,
                                         rng.standard_normal((n - n // 2, 5)) - 1.5]))
    g = self_tuning_graph(x, knn_bruteforce(x, 8))
    labels = np.full(n, -1, np.int32)
    pick = rng.choice(n, n // 10, replace=False)
    labels[pick] = (pick < n // 2).astype(np.int32)
    return g, labels


@pytest.mark.parametrize("kw", [
    dict(eps=100.0, c=11.0, eta=100.0, precond="damped_jacobi"),
    dict(eps=100.0, c=11.0, eta=100.0, precond="richardson", lambda_max=1.7),
    dict(eps=2.0, c=5.0, eta=50.0, precond="perturbed_jacobi", step_k=0.5),
])
def test_f32_run_matches_oracle(kw):
    # float32 storage and arithmetic on a contracting problem: within a few
    # float32 units of the float64 oracle; a wrong sign, a dropped term or a
    # wrong preconditioner in the emulation would be off by orders more
    g, labels = _mixture()
    rp, col, w = g.numpy()
    n = rp.size - 1
    u0 = np.where(labels == 1, 1.0, np.where(labels == 0, -1.0, 0.0))[:, None]
    sched = dict(outer=6, sweeps=4)
    U64, _, _ = gl_oracle.dca_solve(n, rp, col, w, labels, u0, **kw, **sched)
    U32 = precision.dca_solve_rounded(n, rp, col, w, labels, u0, **kw, **sched)
    assert np.abs(U32 - U64).max() <= 2e-6
    assert np.abs(U32 - U64).max() > 0.0       # it really rounds
    # bf16 storage stays within the bf16 bar on this contracting problem
    Ub = precision.dca_solve_rounded(n, rp, col, w, labels, u0, store_w="bf16",
                                     store_u="bf16", **kw, **sched)
    assert 1e-4 < np.abs(Ub - U64).max() <= 2e-2


def test_fixed_point_exact_in_every_storage():
    # unweighted cycle: w_hat = 1/2 exactly, L_s 1 = 0; all nodes class 1 and
    # u^0 = 1 is a fixed point of every sweep, exactly in any rounding
    n = 12
    W = np.zeros((n, n))
    for i in range(n):
        W[i, (i + 1) % n] = W[(i + 1) % n, i] = 1.0
    g = dense_to_graph(W)
    rp, col, w = g.numpy()
    labels = np.ones(n, np.int32)
    u0 = np.ones((n, 1))
    for sw, su in [("f32", "f32"), ("bf16", "bf16"), ("bf16", "f16")]:
        U = precision.dca_solve_rounded(n, rp, col, w, labels, u0, eps=1.0, c=3.0, eta=10.0,
                                        precond="damped_jacobi", outer=3, sweeps=2,
                                        store_w=sw, store_u=su)
        assert np.array_equal(U, u0)


def test_sign_symmetry_bitwise():
    # round to nearest even is symmetric, and so is every step: flipping the
    # labels and negating u^0 negates the result bit for bit
    g, labels = _mixture(300, seed=5)
    rp, col, w = g.numpy()
    n = rp.size - 1
    u0 = np.random.default_rng(1).uniform(-1, 1, (n, 1))
    flip = np.where(labels >= 0, 1 - labels, -1).astype(np.int32)
    kw = dict(eps=1.0, c=3.0, eta=1000.0, precond="damped_jacobi", outer=5, sweeps=3,
              store_w="bf16", store_u="bf16")
    A = precision.dca_solve_rounded(n, rp, col, w, labels, u0, **kw)
    B = precision.dca_solve_rounded(n, rp, col, w, flip, -u0, **kw)
    assert np.array_equal(A, -B)


def test_gap_measures():
    g, labels = _mixture(200, seed=7)
    rp, col, w = g.numpy()
    n = rp.size - 1
    U = np.random.default_rng(2).uniform(-1, 1, (n, 3))
    z = precision.gap(U, U, n, rp, col, w, labels, 1.0, 10.0)
    assert z["max_abs_dU"] == 0.0 and z["label_agreement"] == 1.0 and z["energy_rel_diff"] == 0.0
    V = U.copy()
    V[0] += 0.5
    z = precision.gap(V, U, n, rp, col, w, labels, 1.0, 10.0)
    assert math.isclose(z["max_abs_dU"], 0.5, rel_tol=1e-12) and z["energy_rel_diff"] > 0
