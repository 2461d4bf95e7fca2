"""Reduced-precision runs of the preconditioned DCA on the CPU: the floor of
the parity tolerances.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The steps are those of
``gl_oracle.dca_solve`` (Prop. 1 with finitely many diagonal sweeps, Section
3.1, on L_s of Section 2.2), carried out the way a reduced-precision
implementation has to carry them out:

  * the normalized weights w_ij / (sqrt(d_i) sqrt(d_j)) are formed in float64
    and rounded once to the weight storage type;
  * the field u^t and every sweep's v are rounded to the field storage type
    when they are stored;
  * products, sums and the update are float32 (round to nearest even after
    every operation).

Nothing here is taken from the GPU library: it is the algorithm with its
numbers rounded, so the gap between its result and the float64 oracle's is
what rounding alone does to the iteration.  A GPU result can be expected
within a small multiple of that gap, not closer (its sums run in another
order, so it rounds differently).

Rounding to bfloat16 (8 significant bits) and to float16 (11) is round to
nearest, ties to even, applied once to the exact value.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import gl_oracle


def _round_f64_bits(x: np.ndarray, drop: int) -> np.ndarray:
    """Round float64 values to 52 - drop stored significand bits (nearest,
    ties to even) on the bit pattern.  Valid for normal results."""
    b = np.ascontiguousarray(x, dtype=np.float64).view(np.uint64).copy()
    half = np.uint64((1 << (drop - 1)) - 1)
    b += half + ((b >> np.uint64(drop)) & np.uint64(1))
    b &= ~np.uint64((1 << drop) - 1)
    return b.view(np.float64)


def round_to(x: np.ndarray, store: str) -> np.ndarray:
    """x (float64 or float32) rounded once to `store`, returned as float32
    (every bf16, f16 and f32 value is exact in float32)."""
    x = np.asarray(x)
    if store == "f32":
        return x.astype(np.float32)
    if store == "f16":
        return x.astype(np.float16).astype(np.float32)
    if store == "bf16":
        if x.dtype == np.float64:
            y = _round_f64_bits(x, 45)
            small = np.abs(x) < 2.0 ** -126
            out = y.astype(np.float32)
            if np.any(small):  # subnormal range: round to the bfloat16 quantum
                q = 2.0 ** -133
                out[small] = (np.rint(x[small] / q) * q).astype(np.float32)
            return out
        b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).copy()
        b += np.uint32(0x7FFF) + ((b >> np.uint32(16)) & np.uint32(1))
        b &= np.uint32(0xFFFF0000)
        return b.view(np.float32)
    raise ValueError(f"unknown storage type {store}")


def dca_solve_rounded(n, row_ptr, col, w, labels, u0, *, eps, c, eta, precond, outer,
                      sweeps, store_w="f32", store_u="f32", delta0=1e-6, lambda_max=2.0,
                      step_k=math.inf):
    """The DCA of gl_oracle.dca_solve with stored values rounded to
    store_w / store_u and float32 arithmetic; returns U [n, K] (float64 copy
    of the stored float32 values)."""
    U = np.array(u0, dtype=np.float64, copy=True)
    if U.ndim == 1:
        U = U[:, None]
    K = U.shape[1]
    wh = round_to(gl_oracle.normalized_weights(n, row_ptr, col, w), store_w)
    A = sp.csr_matrix((wh, col.astype(np.int64), row_ptr.astype(np.int64)), shape=(n, n))
    lam64, y64 = gl_oracle.fidelity(labels, K)
    lam = lam64.astype(np.float32)[:, None]
    y = y64.astype(np.float32)
    g = gl_oracle.precond_diag(precond, lam64, eps, c, eta, delta0, lambda_max, step_k)
    ginv = (1.0 / np.asarray(g, dtype=np.float64)).astype(np.float32)[:, None] \
        * np.ones((1, 1), np.float32)
    f = np.float32
    e32, c32, eta32, ie32 = f(eps), f(c), f(eta), f(1.0 / eps)
    finite = not math.isinf(step_k)
    alpha, kappa = (f(1.0), f(step_k)) if finite else (f(0.0), f(1.0))
    Ut = round_to(U, store_u)
    for _ in range(outer):
        u = Ut
        rhs = c32 * u - (u * u * u - u) * ie32 + eta32 * lam * y
        v = u
        for _ in range(sweeps):
            z = A @ v                      # float32 products and sums
            tv = e32 * (v - z) + (eta32 * lam + c32) * v
            r = alpha * (u - v) + kappa * (rhs - tv)
            v = round_to(v + r * ginv, store_u)
        Ut = v
    return Ut.astype(np.float64)


def gap(U_rounded: np.ndarray, U_exact: np.ndarray, n, row_ptr, col, w, labels, eps, eta):
    """Distance of a reduced-precision result from the float64 one: max |dU|,
    argmax label agreement, the 99.9th percentile of |dU| and the relative
    difference of the float64 energies of the two fields (Section 2.1)."""
    d = np.abs(U_rounded - U_exact)
    agree = float(np.mean(gl_oracle.assign_labels(U_rounded) == gl_oracle.assign_labels(U_exact)))
    Fa = gl_oracle.energy(n, row_ptr, col, w, U_rounded, labels, eps, eta)
    Fb = gl_oracle.energy(n, row_ptr, col, w, U_exact, labels, eps, eta)
    return {"max_abs_dU": float(d.max()), "p999_abs_dU": float(np.quantile(d, 0.999)),
            "label_agreement": agree,
            "energy_rel_diff": float(np.max(np.abs(Fa - Fb)) / max(np.max(np.abs(Fb)), 1e-300))}
