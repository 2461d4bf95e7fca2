"""Float64 numpy oracle of the preconditioned DCA inner solve.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function cites
the passage of the paper it writes out; "Prop. 1" is the proposition turning
the proximal DCA into the preconditioned iteration u + M^{-1}(b - T u),
"Prop. 3" the bounds 2D >= L and 2I >= L_s, "Thm. 1" the energy decay.

Readings of points the paper leaves open (each also listed in the design
notes of the repository):
  * energy: F(u) = (eps/2) u^T L_s u + (1/(4 eps)) sum (u^2 - 1)^2
    + (eta/2) sum Lambda (u - y)^2, i.e. GL(u) of Section 2.1 with <u, L u>
    replaced by <u, L_s u>; this is the functional whose gradient gives
    T = eps L_s + eta Lambda + c I (Section 3);
  * inner sweeps: b^t is fixed during a DCA step, the sweeps start from u^t
    and every sweep uses only old values (Jacobi form of the diagonal
    preconditioned iteration, Section 3.1);
  * labels: K = 1 encodes class 1 as y = +1 and class 0 as y = -1; K >= 2
    uses one-vs-rest +-1 columns with a double well per column;
    Lambda_i = 1 iff node i is labelled;
  * Richardson: lambda_hat = min(2, 1.01 * Rayleigh quotient) after the power
    iterations, feasible because 2I >= L_s (Prop. 3); for the unnormalized L
    the cap is 2 max_i d_i, since L <= 2D (Prop. 3);
  * the unnormalized Laplacian L = D - W (Section 2.2) replaces L_s in the
    energy and in T = eps L + eta Lambda + c I, with the D-dependent
    preconditioners G_Jd, G_Jp, G_R and their step-size-k versions of
    Section 3.1.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

PRECONDS = ("damped_jacobi", "perturbed_jacobi", "richardson")
LAPLACIANS = ("normalized", "unnormalized")


# ---------------------------------------------------------------------------
# graph operator (Section 2.2)
# ---------------------------------------------------------------------------

def degrees(n, row_ptr, col, w):
    """d_i = sum_j w_ij (Section 2.2, the degree matrix D)."""
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    return np.bincount(rows, weights=w, minlength=n).astype(np.float64)


def normalized_weights(n, row_ptr, col, w):
    """Entries of D^{-1/2} W D^{-1/2}, the off-diagonal part of
    L_s = I - D^{-1/2} W D^{-1/2} (Section 2.2)."""
    d = degrees(n, row_ptr, col, w)
    if np.any(d <= 0):
        raise ValueError("every degree must be positive")
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    return w / (np.sqrt(d[rows]) * np.sqrt(d[col.astype(np.int64)]))


def normalized_adjacency(n, row_ptr, col, w):
    """scipy CSR of D^{-1/2} W D^{-1/2}."""
    wh = normalized_weights(n, row_ptr, col, w)
    return sp.csr_matrix((wh, col.astype(np.int64), row_ptr.astype(np.int64)), shape=(n, n))


def operator_parts(n, row_ptr, col, w, laplacian="normalized"):
    """(A, dd) with the Laplacian written as diag(dd) - A (Section 2.2):
    normalized   L_s = I - D^{-1/2} W D^{-1/2}:  A = D^{-1/2} W D^{-1/2}, dd = 1;
    unnormalized L   = D - W:                    A = W,                 dd = d."""
    if laplacian == "normalized":
        return normalized_adjacency(n, row_ptr, col, w), np.ones(n)
    if laplacian == "unnormalized":
        d = degrees(n, row_ptr, col, w)
        if np.any(d <= 0):
            raise ValueError("every degree must be positive")
        W = sp.csr_matrix((np.asarray(w, dtype=np.float64), col.astype(np.int64),
                           row_ptr.astype(np.int64)), shape=(n, n))
        return W, d
    raise ValueError(f"unknown laplacian {laplacian}")


def laplacian_apply(n, row_ptr, col, w, X, laplacian="normalized"):
    """L_s X = X - D^{-1/2} W D^{-1/2} X, or L X = D X - W X (Section 2.2);
    X is n x K."""
    A, dd = operator_parts(n, row_ptr, col, w, laplacian)
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        return dd * X - A @ X
    return dd[:, None] * X - A @ X


def dense_laplacian(n, row_ptr, col, w):
    """Dense unnormalized L = D - W built entry by entry (tiny graphs)."""
    W = np.zeros((n, n))
    for i in range(n):
        for p in range(row_ptr[i], row_ptr[i + 1]):
            W[i, col[p]] = w[p]
    return np.diag(W.sum(1)) - W


def dense_normalized_laplacian(n, row_ptr, col, w):
    """Dense L_s built entry by entry from its definition (tiny graphs)."""
    W = np.zeros((n, n))
    for i in range(n):
        for p in range(row_ptr[i], row_ptr[i + 1]):
            W[i, col[p]] = w[p]
    d = W.sum(1)
    Dm = np.diag(1.0 / np.sqrt(d))
    return np.eye(n) - Dm @ W @ Dm


# ---------------------------------------------------------------------------
# fidelity data, right-hand side, preconditioner
# ---------------------------------------------------------------------------

def fidelity(labels, K):
    """Lambda (n,) and y (n, K) from the label vector (Section 2.1: Lambda_i = 1
    on nodes with a known prior label, 0 elsewhere; y the known labels)."""
    labels = np.asarray(labels)
    n = labels.size
    lam = (labels >= 0).astype(np.float64)
    y = np.zeros((n, K))
    if K == 1:
        y[:, 0] = np.where(labels == 1, 1.0, np.where(labels == 0, -1.0, 0.0))
    else:
        lab = labels >= 0
        y[lab, :] = -1.0
        y[np.flatnonzero(lab), labels[lab]] = 1.0
    return lam, y


def double_well_grad(u, eps):
    """Gradient of (1/eps) sum W(u_i), W(u) = (u^2 - 1)^2 / 4 (Section 2.1)."""
    return (u ** 3 - u) / eps


def rhs(u, lam, y, eps, c, eta):
    """b^t = c u^t - grad W(u^t) + eta Lambda y (Prop. 1, and the DCA linear
    system T u^{t+1} = b^t of Section 3)."""
    return c * u - double_well_grad(u, eps) + eta * lam[:, None] * y


def precond_diag(kind, lam, eps, c, eta, delta0=1e-6, lambda_max=2.0, step_k=math.inf, d=None):
    """Diagonal g of the feasible preconditioners (Section 3.1).

    Normalized Laplacian (d is None): for infinite step size
        G_Jd,s = 2(eps + eta Lambda + c),  G_Jp,s = 2 eps + eta Lambda + c + delta0,
        G_R,s  = eps lambda_max + eta Lambda + c + delta0;
    for a finite step size k the T_k versions
        G_Jd,ks = 2(1 + k(eps + c) + k eta Lambda),
        G_Jp,ks = (2 k eps + 1) + k(eta Lambda + c) + delta0,
        G_R,ks  = 1 + k(eps lambda_max + eta Lambda + c) + delta0.
    Unnormalized Laplacian (d the degrees): for infinite step size
        G_Jd = 2(eps D + eta Lambda + c),  G_Jp = 2 eps D + eta Lambda + c + delta0,
        G_R  = eps lambda_max + eta Lambda + c + delta0;
    and for a finite step size k
        G_Jd,k = 2(1 + k(eps D + eta Lambda + c)),
        G_Jp,k = 1 + k(2 eps D + eta Lambda + c) + delta0,
        G_R,k  = 1 + k(eps lambda_max + eta Lambda + c) + delta0."""
    el = eta * lam
    if d is None:
        if math.isinf(step_k):
            if kind == "damped_jacobi":
                return 2.0 * (eps + el + c)
            if kind == "perturbed_jacobi":
                return 2.0 * eps + el + c + delta0
            if kind == "richardson":
                return eps * lambda_max + el + c + delta0
        else:
            k = step_k
            if kind == "damped_jacobi":
                return 2.0 * (1.0 + k * (eps + c) + k * el)
            if kind == "perturbed_jacobi":
                return (2.0 * k * eps + 1.0) + k * (el + c) + delta0
            if kind == "richardson":
                return 1.0 + k * (eps * lambda_max + el + c) + delta0
        raise ValueError(f"unknown preconditioner {kind}")
    d = np.asarray(d, dtype=np.float64)
    if math.isinf(step_k):
        if kind == "damped_jacobi":
            return 2.0 * (eps * d + el + c)
        if kind == "perturbed_jacobi":
            return 2.0 * eps * d + el + c + delta0
        if kind == "richardson":
            return eps * lambda_max + el + c + delta0 + 0.0 * d
    else:
        k = step_k
        if kind == "damped_jacobi":
            return 2.0 * (1.0 + k * (eps * d + el + c))
        if kind == "perturbed_jacobi":
            return 1.0 + k * (2.0 * eps * d + el + c) + delta0
        if kind == "richardson":
            return 1.0 + k * (eps * lambda_max + el + c) + delta0 + 0.0 * d
    raise ValueError(f"unknown preconditioner {kind}")


# ---------------------------------------------------------------------------
# energy (Section 2.1)
# ---------------------------------------------------------------------------

def energy(n, row_ptr, col, w, U, labels, eps, eta, laplacian="normalized"):
    """F(u) per column: (eps/2) u^T L_s u (or u^T L u) + (1/eps) sum W(u_i)
    + (eta/2) sum Lambda_i (u_i - y_i)^2 (Section 2.1)."""
    U = np.asarray(U, dtype=np.float64)
    if U.ndim == 1:
        U = U[:, None]
    K = U.shape[1]
    lam, y = fidelity(labels, K)
    LU = laplacian_apply(n, row_ptr, col, w, U, laplacian)
    lap = 0.5 * eps * (U * LU).sum(0)
    well = ((U ** 2 - 1.0) ** 2).sum(0) / (4.0 * eps)
    fid = 0.5 * eta * (lam[:, None] * (U - y) ** 2).sum(0)
    return lap + well + fid


# ---------------------------------------------------------------------------
# preconditioned DCA (Prop. 1 with finitely many diagonal sweeps, Section 3.1)
# ---------------------------------------------------------------------------

def dca_solve(n, row_ptr, col, w, labels, u0, *, eps, c, eta, precond, outer, sweeps,
              delta0=1e-6, lambda_max=2.0, step_k=math.inf, record=True,
              laplacian="normalized"):
    """Run `outer` DCA steps of `sweeps` preconditioned sweeps each.

    Returns (U [n, K], energies [outer + 1, K], residual_sq [outer, sweeps, K])
    where energies[t] = F(u^t) and residual_sq[t, s] = ||r||^2 of the residual
    r = b - T v (infinite step) or r = b_k - T_k v (finite step k) that sweep s
    of step t divides by g.
    """
    U = np.array(u0, dtype=np.float64, copy=True)
    if U.ndim == 1:
        U = U[:, None]
    K = U.shape[1]
    A, dd = operator_parts(n, row_ptr, col, w, laplacian)
    lam, y = fidelity(labels, K)
    g = precond_diag(precond, lam, eps, c, eta, delta0, lambda_max, step_k,
                     d=None if laplacian == "normalized" else dd)[:, None]
    energies = np.zeros((outer + 1, K))
    res = np.zeros((outer, sweeps, K))

    def T_apply(V):
        # T = eps L_s + eta Lambda + c I, or eps L + eta Lambda + c I (Section 3)
        return eps * (dd[:, None] * V - A @ V) + eta * lam[:, None] * V + c * V

    for t in range(outer):
        if record:
            energies[t] = energy(n, row_ptr, col, w, U, labels, eps, eta, laplacian)
        b = rhs(U, lam, y, eps, c, eta)
        V = U.copy()
        for s in range(sweeps):
            if math.isinf(step_k):
                r = b - T_apply(V)
            else:
                # T_k = I + k T, b_k = u^t + k b^t (Lemma 1)
                r = (U + step_k * b) - (V + step_k * T_apply(V))
            res[t, s] = (r * r).sum(0)
            V = V + r / g
        U = V
    if record:
        energies[outer] = energy(n, row_ptr, col, w, U, labels, eps, eta, laplacian)
    return U, energies, res


def power_max_eig(n, row_ptr, col, w, x0, iters=150, laplacian="normalized"):
    """Power method for the largest eigenvalue of L_s or L (Section 3.1, used
    for G_R,s and G_R; Section 5.1.1 runs 150 iterations).

    x <- x0/||x0||; repeat iters times: x <- L x / ||L x||.  Returns
    (rq, lambda_hat) with rq = x^T L x (x of unit norm) and
    lambda_hat = min(2 max_i dd_i, 1.01 rq) (dd = 1 for L_s, the degrees for L;
    both caps are Prop. 3).
    """
    A, dd = operator_parts(n, row_ptr, col, w, laplacian)
    x = np.asarray(x0, dtype=np.float64).reshape(-1)
    x = x / np.linalg.norm(x)
    for _ in range(iters):
        y = dd * x - A @ x
        x = y / np.linalg.norm(y)
    rq = float(x @ (dd * x - A @ x))
    return rq, min(2.0 * float(dd.max()), 1.01 * rq)


def assign_labels(U):
    """Class per node: K = 1 -> 1 iff u >= 0 (u -> +1 is class 1);
    K >= 2 -> argmax over columns, ties to the lowest column."""
    U = np.asarray(U)
    if U.ndim == 1 or U.shape[1] == 1:
        return (U.reshape(-1) >= 0).astype(np.int32)
    return np.argmax(U, axis=1).astype(np.int32)


# ---------------------------------------------------------------------------
# unsupervised initialisation (Section 5.2, Table 7: the second eigenvector of
# the normalized graph Laplacian starts the unsupervised runs)
# ---------------------------------------------------------------------------

def second_eigenpair(n, row_ptr, col, w, laplacian="normalized"):
    """(lambda_2, v_2) of the dense Laplacian, unit norm, sign fixed so that
    its entry of largest magnitude is positive (dense symmetric eigensolver;
    small graphs only).

    The first eigenvector is the known null vector z (D^{1/2} 1 for L_s,
    Section 2.2; 1 for L) and (lambda_2, v_2) minimises the Rayleigh quotient
    on its orthogonal complement (Courant-Fischer), computed as the smallest
    eigenpair of L + alpha z z^T / |z|^2 with alpha above the spectrum.  For a
    connected graph this is the eigenvector of the second smallest eigenvalue;
    for a disconnected one (lambda_2 = 0) it is the one null vector
    orthogonal to z."""
    if laplacian == "normalized":
        L = dense_normalized_laplacian(n, row_ptr, col, w)
        z = np.sqrt(degrees(n, row_ptr, col, w))
        alpha = 3.0                                   # L_s <= 2I (Prop. 3)
    else:
        L = dense_laplacian(n, row_ptr, col, w)
        z = np.ones(n)
        alpha = 2.0 * float(np.diag(L).max()) + 1.0   # L <= 2D (Prop. 3)
    z = z / np.linalg.norm(z)
    vals, vecs = np.linalg.eigh(L + alpha * np.outer(z, z))
    v = vecs[:, 0].copy()
    i = int(np.argmax(np.abs(v)))
    if v[i] < 0:
        v = -v
    return float(vals[0]), v


def unsupervised_u0(v2):
    """Initial field from the second eigenvector: v_2 scaled to max |u| = 1
    (the paper does not state the scaling; this is the reading used here)."""
    v2 = np.asarray(v2, dtype=np.float64)
    return (v2 / np.abs(v2).max())[:, None]
