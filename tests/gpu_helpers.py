"""Shared helpers of the GPU tests: run a synthetic problem through the C ABI
and through the float64 oracle on the same seeded inputs."""

from __future__ import annotations

import math
import sys

import numpy as np
import torch

import paper_2303_14495_amd as gl
from oracle import c_oracle, gl_oracle

DEV = torch.device("cuda:0") if torch.cuda.is_available() else None


_PROBLEMS = {}


def problem(cfg: int, small: bool = False):
    """Workload `cfg`, built once per test session (on the GPU when present)."""
    key = (cfg, small)
    if key not in _PROBLEMS:
        from synth import make_problem
        say(f"building workload {cfg} small={small}")
        _PROBLEMS[key] = make_problem(cfg, device=DEV if DEV is not None else "cpu", small=small)
    return _PROBLEMS[key]


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def power_x0(n: int, seed: int) -> np.ndarray:
    """Seeded start vector of the power method (an input to both sides)."""
    return np.random.default_rng(10_000 + seed).uniform(-1.0, 1.0, n)


def oracle_lambda(p, iters=150, laplacian="normalized"):
    rp, col, w = p.graph.numpy()
    rq, lam = c_oracle.power_max_eig(p.n, rp, col, w, power_x0(p.n, p.seed), iters,
                                     laplacian=laplacian)
    return rq, lam


def make_operator(p, store_w, layout="auto", use_order=True, laplacian="normalized"):
    g = p.graph
    grid = None
    if layout == "grid":
        grid, use_order = p.extra["grid"], False  # the grid layout takes no order
    order = getattr(p, "order", None) if use_order else None
    return gl.Operator(g.row_ptr.to(DEV), g.col.to(DEV), g.weight.to(DEV).to(torch.float64),
                       store_w=store_w, layout=layout, laplacian=laplacian, grid=grid,
                       order=torch.from_numpy(order).to(DEV) if order is not None else None)


def gpu_solve(p, store_w, store_u, lambda_max=2.0, outer=None, sweeps=None, u0=None,
              labels=None, op=None, stats=True, precond=None, step_k=None):
    outer = p.outer if outer is None else outer
    sweeps = p.sweeps if sweeps is None else sweeps
    op = op or make_operator(p, store_w)
    u0 = p.u0 if u0 is None else u0
    labels = p.labels if labels is None else labels
    U = torch.from_numpy(np.ascontiguousarray(u0)).to(DEV, gl.TORCH_DTYPES[store_u]).contiguous()
    lab = torch.from_numpy(np.ascontiguousarray(labels, dtype=np.int32)).to(DEV)
    st = op.solve(lab, U, eps=p.eps, c=p.c, eta=p.eta,
                  precond=p.precond if precond is None else precond, outer=outer,
                  sweeps=sweeps, delta0=p.delta0, lambda_max=lambda_max,
                  step_k=p.step_k if step_k is None else step_k, stats=stats)
    torch.cuda.synchronize()
    out = U.to(torch.float64).cpu().numpy()
    if not stats:
        return out, None, None, None, U
    e, r, flag = gl.split_stats(st.cpu(), U.shape[1], outer, sweeps)
    return out, e.numpy(), r.numpy(), flag, U


_ORACLE_SOLVES = {}


def oracle_solve(p, lambda_max=2.0, outer=None, sweeps=None, u0=None, labels=None, use_c=True,
                 laplacian="normalized", precond=None, step_k=None):
    key = None
    if u0 is None and labels is None:
        # the same problem and schedule: reuse the oracle's answer within a session
        key = (id(p), lambda_max, outer, sweeps, use_c, laplacian, precond, step_k)
        if key in _ORACLE_SOLVES:
            return _ORACLE_SOLVES[key]
    out = _oracle_solve(p, lambda_max, outer, sweeps, u0, labels, use_c, laplacian, precond, step_k)
    if key is not None:
        _ORACLE_SOLVES[key] = out
    return out


def _oracle_solve(p, lambda_max, outer, sweeps, u0, labels, use_c, laplacian, precond, step_k):
    rp, col, w = p.graph.numpy()
    orc = c_oracle if use_c else gl_oracle
    return orc.dca_solve(p.n, rp, col, w, p.labels if labels is None else labels,
                         p.u0 if u0 is None else u0, eps=p.eps, c=p.c, eta=p.eta,
                         precond=p.precond if precond is None else precond,
                         outer=p.outer if outer is None else outer,
                         sweeps=p.sweeps if sweeps is None else sweeps, delta0=p.delta0,
                         lambda_max=lambda_max, step_k=p.step_k if step_k is None else step_k,
                         laplacian=laplacian)


def label_agreement(Ua, Ub) -> float:
    return float(np.mean(gl_oracle.assign_labels(Ua) == gl_oracle.assign_labels(Ub)))


def rel_close(a, b, rtol):
    a, b = np.asarray(a), np.asarray(b)
    scale = max(1.0, float(np.abs(b).max()))
    return float(np.abs(a - b).max()) <= rtol * scale
