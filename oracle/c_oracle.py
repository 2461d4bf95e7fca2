"""ctypes front end of the plain C float64 oracle (gl_oracle.c).

TEST INFRASTRUCTURE ONLY.  ``build()`` compiles the C file with gcc and
OpenMP into ``oracle/libgl_oracle.so``; ``load()`` compiles it on first use
when the shared object is missing.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "gl_oracle.c")
LIB = os.path.join(_HERE, "libgl_oracle.so")
_PRECOND = {"damped_jacobi": 0, "perturbed_jacobi": 1, "richardson": 2}
_LAPLACIAN = {"normalized": 0, "unnormalized": 1}
_lib = None


def build() -> str:
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall",
                    "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p
    i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.glo_solve.argtypes = [i64, P, P, P, i32, P, P, f64, f64, f64, i32, i32, i32,
                              f64, f64, f64, P, P, i32]
    lib.glo_solve.restype = ctypes.c_int
    lib.glo_power.argtypes = [i64, P, P, P, P, i32, P, P, i32]
    lib.glo_power.restype = ctypes.c_int
    lib.glo_laplacian_apply.argtypes = [i64, P, P, P, i32, P, P, i32]
    lib.glo_laplacian_apply.restype = ctypes.c_int
    lib.glo_window_graph.argtypes = [i32, i32, i32, P, i32, i32, f64, P, P, P, i64]
    lib.glo_window_graph.restype = ctypes.c_int64
    lib.glo_num_threads.argtypes = []
    lib.glo_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(row_ptr, col, w):
    return (np.ascontiguousarray(row_ptr, dtype=np.int64),
            np.ascontiguousarray(col, dtype=np.int32),
            np.ascontiguousarray(w, dtype=np.float64))


def num_threads() -> int:
    return int(load().glo_num_threads())


def dca_solve(n, row_ptr, col, w, labels, u0, *, eps, c, eta, precond, outer, sweeps,
              delta0=1e-6, lambda_max=2.0, step_k=math.inf, record=True,
              laplacian="normalized"):
    """Same contract as gl_oracle.dca_solve."""
    lib = load()
    rp, cl, ww = _csr(row_ptr, col, w)
    U = np.array(u0, dtype=np.float64, copy=True, order="C")
    if U.ndim == 1:
        U = U[:, None].copy()
    K = U.shape[1]
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    en = np.zeros((outer + 1, K)) if record else None
    rs = np.zeros((outer, sweeps, K)) if record else None
    rc = lib.glo_solve(n, _ptr(rp), _ptr(cl), _ptr(ww), K, _ptr(lab), _ptr(U),
                       eps, c, eta, _PRECOND[precond], outer, sweeps, delta0, lambda_max,
                       step_k, _ptr(en) if record else None, _ptr(rs) if record else None,
                       _LAPLACIAN[laplacian])
    if rc != 0:
        raise MemoryError("C oracle allocation failed")
    return U, en, rs


def window_graph(img, rw, rp, sigma):
    """Same contract as window_oracle.window_graph (plain C, OpenMP over pixels)."""
    lib = load()
    im = np.ascontiguousarray(img, dtype=np.float64)
    if im.ndim == 2:
        im = im[:, :, None].copy()
    h, w, C = im.shape
    n = h * w
    cap = n * ((2 * rw + 1) ** 2 - 1)
    row_ptr = np.empty(n + 1, dtype=np.int64)
    col = np.empty(cap, dtype=np.int32)
    ww = np.empty(cap, dtype=np.float64)
    nnz = lib.glo_window_graph(h, w, C, _ptr(im), rw, rp, float(sigma), _ptr(row_ptr), _ptr(col),
                               _ptr(ww), cap)
    if nnz < 0:
        raise MemoryError("window graph larger than its bound")
    return row_ptr, col[:nnz].copy(), ww[:nnz].copy()


def power_max_eig(n, row_ptr, col, w, x0, iters=150, laplacian="normalized"):
    lib = load()
    rp, cl, ww = _csr(row_ptr, col, w)
    x = np.ascontiguousarray(x0, dtype=np.float64).reshape(-1)
    rq = np.zeros(1)
    lh = np.zeros(1)
    if lib.glo_power(n, _ptr(rp), _ptr(cl), _ptr(ww), _ptr(x), iters, _ptr(rq), _ptr(lh),
                     _LAPLACIAN[laplacian]):
        raise MemoryError("C oracle allocation failed")
    return float(rq[0]), float(lh[0])


def laplacian_apply(n, row_ptr, col, w, X, laplacian="normalized"):
    lib = load()
    rp, cl, ww = _csr(row_ptr, col, w)
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None].copy()
    Y = np.empty_like(X)
    if lib.glo_laplacian_apply(n, _ptr(rp), _ptr(cl), _ptr(ww), X.shape[1], _ptr(X), _ptr(Y),
                               _LAPLACIAN[laplacian]):
        raise MemoryError("C oracle allocation failed")
    return Y
