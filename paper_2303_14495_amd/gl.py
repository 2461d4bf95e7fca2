"""ctypes binding of ``libgl_dca.so`` (declared in include/gl_dca.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  torch supplies device memory (tensors) and streams.  If the shared
library has not been built this module raises on first use; there is no
fallback path.
"""

from __future__ import annotations

import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgl_dca.so")

DTYPES = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}
TORCH_DTYPES = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16,
                "f16": torch.float16}
DTYPE_OF_TORCH = {v: k for k, v in TORCH_DTYPES.items()}
PRECONDS = {"damped_jacobi": 0, "perturbed_jacobi": 1, "richardson": 2}
STATUS = {0: "GL_OK", 1: "GL_E_INVALID_ARG", 2: "GL_E_BAD_GRAPH", 3: "GL_E_DTYPE",
          4: "GL_E_NOMEM", 5: "GL_E_BUDGET", 6: "GL_E_NONFINITE", 7: "GL_E_HIP",
          8: "GL_E_QUEUE_FULL", 9: "GL_E_NOT_READY", 10: "GL_E_CANCELLED"}


class GLError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class _Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("weight", ctypes.c_void_p),
                ("weight_dtype", ctypes.c_int32), ("order", ctypes.c_void_p),
                ("layout", ctypes.c_int32), ("laplacian", ctypes.c_int32),
                ("grid_height", ctypes.c_int32), ("grid_width", ctypes.c_int32)]


class _WindowGraph(ctypes.Structure):
    _fields_ = [("image", ctypes.c_void_p), ("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("channels", ctypes.c_int32), ("window_radius", ctypes.c_int32),
                ("patch_radius", ctypes.c_int32), ("laplacian", ctypes.c_int32),
                ("sigma", ctypes.c_double), ("reserved", ctypes.c_int32)]


LAYOUTS = {"auto": 0, "direct": 1, "tile": 2, "grid": 4}
LAYOUT_NAMES = {1: "direct", 2: "tile", 3: "window", 4: "grid"}
LAPLACIANS = {"normalized": 0, "unnormalized": 1}


class _Params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("c", ctypes.c_double), ("eta", ctypes.c_double),
                ("delta0", ctypes.c_double), ("lambda_max", ctypes.c_double),
                ("step_k", ctypes.c_double), ("precond", ctypes.c_int32),
                ("outer_steps", ctypes.c_int32), ("inner_sweeps", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("max_pending", ctypes.c_int32), ("store_w", ctypes.c_int32),
                ("store_u", ctypes.c_int32), ("ticks_in_flight", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("weight", ctypes.c_void_p),
                ("labels", ctypes.c_void_p), ("u0", ctypes.c_void_p), ("K", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("params", _Params)]


class _Result(ctypes.Structure):
    _fields_ = [("U", ctypes.c_void_p), ("labels", ctypes.c_void_p), ("stats", ctypes.c_void_p),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None

# symbol -> (restype, argtypes)
_P, _I32, _I64, _SZ, _D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t,
                          ctypes.c_double)
SIGNATURES = {
    "gl_operator_create": (ctypes.c_int, [_P, _I32, _P, _P]),
    "gl_window_operator_create": (ctypes.c_int, [_P, _I32, _P, _P]),
    "gl_knn_graph": (ctypes.c_int, [_I64, _I32, _P, _P, _I32, _P, _P, _P, _I64, _P, _P]),
    "gl_knn_fallback_rows": (ctypes.c_int64, []),
    "gl_operator_destroy": (ctypes.c_int, [_P]),
    "gl_operator_info": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "gl_operator_layout": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "gl_laplacian_apply": (ctypes.c_int, [_P, _I32, _I32, _P, _P, _P]),
    "gl_power_workspace_size": (ctypes.c_int, [_P, _P]),
    "gl_power_max_eig": (ctypes.c_int, [_P, _I32, _P, _P, _SZ, _P, _P, _P]),
    "gl_solve_workspace_size": (ctypes.c_int, [_P, _I32, _I32, _P]),
    "gl_stats_length": (ctypes.c_int64, [_I32, _I32, _I32]),
    "gl_solve": (ctypes.c_int, [_P, _P, _I32, _P, _I32, _P, _P, _SZ, _P, _P]),
    "gl_solve_noalloc": (ctypes.c_int, [_P, _P, _I32, _P, _I32, _P, _P, _P]),
    "gl_assign_labels": (ctypes.c_int, [_I64, _I32, _I32, _P, _P, _P]),
    "gl_params_validate": (ctypes.c_int, [_P]),
    "gl_time_sweeps": (ctypes.c_int, [_P, _P, _I32, _P, _I32, _P, _P, _SZ, _I32, _P, _P]),
    "gl_time_stream": (ctypes.c_int, [_I32, _P, _SZ, _I32, _P, _P]),
    "gl_server_create": (ctypes.c_int, [_P, _P]),
    "gl_server_submit": (ctypes.c_int, [_P, _P, _P]),
    "gl_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, _I32, _P]),
    "gl_server_cancel": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "gl_server_request_bytes": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                               ctypes.c_int32, ctypes.c_int32, ctypes.c_int,
                                               ctypes.c_int, _P, _P]),
    "gl_server_info": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "gl_server_destroy": (ctypes.c_int, [_P]),
    "gl_knn": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P, _P, _P]),
    "gl_second_eigenpair_workspace_size": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "gl_second_eigenpair": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, _P,
                                           _P, _P, ctypes.c_size_t, _P, _P, _P, _P]),
    "gl_last_error": (ctypes.c_char_p, []),
    "gl_version": (ctypes.c_char_p, []),
}


def load_library(path: str = LIB_PATH):
    """Load the HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        msg = load_library().gl_last_error()
        raise GLError(status, msg.decode() if msg else "")


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def stats_length(K: int, outer: int, sweeps: int) -> int:
    return int(load_library().gl_stats_length(K, outer, sweeps))


def split_stats(stats: torch.Tensor, K: int, outer: int, sweeps: int):
    """(energies [T+1, K], residual_sq [T, m, K], nonfinite flag) from a stats vector."""
    e = stats[: (outer + 1) * K].view(outer + 1, K)
    r = stats[(outer + 1) * K: (outer + 1) * K + outer * sweeps * K].view(outer, sweeps, K)
    return e, r, float(stats[-1])


class Operator:
    """Graph operator held on the GPU: the normalized What = D^{-1/2} W D^{-1/2}
    of L_s (laplacian="normalized") or W and D of L = D - W ("unnormalized").

    row_ptr (int64 [n+1]), col (int32 [nnz]) and weight (float64 or float32
    [nnz]) are CUDA tensors of a symmetric graph without self-loops.
    """

    def __init__(self, row_ptr, col, weight, store_w: str = "f32", stream=None, order=None,
                 layout: str = "auto", laplacian: str = "normalized", grid=None):
        lib = load_library()
        if not (row_ptr.is_cuda and col.is_cuda and weight.is_cuda):
            raise ValueError("graph tensors must live on the GPU")
        if row_ptr.dtype != torch.int64 or col.dtype != torch.int32:
            raise ValueError("row_ptr must be int64 and col int32")
        if weight.dtype not in (torch.float64, torch.float32):
            raise ValueError("weight must be float64 or float32")
        self.row_ptr, self.col, self.weight = (row_ptr.contiguous(), col.contiguous(),
                                               weight.contiguous())
        self.n = int(row_ptr.numel() - 1)
        self.nnz = int(col.numel())
        self.store_w = store_w
        self.device = row_ptr.device
        order_t = None
        if order is not None:
            order_t = order.to(device=row_ptr.device, dtype=torch.int32).contiguous()
        g = _Graph(self.n, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(),
                   self.weight.data_ptr(), DTYPES[DTYPE_OF_TORCH[weight.dtype]],
                   order_t.data_ptr() if order_t is not None else None, LAYOUTS[layout],
                   LAPLACIANS[laplacian], *((0, 0) if grid is None else (int(grid[0]), int(grid[1]))))
        self.laplacian = laplacian
        handle = ctypes.c_void_p()
        self._h = None
        _check(lib.gl_operator_create(ctypes.byref(g), DTYPES[store_w], _stream_handle(stream),
                                      ctypes.byref(handle)))
        self._h = handle
        self._ws = {}
        # the library holds its own copies; drop the references
        self.row_ptr = self.col = self.weight = None

    @classmethod
    def window(cls, image: torch.Tensor, window_radius: int = 7, patch_radius: int = 2,
               sigma: float | None = None, store_w: str = "f32", laplacian: str = "normalized",
               stream=None) -> "Operator":
        """Operator of the paper's image graph (Section 2.2), built on the GPU:
        every pixel joined to its (2 window_radius + 1)^2 - 1 window neighbours
        with patch-similarity weights over (2 patch_radius + 1)^2 patches.
        image: CUDA float32 [h, w] or [h, w, channels], row-major pixels (the
        nodes).  sigma defaults to log(h w) + 1."""
        lib = load_library()
        if not image.is_cuda:
            raise ValueError("image must live on the GPU")
        img = image.to(torch.float32).contiguous()
        if img.dim() == 2:
            img = img.unsqueeze(-1)
        if img.dim() != 3:
            raise ValueError("image must be [h, w] or [h, w, channels]")
        h, w, ch = (int(v) for v in img.shape)
        if sigma is None:
            sigma = math.log(h * w) + 1.0
        g = _WindowGraph(img.data_ptr(), h, w, ch, int(window_radius), int(patch_radius),
                         LAPLACIANS[laplacian], float(sigma), 0)
        self = cls.__new__(cls)
        self._h = None
        handle = ctypes.c_void_p()
        _check(lib.gl_window_operator_create(ctypes.byref(g), DTYPES[store_w],
                                             _stream_handle(stream), ctypes.byref(handle)))
        self._h = handle
        self._ws = {}
        self.row_ptr = self.col = self.weight = None
        self.store_w = store_w
        self.device = image.device
        self.laplacian = laplacian
        self.n = h * w
        self.nnz = self.info()["nnz"]
        self.image_shape = (h, w)
        return self

    def close(self):
        if getattr(self, "_h", None) is not None:
            load_library().gl_operator_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        n, nnz, sw, lanes, by = (ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(),
                                 ctypes.c_int32(), ctypes.c_size_t())
        _check(load_library().gl_operator_info(self._h, ctypes.byref(n), ctypes.byref(nnz),
                                               ctypes.byref(sw), ctypes.byref(lanes),
                                               ctypes.byref(by)))
        lay, stored, hmax, htot, sb = (ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(),
                                       ctypes.c_int64(), ctypes.c_int64())
        _check(load_library().gl_operator_layout(self._h, ctypes.byref(lay), ctypes.byref(stored),
                                                 ctypes.byref(hmax), ctypes.byref(htot),
                                                 ctypes.byref(sb)))
        return {"n": n.value, "nnz": nnz.value, "lanes_per_row": lanes.value,
                "device_bytes": by.value,
                "layout": LAYOUT_NAMES[lay.value], "stored_entries": stored.value,
                "halo_max": hmax.value, "halo_total": htot.value, "stream_bytes": sb.value,
                "laplacian": self.laplacian}

    def _workspace(self, key, nbytes):
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def laplacian_apply(self, X: torch.Tensor, stream=None) -> torch.Tensor:
        X2 = X if X.dim() == 2 else X.view(-1, 1)
        X2 = X2.contiguous()
        Y = torch.empty_like(X2)
        _check(load_library().gl_laplacian_apply(self._h, X2.shape[1],
                                                 DTYPES[DTYPE_OF_TORCH[X2.dtype]], _ptr(X2),
                                                 _ptr(Y), _stream_handle(stream)))
        return Y.view_as(X)

    def power_max_eig(self, x0: torch.Tensor, iters: int = 150, stream=None):
        lib = load_library()
        nb = ctypes.c_size_t()
        _check(lib.gl_power_workspace_size(self._h, ctypes.byref(nb)))
        ws = self._workspace("power", nb.value)
        x0 = x0.to(torch.float32).contiguous()
        rq, lam = ctypes.c_double(), ctypes.c_double()
        _check(lib.gl_power_max_eig(self._h, iters, _ptr(x0), _ptr(ws), ws.numel(),
                                    ctypes.byref(rq), ctypes.byref(lam), _stream_handle(stream)))
        return rq.value, lam.value

    def second_eigenpair(self, x0: torch.Tensor, krylov: int = 64, max_restarts: int = 20,
                         tol: float = 1e-5, stream=None):
        """(lambda_2, v_2 [n] float, residual, restarts) of the operator's Laplacian."""
        lib = load_library()
        need = ctypes.c_size_t()
        _check(lib.gl_second_eigenpair_workspace_size(self.handle, krylov, ctypes.byref(need)))
        ws = self._workspace(("eig", krylov), need.value)
        x0 = x0.to(torch.float32).contiguous()
        v = torch.empty(self.n, dtype=torch.float32, device=self.device)
        lam, res, rs = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        _check(lib.gl_second_eigenpair(self.handle, krylov, max_restarts, tol, _ptr(x0), _ptr(v),
                                       _ptr(ws), ws.numel(), ctypes.byref(lam), ctypes.byref(res),
                                       ctypes.byref(rs), _stream_handle(stream)))
        return lam.value, v, res.value, rs.value
    def workspace_bytes(self, K: int, store_u: str) -> int:
        nb = ctypes.c_size_t()
        _check(load_library().gl_solve_workspace_size(self._h, K, DTYPES[store_u],
                                                      ctypes.byref(nb)))
        return nb.value

    def solve(self, labels: torch.Tensor, U: torch.Tensor, *, eps, c, eta, precond, outer,
              sweeps, delta0=1e-6, lambda_max=2.0, step_k=math.inf, stats=True, stream=None,
              stats_out: torch.Tensor | None = None):
        """Run the preconditioned DCA in place on U (n x K, f64/f32/bf16/f16).

        Returns the stats vector (float64 on the GPU) or None.
        """
        lib = load_library()
        if U.dim() == 1:
            raise ValueError("U must be n x K")
        if not U.is_contiguous() or labels.dtype != torch.int32 or not labels.is_contiguous():
            raise ValueError("U must be contiguous and labels contiguous int32")
        K = U.shape[1]
        store_u = DTYPE_OF_TORCH[U.dtype]
        ws = self._workspace(("solve", K, store_u), self.workspace_bytes(K, store_u))
        p = _Params(eps, c, eta, delta0, lambda_max, step_k, PRECONDS[precond], outer, sweeps, 0)
        st = None
        if stats:
            st = stats_out if stats_out is not None else torch.empty(
                stats_length(K, outer, sweeps), dtype=torch.float64, device=U.device)
        _check(lib.gl_solve(self._h, ctypes.byref(p), K, _ptr(labels), DTYPES[store_u], _ptr(U),
                            _ptr(ws), ws.numel(), _ptr(st) if st is not None else None,
                            _stream_handle(stream)))
        return st

    def solve_noalloc(self, labels: torch.Tensor, U: torch.Tensor, stats_out: torch.Tensor | None,
                      *, eps, c, eta, precond, outer, sweeps, delta0=1e-6, lambda_max=2.0,
                      step_k=math.inf, stream=None):
        """solve() through gl_solve_noalloc: the library's static workspace, no
        allocation by the library or here (stats_out, if given, is the caller's
        float64 [stats_length] device tensor)."""
        if U.dim() != 2 or not U.is_contiguous() or labels.dtype != torch.int32 \
                or not labels.is_contiguous():
            raise ValueError("U must be contiguous n x K and labels contiguous int32")
        p = _Params(eps, c, eta, delta0, lambda_max, step_k, PRECONDS[precond], outer, sweeps, 0)
        _check(load_library().gl_solve_noalloc(
            self._h, ctypes.byref(p), U.shape[1], _ptr(labels), DTYPES[DTYPE_OF_TORCH[U.dtype]],
            _ptr(U), _ptr(stats_out) if stats_out is not None else None, _stream_handle(stream)))


def time_sweeps(op: Operator, labels: torch.Tensor, U: torch.Tensor, *, eps, c, eta, precond,
                delta0=1e-6, lambda_max=2.0, step_k=math.inf, reps=20, stream=None) -> float:
    """Mean time per sweep launch (ms): `reps` launches back to back between one
    pair of HIP events on the stream, gaps between launches included."""
    lib = load_library()
    K = U.shape[1]
    store_u = DTYPE_OF_TORCH[U.dtype]
    ws = op._workspace(("solve", K, store_u), op.workspace_bytes(K, store_u))
    p = _Params(eps, c, eta, delta0, lambda_max, step_k, PRECONDS[precond], 1, 1, 0)
    out = ctypes.c_double()
    _check(lib.gl_time_sweeps(op.handle, ctypes.byref(p), K, _ptr(labels), DTYPES[store_u],
                              _ptr(U), _ptr(ws), ws.numel(), reps, ctypes.byref(out),
                              _stream_handle(stream)))
    return out.value


def time_stream(buf: torch.Tensor, kind: str = "read", reps: int = 20, stream=None) -> float:
    """Mean time per launch (ms) of the library's plain streaming kernel
    ("read": reads all of buf) or copy kernel ("copy": first half to second
    half) over a device byte tensor, `reps` launches between one event pair."""
    if not buf.is_cuda or buf.dtype != torch.uint8 or not buf.is_contiguous():
        raise ValueError("buf must be a contiguous CUDA uint8 tensor")
    out = ctypes.c_double()
    _check(load_library().gl_time_stream({"read": 0, "copy": 1}[kind], _ptr(buf), buf.numel(),
                                         reps, ctypes.byref(out), _stream_handle(stream)))
    return out.value


def knn_graph(idx: torch.Tensor, d2: torch.Tensor, scale_rank: int = 7, stream=None):
    """Union-symmetric kNN graph with local-scaling weights (Section 2.2) from
    kNN lists on the GPU: returns (row_ptr int64 [n+1], col int32 [nnz],
    weight float64 [nnz]) CUDA tensors."""
    idx = idx.to(torch.int32).contiguous()
    d2 = d2.to(torch.float32).contiguous()
    n, k = (int(v) for v in idx.shape)
    cap = 2 * n * k
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=idx.device)
    col = torch.empty(cap, dtype=torch.int32, device=idx.device)
    w = torch.empty(cap, dtype=torch.float64, device=idx.device)
    nnz = ctypes.c_int64()
    _check(load_library().gl_knn_graph(n, k, _ptr(idx), _ptr(d2), int(scale_rank), _ptr(row_ptr),
                                       _ptr(col), _ptr(w), cap, ctypes.byref(nnz),
                                       _stream_handle(stream)))
    m = nnz.value
    return row_ptr, col[:m].clone(), w[:m].clone()


def assign_labels(U: torch.Tensor, stream=None) -> torch.Tensor:
    """Class per node (K = 1: u >= 0 -> 1; K >= 2: argmax, ties to the lowest)."""
    U2 = U if U.dim() == 2 else U.view(-1, 1)
    U2 = U2.contiguous()
    out = torch.empty(U2.shape[0], dtype=torch.int32, device=U.device)
    _check(load_library().gl_assign_labels(U2.shape[0], U2.shape[1],
                                           DTYPES[DTYPE_OF_TORCH[U2.dtype]], _ptr(U2), _ptr(out),
                                           _stream_handle(stream)))
    return out


def knn_fallback_rows() -> int:
    """Queries of this thread's last wide-feature (d > 64) kNN call that needed
    the exact rescan."""
    return int(load_library().gl_knn_fallback_rows())


def knn(x: torch.Tensor, k: int, with_distances: bool = True, stream=None):
    """Exact k nearest neighbours of every row of x (device f32 [n, d]):
    (indices int32 [n, k], squared distances f32 [n, k] or None)."""
    if x.dtype != torch.float32 or x.dim() != 2 or not x.is_cuda:
        raise GLError(1, "x must be a device float32 [n, d] tensor")
    x = x.contiguous()
    n, d = x.shape
    idx = torch.empty((n, k), dtype=torch.int32, device=x.device)
    d2 = torch.empty((n, k), dtype=torch.float32, device=x.device) if with_distances else None
    _check(load_library().gl_knn(_ptr(x), n, d, k, _ptr(idx), _ptr(d2) if d2 is not None else None,
                                 _stream_handle(stream)))
    return idx, d2


class Server:
    """Continuous-batching server (gl_server_*): host requests in, host results out."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 32, max_pending: int = 1024,
                 store_w: str = "bf16", store_u: str = "bf16", ticks_in_flight: int = 2):
        lib = load_library()
        cfg = _ServerConfig(hbm_budget_bytes, max_slots, max_pending, DTYPES[store_w],
                            DTYPES[store_u], ticks_in_flight, 0)
        h = ctypes.c_void_p()
        self._h = None
        _check(lib.gl_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._meta = {}

    def submit(self, row_ptr, col, weight, labels, u0, *, eps, c, eta, precond, outer, sweeps,
               delta0=1e-6, lambda_max=2.0, step_k=math.inf, borrow=False) -> int:
        """Queue a request.  borrow=True: the server reads the arrays in place
        (GL_REQ_BORROW); they are kept referenced here until the result is
        polled."""
        import numpy as np
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        w = np.ascontiguousarray(weight, dtype=np.float64)
        lab = np.ascontiguousarray(labels, dtype=np.int32)
        U0 = np.ascontiguousarray(u0, dtype=np.float32)
        if U0.ndim == 1:
            U0 = U0[:, None].copy()
        n, K = U0.shape
        p = _Params(eps, c, eta, delta0, lambda_max, step_k, PRECONDS[precond], outer, sweeps, 0)
        req = _Request(n, cl.size, rp.ctypes.data, cl.ctypes.data, w.ctypes.data, lab.ctypes.data,
                       U0.ctypes.data, K, 1 if borrow else 0, p)
        t = ctypes.c_uint64()
        _check(load_library().gl_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        self._meta[t.value] = (n, K, outer, sweeps, (rp, cl, w, lab, U0) if borrow else None)
        return t.value

    def poll(self, ticket: int, wait: bool = True):
        """Result dict, or None while not ready (wait=False)."""
        import numpy as np
        if ticket not in self._meta:
            raise GLError(1, "unknown or consumed ticket")
        n, K, T, m, _ = self._meta[ticket]
        U = np.empty((n, K), dtype=np.float32)
        lab = np.empty(n, dtype=np.int32)
        st = np.empty(stats_length(K, T, m), dtype=np.float64)
        r = _Result(U.ctypes.data, lab.ctypes.data, st.ctypes.data, 0, 0, 0, 0, 0)
        rc = load_library().gl_server_poll(self._h, ticket, 1 if wait else 0, ctypes.byref(r))
        if rc == 9:  # GL_E_NOT_READY
            return None
        _check(rc)
        del self._meta[ticket]
        return {"status": STATUS.get(r.status, r.status), "U": U, "labels": lab, "stats": st,
                "t_submit": r.t_submit, "t_admit": r.t_admit, "t_done": r.t_done}

    @staticmethod
    def request_bytes(n, nnz, K, outer, sweeps, store_w="bf16", store_u="bf16"):
        """(peak, held) arena bytes of a request (gl_server_request_bytes)."""
        peak, held = ctypes.c_size_t(), ctypes.c_size_t()
        _check(load_library().gl_server_request_bytes(n, nnz, K, outer, sweeps, DTYPES[store_w],
                                                      DTYPES[store_u], ctypes.byref(peak),
                                                      ctypes.byref(held)))
        return peak.value, held.value

    def cancel(self, ticket: int):
        _check(load_library().gl_server_cancel(self._h, ticket))

    def info(self) -> dict:
        v = [ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t(),
             ctypes.c_int64()]
        _check(load_library().gl_server_info(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("pending", "active", "finished", "arena_used", "ticks"),
                        [x.value for x in v]))

    def close(self):
        if getattr(self, "_h", None) is not None:
            load_library().gl_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version() -> str:
    return load_library().gl_version().decode()
