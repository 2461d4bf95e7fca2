"""Host-side checks of the C ABI: the library loads without a GPU, exports
every entry point the header declares, and rejects bad arguments before any
launch."""

import ctypes
import math
import os
import re

import pytest

import paper_2303_14495_amd as gl
from paper_2303_14495_amd import gl as glmod

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", fn)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(gl_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = gl.load_library()
    declared = _declared_functions()
    assert "gl_solve" in declared and "gl_operator_create" in declared
    for name in sorted(declared):
        assert hasattr(lib, name), f"{name} declared in include/ but not exported"


def test_binding_covers_declared_symbols():
    declared = _declared_functions()
    missing = declared - set(glmod.SIGNATURES)
    assert not missing, missing


def test_version_and_stats_length():
    assert "gfx950" in gl.version()
    K, T, m = 3, 5, 4
    assert gl.stats_length(K, T, m) == (T + 1) * K + T * m * K + 1
    assert gl.stats_length(0, T, m) == 0


def _params(**kw):
    base = dict(eps=1.0, c=3.0, eta=10.0, delta0=1e-6, lambda_max=1.5, step_k=math.inf,
                precond=0, outer_steps=2, inner_sweeps=2, reserved=0)
    base.update(kw)
    return glmod._Params(**base)


@pytest.mark.parametrize("bad", [
    dict(eps=0.0), dict(eps=-1.0), dict(eps=math.nan), dict(c=0.0), dict(eta=-1.0),
    dict(delta0=-1e-3), dict(precond=7), dict(precond=2, lambda_max=0.0),
    dict(precond=2, lambda_max=math.inf), dict(precond=2, lambda_max=math.nan),
    dict(step_k=0.0), dict(step_k=-math.inf),
    dict(step_k=math.nan), dict(outer_steps=-1), dict(inner_sweeps=0), dict(reserved=1),
])
def test_params_rejected(bad):
    lib = gl.load_library()
    p = _params(**bad)
    assert lib.gl_params_validate(ctypes.byref(p)) == 1
    assert lib.gl_last_error()


def test_params_accepted():
    lib = gl.load_library()
    for kw in [dict(), dict(precond=2, lambda_max=2.0), dict(step_k=0.5), dict(eta=0.0),
               dict(outer_steps=0)]:
        p = _params(**kw)
        assert lib.gl_params_validate(ctypes.byref(p)) == 0


def test_null_arguments_rejected():
    lib = gl.load_library()
    assert lib.gl_operator_create(None, 1, None, None) == 1
    assert lib.gl_solve(None, None, 1, None, 1, None, None, 0, None, None) == 1
    assert lib.gl_laplacian_apply(None, 1, 1, None, None, None) == 1
    assert lib.gl_assign_labels(10, 1, 1, None, None, None) == 1
    assert lib.gl_params_validate(None) == 1
    assert lib.gl_operator_destroy(None) == 0
    assert lib.gl_knn(None, 100, 3, 5, None, None, None) == 1


@pytest.mark.parametrize("n,d,k", [(100, 0, 5), (100, 4097, 5), (100, 3, 0), (100, 3, 33), (5, 3, 5)])
def test_knn_sizes_rejected(n, d, k):
    # size checks come before any device access (dummy non-NULL pointers)
    lib = gl.load_library()
    dummy = ctypes.c_void_p(256)
    assert lib.gl_knn(dummy, n, d, k, dummy, None, None) == 1


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(glmod, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        glmod.load_library(str(tmp_path / "nope.so"))


def _window_graph(**kw):
    base = dict(image=4096, height=8, width=8, channels=3, window_radius=2, patch_radius=1,
                laplacian=0, sigma=1.0, reserved=0)
    base.update(kw)
    return glmod._WindowGraph(**base)


@pytest.mark.parametrize("bad,status", [
    (dict(image=None), 1), (dict(image=4098), 1), (dict(height=0), 1), (dict(width=-1), 1),
    (dict(height=65536, width=32768), 1), (dict(channels=0), 1), (dict(channels=5), 1),
    (dict(window_radius=0), 1), (dict(window_radius=28), 1), (dict(patch_radius=-1), 1),
    (dict(patch_radius=5), 1), (dict(sigma=0.0), 1), (dict(sigma=math.inf), 1),
    (dict(sigma=math.nan), 1), (dict(laplacian=2), 1), (dict(reserved=1), 1),
])
def test_window_operator_rejects_bad_arguments(bad, status):
    lib = gl.load_library()
    g = _window_graph(**bad)
    out = ctypes.c_void_p()
    assert lib.gl_window_operator_create(ctypes.byref(g), 1, None, ctypes.byref(out)) == status
    assert out.value is None
    assert lib.gl_last_error()


def test_window_operator_rejects_bad_dtype_and_nulls():
    lib = gl.load_library()
    g = _window_graph()
    out = ctypes.c_void_p()
    assert lib.gl_window_operator_create(ctypes.byref(g), 9, None, ctypes.byref(out)) == 3
    assert lib.gl_window_operator_create(None, 1, None, ctypes.byref(out)) == 1
    assert lib.gl_window_operator_create(ctypes.byref(g), 1, None, None) == 1


@pytest.mark.parametrize("n,k,rank,cap,status", [
    (1, 1, 1, 2, 1), (10, 0, 1, 20, 1), (10, 10, 1, 200, 1), (10, 3, 0, 60, 1),
    (10, 3, 4, 60, 1), (10, 3, 2, 59, 1), (1 << 31, 3, 2, 6 << 31, 1),
])
def test_knn_graph_rejects_bad_sizes(n, k, rank, cap, status):
    lib = gl.load_library()
    fake = ctypes.c_void_p(4096)
    nnz = ctypes.c_int64()
    assert lib.gl_knn_graph(n, k, fake, fake, rank, fake, fake, fake, cap, ctypes.byref(nnz),
                            None) == status
    assert lib.gl_last_error()


def test_knn_graph_rejects_nulls():
    lib = gl.load_library()
    fake = ctypes.c_void_p(4096)
    nnz = ctypes.c_int64()
    args = [10, 3, fake, fake, 2, fake, fake, fake, 60, ctypes.byref(nnz), None]
    for pos in (2, 3, 5, 6, 7, 9):
        a = list(args)
        a[pos] = None
        assert lib.gl_knn_graph(*a) == 1


@pytest.mark.parametrize("h,w", [(2, 3), (1, 1 << 24), (0, 6)])
def test_grid_operator_rejects_bad_shapes(h, w):
    # shape checks come before any device access (dummy non-NULL pointers)
    lib = gl.load_library()
    fake = ctypes.c_void_p(4096)
    n = 6 if (h, w) != (1, 1 << 24) else 1 << 24
    g = glmod._Graph(n=n, nnz=10, row_ptr=fake.value, col_idx=fake.value, weight=fake.value,
                     weight_dtype=1, order=None, layout=glmod.LAYOUTS["grid"], laplacian=0,
                     grid_height=h, grid_width=w if (h, w) != (2, 3) else 4)
    out = ctypes.c_void_p()
    assert lib.gl_operator_create(ctypes.byref(g), 1, None, ctypes.byref(out)) == 1
    assert out.value is None
    assert b"grid" in lib.gl_last_error()


def test_grid_operator_rejects_order():
    lib = gl.load_library()
    fake = ctypes.c_void_p(4096)
    g = glmod._Graph(n=6, nnz=10, row_ptr=fake.value, col_idx=fake.value, weight=fake.value,
                     weight_dtype=1, order=fake.value, layout=glmod.LAYOUTS["grid"], laplacian=0,
                     grid_height=2, grid_width=3)
    out = ctypes.c_void_p()
    assert lib.gl_operator_create(ctypes.byref(g), 1, None, ctypes.byref(out)) == 1
    assert b"order" in lib.gl_last_error()


def _fake_handle(magic: int):
    """A host buffer standing in for a handle of another type: only its first
    8 bytes (the type tag) are read before the entry point rejects it."""
    buf = ctypes.create_string_buffer(4096)
    ctypes.memmove(buf, int(magic).to_bytes(8, "little"), 8)
    return buf


@pytest.mark.parametrize("magic", [0, 0x7365727665722121, 0x6f70657261746f72 ^ 1])
def test_operator_entry_points_reject_foreign_handles(magic):
    # a server handle (its tag), a zeroed block or a near miss where an
    # operator is expected: rejected, nothing freed or launched
    lib = gl.load_library()
    buf = _fake_handle(magic)
    h = ctypes.cast(buf, ctypes.c_void_p)
    n = ctypes.c_int64()
    assert lib.gl_operator_info(h, ctypes.byref(n), None, None, None, None) == 1
    assert lib.gl_operator_layout(h, None, None, None, None, None) == 1
    nb = ctypes.c_size_t()
    assert lib.gl_solve_workspace_size(h, 1, 1, ctypes.byref(nb)) == 1
    assert lib.gl_power_workspace_size(h, ctypes.byref(nb)) == 1
    fake = ctypes.c_void_p(4096)
    p = _params()
    assert lib.gl_solve(h, ctypes.byref(p), 1, fake, 1, fake, fake, 1 << 20, None, None) == 1
    assert lib.gl_laplacian_apply(h, 1, 1, fake, fake, None) == 1
    assert lib.gl_operator_destroy(h) == 1
    assert b"operator" in lib.gl_last_error()
    # the buffer was not freed or modified
    assert int.from_bytes(buf.raw[:8], "little") == magic


@pytest.mark.parametrize("magic", [0, 0x6f70657261746f72])
def test_server_entry_points_reject_foreign_handles(magic):
    # an operator handle (its tag) or a zeroed block where a server is expected
    lib = gl.load_library()
    buf = _fake_handle(magic)
    h = ctypes.cast(buf, ctypes.c_void_p)
    v = [ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t(), ctypes.c_int64()]
    assert lib.gl_server_info(h, *[ctypes.byref(x) for x in v]) == 1
    assert lib.gl_server_cancel(h, 1) == 1
    res = glmod._Result()
    assert lib.gl_server_poll(h, 1, 0, ctypes.byref(res)) == 1
    req = glmod._Request()
    t = ctypes.c_uint64()
    assert lib.gl_server_submit(h, ctypes.byref(req), ctypes.byref(t)) == 1
    assert lib.gl_server_destroy(h) == 1
    assert b"server" in lib.gl_last_error()
    assert int.from_bytes(buf.raw[:8], "little") == magic


@pytest.mark.parametrize("kind,nbytes,reps,addr", [
    (2, 1 << 20, 1, 4096), (0, 1 << 19, 1, 4096), (0, (1 << 20) + 1, 1, 4096), (1, 1 << 20, 0, 4096),
    (1, 1 << 20, 10001, 4096), (0, 1 << 20, 1, 4100), (0, 1 << 20, 1, 0),
])
def test_time_stream_rejects_bad_arguments(kind, nbytes, reps, addr):
    # checked on the host before any launch (dummy device address)
    lib = gl.load_library()
    out = ctypes.c_double()
    assert lib.gl_time_stream(kind, ctypes.c_void_p(addr) if addr else None, nbytes, reps,
                              ctypes.byref(out), None) == 1
