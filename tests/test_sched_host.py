"""CPU tests of the server's host logic (no GPU): the arena allocator, the
footprint, the direct geometry and the per-solve sweep schedule, compiled from
the library's header with g++ under AddressSanitizer/UBSan; and server
argument checks through the C ABI that fail before any HIP call."""

import ctypes
import os
import shutil
import subprocess

import pytest

import paper_2303_14495_amd as gl
from paper_2303_14495_amd import gl as glmod

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_sched_host_logic(tmp_path):
    exe = tmp_path / "sched_host_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-omit-frame-pointer", os.path.join(HERE, "sched_host_test.cpp"),
                    "-o", str(exe)], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "ok" in res.stdout


@pytest.mark.parametrize("kw", [
    dict(hbm_budget_bytes=1000), dict(max_slots=0), dict(max_slots=65), dict(max_pending=0),
    dict(store_w=0), dict(store_u=7), dict(ticks_in_flight=0), dict(ticks_in_flight=9),
    dict(reserved=1),
])
def test_server_config_rejected(kw):
    lib = gl.load_library()
    base = dict(hbm_budget_bytes=1 << 30, max_slots=8, max_pending=16, store_w=2, store_u=2,
                ticks_in_flight=2, reserved=0)
    base.update(kw)
    cfg = glmod._ServerConfig(**base)
    h = ctypes.c_void_p()
    assert lib.gl_server_create(ctypes.byref(cfg), ctypes.byref(h)) != 0
    assert not h.value


def test_server_null_arguments():
    lib = gl.load_library()
    assert lib.gl_server_submit(None, None, None) == 1
    assert lib.gl_server_poll(None, 1, 0, None) == 1
    assert lib.gl_server_cancel(None, 1) == 1
    assert lib.gl_server_destroy(None) == 0


def test_request_bytes():
    peak, held = gl.Server.request_bytes(10000, 150000, 4, 20, 4, "bf16", "bf16")
    assert 0 < held < peak
    p32, h32 = gl.Server.request_bytes(10000, 150000, 4, 20, 4, "f32", "f32")
    assert p32 > peak and h32 > held
    for bad in [dict(n=1), dict(K=11), dict(sweeps=0)]:
        kw = dict(n=10000, nnz=150000, K=4, outer=20, sweeps=4)
        kw.update(bad)
        with pytest.raises(glmod.GLError):
            gl.Server.request_bytes(**kw)
    with pytest.raises(glmod.GLError):
        gl.Server.request_bytes(100, 1000, 2, 1, 1, "f64", "f32")
