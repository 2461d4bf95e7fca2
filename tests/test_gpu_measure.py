"""GPU checks of the measurement helper behind the benchmark's roofline:
gl_time_sweeps launches the solve's sweep kernel back to back and reports the
mean time per launch; it must leave U untouched and reject bad counts."""

import math

import numpy as np
import pytest
import torch

import paper_2303_14495_amd as gl
from tests.gpu_helpers import DEV, make_operator, problem, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("layout", ["grid", "tile", "direct"])
@pytest.mark.parametrize("store", [("bf16", "f16"), ("f32", "f32")])
def test_time_sweeps(layout, store):
    p = problem(4, small=True)
    store_w, store_u = store
    op = make_operator(p, store_w, layout=layout)
    lab = torch.from_numpy(p.labels).to(DEV)
    dt = {"f16": torch.float16, "f32": torch.float32}[store_u]
    U = torch.from_numpy(p.u0).to(DEV, dt).contiguous()
    before = U.clone()
    # the first launch of a kernel also loads its code: warm up once
    gl.time_sweeps(op, lab, U, eps=p.eps, c=p.c, eta=p.eta, precond=p.precond, lambda_max=1.4, reps=1)
    t1 = gl.time_sweeps(op, lab, U, eps=p.eps, c=p.c, eta=p.eta, precond=p.precond, lambda_max=1.4, reps=1)
    t20 = gl.time_sweeps(op, lab, U, eps=p.eps, c=p.c, eta=p.eta, precond=p.precond, lambda_max=1.4, reps=20)
    say(f"time_sweeps {layout} {store}: reps=1 {t1 * 1e3:.1f} us, reps=20 {t20 * 1e3:.1f} us per launch")
    assert math.isfinite(t1) and math.isfinite(t20) and t1 > 0 and t20 > 0
    # the mean per launch of a longer run is no longer than a single launch by much
    assert t20 <= 3 * t1 + 0.05
    assert torch.equal(U, before)
    for bad in (0, 10001):
        with pytest.raises(gl.GLError):
            gl.time_sweeps(op, lab, U, eps=p.eps, c=p.c, eta=p.eta, precond=p.precond, lambda_max=1.4,
                           reps=bad)


def test_time_stream_ceilings():
    # the plain streaming and copy kernels behind the measured HBM ceiling:
    # finite times, the copy really copies, the read leaves the buffer alone
    nb = 256 << 20
    buf = torch.randint(0, 256, (nb,), dtype=torch.uint8, device=DEV)
    ref = buf.clone()
    tr = gl.time_stream(buf, "read", 5)
    assert torch.equal(buf, ref)
    tc = gl.time_stream(buf, "copy", 5)
    torch.cuda.synchronize()
    assert torch.equal(buf[nb // 2:], ref[: nb // 2]) and torch.equal(buf[: nb // 2], ref[: nb // 2])
    say(f"time_stream 256 MiB: read {nb / tr / 1e6:.0f} GB/s, copy {nb / tc / 1e6:.0f} GB/s")
    assert 0 < tr < 50 and 0 < tc < 50
    with pytest.raises(gl.GLError):
        gl.time_stream(buf[:1000], "read", 1)
