"""Write tests/golden/precision_floor.json: for each workload, storage pair
and parameter set, how far the reduced-precision run of the method
(oracle/precision.py) lands from the float64 oracle after the workload's
fixed schedule.  CPU only; calls nothing but oracle/ and the input
generators.

    python -m oracle.floor_table [--quick]

The stiff parameters eps = 1, c = 3 (the smallest c that keeps the second
convex part of the DCA splitting convex for |u| <= 1.155, Section 3) make the
DCA map expand perturbations of undecided nodes (u near 0) by
(c + 1/eps)/c = 4/3 per step, so rounding errors grow by (4/3)^T over T steps;
eps = 100, c = 101, eta = 100 are the paper's values for its MNIST run
(Section 5.2), where the map contracts.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import c_oracle, precision  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "precision_floor.json")

STIFF = dict(eps=1.0, c=3.0, eta=1000.0)
MNIST = dict(eps=100.0, c=101.0, eta=100.0)

# (workload, small, parameter set name, parameter override, storage pairs)
CASES = [
    (1, False, "given (1, 3, 1000)", {}, [("f32", "f32"), ("bf16", "bf16"), ("bf16", "f32")]),
    (3, False, "stiff (1, 3, 1000)", STIFF, [("f32", "f32"), ("bf16", "bf16"), ("bf16", "f32")]),
    (3, False, "MNIST (100, 101, 100)", MNIST, [("f32", "f32"), ("bf16", "bf16"), ("bf16", "f32")]),
    (2, False, "image (100, 11, 100)", {}, [("f32", "f32"), ("bf16", "f16")]),
    (4, False, "image (100, 11, 100)", {}, [("f32", "f32"), ("bf16", "f16")]),
]


def run_case(cfg, small, pname, over, pairs):
    from synth import make_problem
    t0 = time.perf_counter()
    p = make_problem(cfg, small=small)
    rp, col, w = p.graph.numpy()
    kw = dict(eps=p.eps, c=p.c, eta=p.eta)
    kw.update(over)
    lam = 2.0
    if p.precond == "richardson":
        x0 = np.random.default_rng(10_000 + p.seed).uniform(-1.0, 1.0, p.n)
        _, lam = c_oracle.power_max_eig(p.n, rp, col, w, x0, 150)
    sched = dict(precond=p.precond, outer=p.outer, sweeps=p.sweeps, delta0=p.delta0,
                 lambda_max=lam, step_k=p.step_k)
    U64, _, _ = c_oracle.dca_solve(p.n, rp, col, w, p.labels, p.u0, **kw, **sched)
    rows = []
    for sw, su in pairs:
        Ur = precision.dca_solve_rounded(p.n, rp, col, w, p.labels, p.u0, store_w=sw,
                                         store_u=su, **kw, **sched)
        g = precision.gap(Ur, U64, p.n, rp, col, w, p.labels, kw["eps"], kw["eta"])
        g.update({"workload": p.name, "n": p.n, "K": p.K, "parameters": pname,
                  "eps": kw["eps"], "c": kw["c"], "eta": kw["eta"], "store_w": sw,
                  "store_u": su, "outer": p.outer, "sweeps": p.sweeps, "precond": p.precond})
        rows.append(g)
        print(f"{p.name:28s} {pname:22s} {sw:>4s}/{su:<4s} max|dU| {g['max_abs_dU']:.3e} "
              f"p99.9 {g['p999_abs_dU']:.3e} labels {g['label_agreement']:.6f} "
              f"dF/F {g['energy_rel_diff']:.2e}", flush=True)
    print(f"  ({time.perf_counter() - t0:.0f} s)", flush=True)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="workloads 1 and 3 only")
    ap.add_argument("--out", default=OUT)
    a = ap.parse_args()
    rows = []
    for cfg, small, pname, over, pairs in CASES:
        if a.quick and cfg not in (1, 3):
            continue
        rows += run_case(cfg, small, pname, over, pairs)
    rec = {"what": "distance of a reduced-precision run of the DCA (stored values rounded to "
                   "the storage types, float32 arithmetic) from the float64 oracle after each "
                   "workload's fixed schedule",
           "script": "oracle/floor_table.py", "cases": rows}
    with open(a.out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(f"wrote {a.out}")


if __name__ == "__main__":
    main()
