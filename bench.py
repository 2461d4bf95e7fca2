"""Benchmark of the preconditioned-DCA inner solve on one MI355X.

Workload (default): the 2048 x 2048 textured-image segmentation graph
(4 194 304 nodes, symmetrised 20-NN within a 15 x 15 window, self-tuning
weights), K = 4 phases, 0.5 % labelled pixels, 10 DCA steps x 8 generalized-
Richardson sweeps, weights stored in bf16 and the label field in f16 with
f32 accumulation.  One step = one DCA solve (all sweeps with the fused
right-hand side, update, energy and residual reductions) plus labelling, on an
operator and a lambda_max estimate built once per graph (their times are
reported separately).  The same solve with f32 storage, the roofline of the
sweep kernel and the float64 CPU oracle on the host cores are reported beside
it.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--workload 4]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "Laplacian-sweep HBM GB/s + DCA solves/s (FP32 vs BF16); served p50/p99 latency"
DSIZE = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "grid_sweep_image2048_k4_traffic.json")
# sources whose change invalidates recorded counter traffic of the sweep kernel
WINDOW_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "window_sweep_1024_r12_traffic.json")  # + _<weights>
HBM_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "grid_sweep_image4096_k4_traffic.json")  # + _<weights>
# the sources of each sweep kernel whose counter summaries bench.py reads: a
# summary counts only while their SHA-256 matches the one it was taken with
TRAFFIC_SOURCES = {
    "grid": ["gl_grid.hpp", "gl_device.hpp", "gl_kernels.hpp", "gl_launch_impl.hpp",
             "gl_internal.hpp", "gl_layout.hpp", "gl_unit_grid_f16.hip",
             "gl_unit_grid_bf16.hip", "gl_unit_grid_f32.hip"],
    "window": ["gl_window.hpp", "gl_window.hip", "gl_device.hpp", "gl_kernels.hpp",
               "gl_launch_impl.hpp", "gl_internal.hpp", "gl_unit_f32.hip"],
}


def sweep_source_hash(kind="grid"):
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_2303_14495_amd", "csrc", f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def recorded_traffic(workload_name, storage, path=TRAFFIC_FILE, kind="grid"):
    """HBM bytes per sweep launch from the committed counter summary (FETCH_SIZE
    and WRITE_SIZE of the sweep kernel, each scaled by what the counter reads
    for a 1 GiB elementwise copy), or None when the summary is missing, is for
    another workload or storage, or predates the current kernel sources."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if (t.get("source_sha256") != sweep_source_hash(kind) or t.get("workload") != workload_name
            or t.get("storage") != storage):
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0


def sweep_bytes(info, n, K, store_u):
    """Algorithmic bytes of one sweep: the operator's index, weight, row-offset
    and order streams as stored (padding included), the compulsory read of the
    gathered field, the own-row read of u^t, the write of the new field, and
    the labels."""
    return info["stream_bytes"] + 3 * n * K * DSIZE[store_u] + 4 * n


# index bytes stored per entry slot, by layout (padding slots carry them too)
SLOT_INDEX_BYTES = {"grid": 1, "tile": 2, "direct": 4, "window": 0}


def method_bytes(info, n, K, store_w, store_u):
    """sweep_bytes without the layout's padding slots: what the graph's own
    nonzeros, row data and the field cost per sweep."""
    pad = info["stored_entries"] - info["nnz"]
    return (sweep_bytes(info, n, K, store_u)
            - pad * (SLOT_INDEX_BYTES[info["layout"]] + DSIZE[store_w]))


def ceilings(dev, gib=4, reps=20):
    """The practical HBM ceiling on this GPU: the library's plain read-only
    streaming kernel and plain copy kernel over `gib` GiB (far beyond the
    caches), mean time per launch over `reps` back-to-back launches."""
    import torch
    import paper_2303_14495_amd as gl
    nb = gib << 30
    buf = torch.empty(nb, dtype=torch.uint8, device=dev)
    gl.time_stream(buf, "read", 3)
    gl.time_stream(buf, "copy", 3)
    read_ms = gl.time_stream(buf, "read", reps)
    copy_ms = gl.time_stream(buf, "copy", reps)
    del buf
    torch.cuda.empty_cache()
    return {"bytes": nb, "read_gbps": nb / (read_ms * 1e-3) / 1e9,
            "copy_gbps": nb / (copy_ms * 1e-3) / 1e9,
            "kernels": "stream_read_kernel (reads all bytes), stream_copy_kernel (reads half, "
                       "writes half); 16-byte non-temporal vectors, 4096 x 256 lanes"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--sweep-reps", type=int, default=40)
    ap.add_argument("--no-served", action="store_true", help="skip the served stream")
    ap.add_argument("--no-window", action="store_true", help="skip the window-graph run")
    ap.add_argument("--no-grid", action="store_true",
                    help="image workloads: tile layout in Z-order instead of the grid layout")
    ap.add_argument("--window-only", action="store_true")
    ap.add_argument("--served-only", action="store_true")
    ap.add_argument("--served-count", type=int, default=256)
    ap.add_argument("--served-rate", type=float, default=0.8,
                    help="arrival rate as a fraction of one-at-a-time f32 capacity")
    ap.add_argument("--served-budget-gib", type=float, default=32.0)
    ap.add_argument("--served-rates", default="",
                    help="comma-separated extra arrival rates, as multiples of the f32 capacity")
    ap.add_argument("--served-slots", type=int, default=32)
    ap.add_argument("--no-hbm-scale", action="store_true",
                    help="skip the 4096 x 4096 grid sweep (over 1 GB per sweep)")
    ap.add_argument("--hbm-scale-only", action="store_true")
    ap.add_argument("--no-precond", action="store_true",
                    help="skip the preconditioner / step-size / Laplacian comparison")
    ap.add_argument("--precond-only", action="store_true")
    ap.add_argument("--knn-only", action="store_true",
                    help="only the graph-construction section (exact kNN in R^10 and R^784)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="finish with a 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed_solves(op, labels, U, p, lam, steps, warmup):
    import torch
    import paper_2303_14495_amd as gl
    kw = dict(eps=p.eps, c=p.c, eta=p.eta, precond=p.precond, outer=p.outer, sweeps=p.sweeps,
              delta0=p.delta0, lambda_max=lam, step_k=p.step_k)
    stats = torch.empty(gl.stats_length(U.shape[1], p.outer, p.sweeps), dtype=torch.float64,
                        device=U.device)
    for _ in range(warmup):
        op.solve(labels, U, stats_out=stats, **kw)
        gl.assign_labels(U)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        op.solve(labels, U, stats_out=stats, **kw)
        gl.assign_labels(U)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    return wall, ev_ms, stats


SERVED_PARAMS = dict(eps=100.0, c=11.0, eta=100.0, precond="damped_jacobi", outer=20, sweeps=4)


class PinnedPool:
    """Page-locked host staging for the request arrays: 1 GiB pinned buffers
    carved into 256-byte aligned pieces (the way a server front end would
    receive requests into DMA-able memory)."""

    def __init__(self, chunk=1 << 30):
        self.chunk, self.bufs, self.off = chunk, [], 0

    def put(self, arr):
        import numpy as np
        import torch
        arr = np.ascontiguousarray(arr)
        nb = max(arr.nbytes, 1)
        need = (nb + 255) // 256 * 256
        if need > self.chunk:
            buf, off = torch.empty(need, dtype=torch.uint8, pin_memory=True), 0
            self.bufs.append(buf)
        else:
            if not self.bufs or self.off + need > self.chunk:
                self.bufs.append(torch.empty(self.chunk, dtype=torch.uint8, pin_memory=True))
                self.off = 0
            buf, off = self.bufs[-1], self.off
            self.off += need
        t = buf[off:off + arr.nbytes].view(torch.from_numpy(arr[:0].copy()).dtype).view(arr.shape)
        t.numpy()[...] = arr
        return t


def served_requests(dev, count, seed, pool):
    """The served stream's requests in pinned host memory; graphs built on
    the GPU with the library's exact kNN, then union-symmetrised with
    self-tuning weights."""
    import numpy as np
    import torch
    import paper_2303_14495_amd as gl
    from synth.configs import served_problem, served_stream

    def knn(x, k):
        return gl.knn(x.to(torch.float32), k, with_distances=False)[0].to(torch.int64)

    reqs = []
    for item in served_stream(count, seed=seed):
        p = served_problem(item, device=dev, knn=knn)
        rp, col, w = p.graph.numpy()
        r = {"n": p.n, "nnz": int(col.size), "K": p.K, "t": item.arrival, "truth": p.truth,
             "rp": pool.put(rp), "col": pool.put(col), "w": pool.put(w),
             "labels": pool.put(np.asarray(p.labels, dtype=np.int32)),
             "u0": pool.put(np.asarray(p.u0, dtype=np.float32))}
        reqs.append(r)
        del p, rp, col, w
    torch.cuda.synchronize()
    return reqs


def fp32_one(dev, r):
    """One request alone, plain f32: upload, operator, solve, labels, download."""
    import torch
    import paper_2303_14495_amd as gl
    op = gl.Operator(r["rp"].to(dev, non_blocking=True), r["col"].to(dev, non_blocking=True),
                     r["w"].to(dev, non_blocking=True), store_w="f32")
    U = r["u0"].to(dev, non_blocking=True)
    lab = r["labels"].to(dev, non_blocking=True)
    op.solve(lab, U, stats=True, **SERVED_PARAMS)
    cls = gl.assign_labels(U).cpu().numpy()
    U = U.cpu().numpy()
    op.close()
    return U, cls


def run_fp32_stream(dev, reqs, arrivals):
    """Requests one after another in arrival order (None: all at time 0);
    returns (latencies s, makespan s, classes)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat, out = [], []
    for i, r in enumerate(reqs):
        a = 0.0 if arrivals is None else arrivals[i]
        while time.perf_counter() - t0 < a:
            time.sleep(min(1e-3, max(0.0, a - (time.perf_counter() - t0))))
        _, cls = fp32_one(dev, r)
        lat.append(time.perf_counter() - t0 - a)
        out.append(cls)
    return lat, time.perf_counter() - t0, out


def run_served_stream(reqs, arrivals, budget, slots):
    """Submit at the arrival times from one thread, collect from another;
    returns (latencies s, makespan s, classes, server counters)."""
    import threading
    import paper_2303_14495_amd as gl
    srv = gl.Server(budget, max_slots=slots, max_pending=len(reqs) + 1, store_w="bf16",
                    store_u="bf16")
    t_srv = time.perf_counter()  # the server's own clock starts at creation
    tickets = [None] * len(reqs)
    ready = threading.Semaphore(0)
    res = [None] * len(reqs)

    def collect():
        for i in range(len(reqs)):
            ready.acquire()
            res[i] = srv.poll(tickets[i])

    th = threading.Thread(target=collect)
    th.start()
    t0 = time.perf_counter()
    for i, r in enumerate(reqs):
        a = 0.0 if arrivals is None else arrivals[i]
        while time.perf_counter() - t0 < a:
            time.sleep(min(1e-3, max(0.0, a - (time.perf_counter() - t0))))
        tickets[i] = srv.submit(r["rp"].numpy(), r["col"].numpy(), r["w"].numpy(),
                                r["labels"].numpy(), r["u0"].numpy(), borrow=True,
                                **SERVED_PARAMS)
        ready.release()
    th.join()
    info = srv.info()
    srv.close()
    off = t0 - t_srv
    lat = [(x["t_done"] - off) - (0.0 if arrivals is None else arrivals[i])
           for i, x in enumerate(res)]
    makespan = max(x["t_done"] for x in res) - off
    bad = [x["status"] for x in res if x["status"] != "GL_OK"]
    if bad:
        raise RuntimeError(f"served requests failed: {bad[:5]}")
    return lat, makespan, [x["labels"] for x in res], info


def served_bench(dev, count, rate_factor, budget_gib, slots, extra_rates=()):
    import numpy as np
    log(f"served stream: generating {count} requests")
    t = time.perf_counter()
    pool = PinnedPool()
    reqs = served_requests(dev, count, seed=4, pool=pool)
    ns = [r["n"] for r in reqs]
    log(f"  generated in {time.perf_counter() - t:.1f} s; N {min(ns)}..{max(ns)}, "
        f"sum nnz {sum(r['nnz'] for r in reqs)}")
    budget = int(budget_gib * (1 << 30))
    # warm both paths on the first requests, then measure capacity (all at t = 0)
    run_fp32_stream(dev, reqs[:4], None)
    run_served_stream(reqs[:4], None, budget, slots)
    lat32_cap, span32_cap, cls32 = run_fp32_stream(dev, reqs, None)
    cap32 = count / span32_cap
    lat_s_cap, span_s_cap, cls_s, info_cap = run_served_stream(reqs, None, budget, slots)
    log(f"  capacity: fp32 one-at-a-time {cap32:.1f} solves/s, served bf16 "
        f"{count / span_s_cap:.1f} solves/s ({info_cap['ticks']} ticks)")
    # Poisson arrivals (unit-rate gaps of the stream scaled to the target rate)
    rate = rate_factor * cap32
    arrivals = [r["t"] / rate for r in reqs]
    lat32, span32, _ = run_fp32_stream(dev, reqs, arrivals)
    lat_s, span_s, _, info = run_served_stream(reqs, arrivals, budget, slots)
    agree = float(np.mean([np.mean(a == b) for a, b in zip(cls_s, cls32)]))
    acc_s = float(np.mean([np.mean(c == r["truth"]) for c, r in zip(cls_s, reqs)]))

    def pct(v, q):
        return float(np.percentile(np.asarray(v) * 1e3, q))

    out = {
        "requests": count, "rate_factor": rate_factor, "arrival_rate_per_s": rate,
        "hbm_budget_gib": budget_gib, "max_slots": slots,
        "served_bf16": {"solves_per_s": count / span_s, "p50_ms": pct(lat_s, 50),
                        "p99_ms": pct(lat_s, 99), "capacity_solves_per_s": count / span_s_cap,
                        "ticks": info["ticks"]},
        "fp32_one_at_a_time": {"solves_per_s": count / span32, "p50_ms": pct(lat32, 50),
                               "p99_ms": pct(lat32, 99), "capacity_solves_per_s": cap32},
        "label_agreement_served_vs_fp32": agree,
        "served_accuracy_vs_truth": acc_s,
    }
    log(f"  at {rate:.1f} req/s: served p50 {out['served_bf16']['p50_ms']:.1f} ms p99 "
        f"{out['served_bf16']['p99_ms']:.1f} ms; fp32 p50 "
        f"{out['fp32_one_at_a_time']['p50_ms']:.1f} ms p99 "
        f"{out['fp32_one_at_a_time']['p99_ms']:.1f} ms; agreement {agree:.5f}")
    # the same stream at other arrival rates (multiples of the f32 capacity)
    sweep = []
    for f in extra_rates:
        r2 = f * cap32
        arr2 = [r["t"] / r2 for r in reqs]
        l32, sp32, _ = run_fp32_stream(dev, reqs, arr2)
        ls, sps, _, inf2 = run_served_stream(reqs, arr2, budget, slots)
        row = {"rate_factor": f, "arrival_rate_per_s": r2,
               "served_bf16": {"solves_per_s": count / sps, "p50_ms": pct(ls, 50), "p99_ms": pct(ls, 99)},
               "fp32_one_at_a_time": {"solves_per_s": count / sp32, "p50_ms": pct(l32, 50),
                                      "p99_ms": pct(l32, 99)}}
        sweep.append(row)
        log(f"  at {f:.2f} x capacity ({r2:.1f} req/s): served p50 {row['served_bf16']['p50_ms']:.1f} ms "
            f"p99 {row['served_bf16']['p99_ms']:.1f} ms; fp32 p50 {row['fp32_one_at_a_time']['p50_ms']:.1f} ms "
            f"p99 {row['fp32_one_at_a_time']['p99_ms']:.1f} ms")
    if sweep:
        out["rate_sweep"] = sweep
    return out


def unsupervised_bench(dev):
    """Unsupervised run of the paper's clustering section on the 4096-point
    two-component mixture: second eigenvector of L_s (Lanczos, 64 steps per
    restart, residual <= 1e-5), then 20 x 4 damped-Jacobi DCA steps with no
    labels from u^0 = v_2 / max |v_2| (eps = 100, c = 11, eta = 100)."""
    import numpy as np
    import torch
    import paper_2303_14495_amd as gl
    from synth import make_problem
    p = make_problem(1, device=dev)
    g = p.graph
    op = gl.Operator(g.row_ptr, g.col, g.weight.to(torch.float64), store_w="f32")
    x0 = torch.from_numpy(np.random.default_rng(20_000).uniform(-1, 1, p.n)).to(dev, torch.float32)
    op.second_eigenpair(x0, krylov=64, max_restarts=50, tol=1e-5)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam, v, res, restarts = op.second_eigenpair(x0, krylov=64, max_restarts=50, tol=1e-5)
    t_eig = time.perf_counter() - t0
    labels = torch.full((p.n,), -1, dtype=torch.int32, device=dev)
    kw = dict(eps=100.0, c=11.0, eta=100.0, precond="damped_jacobi", outer=20, sweeps=4)
    U = (v / v.abs().max()).view(-1, 1).contiguous()
    op.solve(labels, U.clone(), stats=False, **kw)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op.solve(labels, U, stats=False, **kw)
    cls = gl.assign_labels(U).cpu().numpy()
    t_solve = time.perf_counter() - t0
    acc = float(max(np.mean(cls == p.truth), np.mean(cls != p.truth)))
    op.close()
    return {"workload": p.name, "n": p.n, "second_eigenpair_ms": t_eig * 1e3, "lambda2": lam,
            "residual": res, "restarts": restarts, "solve_ms": t_solve * 1e3,
            "accuracy_vs_truth": acc}


def window_bench(dev, steps, warmup, reps):
    """The paper's own image graph (window proximity + patch similarity,
    Section 2.2) through the matrix-free window operator: a 1024 x 1024
    rectangles image, 25 x 25 window, 5 x 5 patches, sigma = log(N) + 1,
    K = 1, 1% labelled pixels, 10 DCA steps x 4 damped-Jacobi sweeps
    (eps = 100, c = 11, eta = 100).  Weights are built on the GPU from the
    image; BF16 and F32 weight storage are timed on the same input."""
    import numpy as np
    import torch
    import paper_2303_14495_amd as gl
    from synth.configs import window_problem
    p = window_problem()
    img = torch.from_numpy(p.image).to(dev, torch.float32)
    labels = torch.from_numpy(p.labels).to(dev)
    out = {"workload": p.name, "n": p.n, "window": 2 * p.rw + 1, "patch": 2 * p.rp + 1,
           "sigma": p.sigma, "K": p.K, "outer_steps": p.outer, "sweeps": p.sweeps,
           "precond": p.precond}
    fields = {}
    for store_w in ("bf16", "f32"):
        gl.Operator.window(img, p.rw, p.rp, p.sigma, store_w=store_w).close()  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op = gl.Operator.window(img, p.rw, p.rp, p.sigma, store_w=store_w)
        torch.cuda.synchronize()
        t_build = time.perf_counter() - t0
        info = op.info()
        U = torch.from_numpy(p.u0).to(dev, torch.float32).contiguous()
        U0 = U.clone()
        wall, ev_ms, _ = timed_solves(op, labels, U, p, 2.0, steps, warmup)
        Uf = U0.clone()
        op.solve(labels, Uf, eps=p.eps, c=p.c, eta=p.eta, precond=p.precond, outer=p.outer,
                 sweeps=p.sweeps, stats=False)
        fields[store_w] = Uf.double().cpu().numpy()[:, 0]
        sweep_ms = gl.time_sweeps(op, labels, U0, eps=p.eps, c=p.c, eta=p.eta,
                                  precond=p.precond, reps=reps)
        # algorithmic bytes: one weight per pair of neighbours (W is stored
        # once), the gathered field once, u^t, the new field and the labels
        # (the stored zeros of border offsets, the halo re-reads and the region
        # sums the two passes of a product exchange are not counted)
        wsize = 2 if store_w == "bf16" else 4
        B = info["nnz"] // 2 * wsize + 3 * p.n * 4 + 4 * p.n
        out[store_w] = {"solves_per_s": steps / wall, "ms_per_solve": wall / steps * 1e3,
                        "sweep_kernel_ms": sweep_ms, "sweep_bytes": B,
                        "sweep_gbps": B / (sweep_ms * 1e-3) / 1e9,
                        "frac_of_hbm_peak": B / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                        "weight_build_ms": t_build * 1e3, "nnz": info["nnz"],
                        "stored_entries": info["stored_entries"],
                        "kernel": f"window_part_kernel<1, {store_w}, f32> + window_sweep_kernel<1, {store_w}, f32>",
                        "traffic": recorded_traffic(p.name, f"{store_w}/f32",
                                                    WINDOW_TRAFFIC_FILE.replace(
                                                        ".json", f"_{store_w}.json"),
                                                    kind="window")}
        op.close()
        del U, U0, Uf
        torch.cuda.empty_cache()
    a, b = fields["bf16"], fields["f32"]
    dec = np.abs(b) > 2e-2
    out["bf16_vs_f32"] = {"max_abs_diff": float(np.abs(a - b).max()),
                          "label_agreement_decided": float(np.mean((a[dec] >= 0) == (b[dec] >= 0))),
                          "decided_fraction": float(dec.mean())}
    out["accuracy_vs_ground_truth_f32"] = float(np.mean((b >= 0) == (p.truth == 1)))
    out["csr_bytes_per_nonzero"] = {"window_bf16": 1, "csr_bf16_int32": 6}
    return out


def knn_graph_bench(dev):
    """Graph construction on the GPU (exact kNN, then the union-symmetric
    graph with local-scaling weights): 262 144 points in R^10 from a
    5-component mixture, k = 10, bandwidth from the 7th neighbour."""
    import numpy as np
    import torch
    import paper_2303_14495_amd as gl
    rng = np.random.default_rng(31)
    n, d, k = 262144, 10, 10
    means = 3.0 * rng.standard_normal((5, d))
    x = (means[rng.integers(0, 5, n)] + rng.standard_normal((n, d))).astype(np.float32)
    xt = torch.from_numpy(x).to(dev)
    idx, d2 = gl.knn(xt, k)  # warm-up
    gl.knn_graph(idx, d2, 7)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx, d2 = gl.knn(xt, k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rp, col, w = gl.knn_graph(idx, d2, 7)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out = {"points": n, "dim": d, "k": k, "scale_rank": 7, "knn_ms": (t1 - t0) * 1e3,
           "graph_ms": (t2 - t1) * 1e3, "nnz": int(col.numel()),
           "knn_pair_rate_per_s": n * (n - 1) / (t1 - t0)}
    del xt, idx, d2, rp, col, w
    # wide features through the matrix cores: the 784-dimensional clustering
    # workload's points (70 000, 10 components), k = 10
    r = np.random.default_rng(2)
    means = r.standard_normal((10, 784))
    nw = 70000
    xw = np.maximum(means[r.integers(0, 10, nw)] + 0.8 * r.standard_normal((nw, 784)), 0.0)
    xwt = torch.from_numpy(xw.astype(np.float32)).to(dev)
    del xw
    gl.knn(xwt, 10)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gl.knn(xwt, 10)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out["wide"] = {"points": nw, "dim": 784, "k": 10, "knn_ms": (t1 - t0) * 1e3,
                   "exact_rescans": gl.knn_fallback_rows(),
                   "pair_tflops": 2.0 * nw * nw * 784 / (t1 - t0) / 1e12}
    return out


def hbm_scale_bench(dev, reps):
    """Workload 4's recipe on a 4096 x 4096 image (16.8 M pixels, about 370 M
    stored nonzeros): the grid sweep at more than 1 GB per sweep, far beyond
    the 256 MB Infinity Cache, with bf16/f16 and f32 storage; per form the
    sweep time (back-to-back launches) and three timed solves."""
    import numpy as np
    import torch
    import paper_2303_14495_amd as gl
    from synth.configs import texture_problem
    t0 = time.perf_counter()
    p = texture_problem(4096, device=dev)
    g = p.graph
    torch.cuda.synchronize()
    out = {"workload": p.name, "n": p.n, "nnz": g.nnz, "K": p.K, "outer_steps": p.outer,
           "sweeps": p.sweeps, "graph_build_s": time.perf_counter() - t0}
    log(f"  {p.name}: n={p.n} nnz={g.nnz} built in {out['graph_build_s']:.1f} s")
    labels = torch.from_numpy(p.labels).to(dev)
    x0 = torch.from_numpy(np.random.default_rng(10_000 + p.seed).uniform(-1, 1, p.n)).to(
        dev, torch.float32)
    for sw, su in (("bf16", "f16"), ("f32", "f32")):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        op = gl.Operator(g.row_ptr, g.col, g.weight, store_w=sw, layout="grid",
                         grid=p.extra["grid"])
        torch.cuda.synchronize()
        t_create = time.perf_counter() - t1
        _, lam = op.power_max_eig(x0, 150)
        U = torch.from_numpy(p.u0).to(dev, gl.TORCH_DTYPES[su]).contiguous()
        # the solves first: the sweep timing starts on a busy GPU, as in a solve
        wall, _, _ = timed_solves(op, labels, U.clone(), p, lam, 3, 1)
        sweep_ms = min(gl.time_sweeps(op, labels, U, eps=p.eps, c=p.c, eta=p.eta,
                                      precond=p.precond, delta0=p.delta0, lambda_max=lam,
                                      step_k=p.step_k, reps=reps) for _ in range(3))
        info = op.info()
        B = sweep_bytes(info, p.n, p.K, su)
        Bm = method_bytes(info, p.n, p.K, sw, su)
        out[f"{sw}/{su}"] = {
            "kernel": f"grid_sweep_kernel<{p.K}, {sw}, {su}>", "sweep_kernel_ms": sweep_ms,
            "sweep_bytes": B, "sweep_bytes_method": Bm,
            "sweep_gbps": B / (sweep_ms * 1e-3) / 1e9,
            "frac_of_hbm_peak": B / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
            "frac_method": Bm / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
            "solves_per_s": 3 / wall, "ms_per_solve": wall / 3 * 1e3,
            "operator_create_ms": t_create * 1e3, "stored_entries": info["stored_entries"],
            "traffic": recorded_traffic(p.name, f"{sw}/{su}",
                                        HBM_TRAFFIC_FILE.replace(".json", f"_{sw}.json"))}
        log(f"  {sw}/{su}: {B / 1e9:.2f} GB per sweep in {sweep_ms * 1e3:.1f} us "
            f"({out[f'{sw}/{su}']['sweep_gbps']:.0f} GB/s), {wall / 3 * 1e3:.1f} ms per solve")
        op.close()
        del U
        torch.cuda.empty_cache()
    del p, g, labels, x0
    torch.cuda.empty_cache()
    return out


def precond_bench(dev, targets=(0.99, 0.995), max_steps=500):
    """Synthetic analogs of the paper's preconditioner comparisons (Section
    5.1.3, Tables 3-6) on its own image graph: the 1024 x 1024 rectangles
    image, 25 x 25 window, 5 x 5 patches, eps = 100, c = 11, eta = 100, four
    sweeps per DCA step, f32 storage, labels given as scribbles (a short stroke
    through each rectangle and four in the background, as the paper's inputs
    mark each object with a few strokes).  For each setting: the DCA steps (and
    sweeps) until the labels first reach each accuracy target against the
    synthetic ground truth (the paper stops on DICE against its ground truth),
    and the time of one solve of that many steps.  Settings: L_s against L
    with perturbed Jacobi (Table 3); damped Jacobi, perturbed Jacobi and
    Richardson on L_s (Table 4); step sizes k = 0.01 ... 5 and infinity for
    perturbed Jacobi and Richardson (Tables 5 and 6)."""
    import numpy as np
    import torch
    import paper_2303_14495_amd as gl
    from synth.configs import window_problem
    p = window_problem(scribbles=True)
    img = torch.from_numpy(p.image).to(dev, torch.float32)
    labels = torch.from_numpy(p.labels).to(dev)
    truth = torch.from_numpy(p.truth).to(dev)
    U0 = torch.from_numpy(p.u0).to(dev, torch.float32).contiguous()
    x0 = torch.from_numpy(np.random.default_rng(10_000 + p.seed).uniform(-1, 1, p.n)).to(
        dev, torch.float32)
    ops, lam = {}, {}
    for lap in ("normalized", "unnormalized"):
        ops[lap] = gl.Operator.window(img, p.rw, p.rp, p.sigma, store_w="f32", laplacian=lap)
        lam[lap] = ops[lap].power_max_eig(x0, 150)[1]
    base = dict(eps=p.eps, c=p.c, eta=p.eta, sweeps=p.sweeps, delta0=p.delta0, stats=False)

    def run(lap, precond, k):
        op = ops[lap]
        kw = dict(base, precond=precond, lambda_max=lam[lap], step_k=k)
        U = U0.clone()
        first = {t: None for t in targets}
        acc = 0.0
        steps = 0
        while steps < max_steps and first[targets[-1]] is None:
            op.solve(labels, U, outer=1, **kw)
            steps += 1
            acc = float((gl.assign_labels(U) == truth).float().mean())
            for t in targets:
                if first[t] is None and acc >= t:
                    first[t] = steps
        # one solve of that many steps (bitwise the same iterates), timed alone
        U = U0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op.solve(labels, U, outer=steps, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        return {"laplacian": lap, "precond": precond, "step_k": "inf" if math.isinf(k) else k,
                "steps_to": {str(t): first[t] for t in targets},
                "sweeps_to": {str(t): (None if first[t] is None else first[t] * p.sweeps)
                              for t in targets},
                "steps_run": steps, "final_accuracy": acc, "ms": ms}

    inf = math.inf
    rows = []
    seen = {}
    plan = [("normalized", "perturbed_jacobi", inf), ("unnormalized", "perturbed_jacobi", inf),
            ("normalized", "damped_jacobi", inf), ("normalized", "richardson", inf)]
    plan += [("normalized", pc, k) for pc in ("perturbed_jacobi", "richardson")
             for k in (0.01, 0.05, 0.1, 1.0, 5.0)]
    for lap, pc, k in plan:
        r = run(lap, pc, k)
        seen[(lap, pc, k)] = r
        rows.append(r)
        log(f"  {lap:12s} {pc:16s} k={r['step_k']}: steps to {targets}: "
            f"{[r['steps_to'][str(t)] for t in targets]}, {r['ms']:.1f} ms")
    for op in ops.values():
        op.close()
    return {"workload": p.name, "n": p.n, "window": 2 * p.rw + 1, "storage": "f32/f32",
            "labelled": int((p.labels >= 0).sum()),
            "eps": p.eps, "c": p.c, "eta": p.eta, "sweeps_per_step": p.sweeps,
            "accuracy_targets": list(targets), "max_steps": max_steps,
            "lambda_hat": lam, "runs": rows}


def calib_copy(dev):
    """Counter calibration: one elementwise kernel that reads 1 GiB and writes
    1 GiB, far beyond the L2 and the Infinity Cache."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    log(f"calibration: mul over {src.numel() * 4} bytes in, {dst.numel() * 4} out")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU (the multi-GPU sharding is a design, not code); --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2303_14495_amd as gl
    from synth import make_problem

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.window_only:
        print(json.dumps(window_bench(dev, args.steps, args.warmup, args.sweep_reps)), flush=True)
        if args.calib_copy:
            calib_copy(dev)
        return
    if args.precond_only:
        print(json.dumps(precond_bench(dev)), flush=True)
        if args.calib_copy:
            calib_copy(dev)
        return
    if args.knn_only:
        print(json.dumps(knn_graph_bench(dev)), flush=True)
        return
    if args.hbm_scale_only:
        print(json.dumps(hbm_scale_bench(dev, args.sweep_reps)), flush=True)
        if args.calib_copy:
            calib_copy(dev)
        return
    if args.served_only:
        rates = [float(v) for v in args.served_rates.split(",") if v]
        print(json.dumps(served_bench(dev, args.served_count, args.served_rate,
                                      args.served_budget_gib, args.served_slots, rates)), flush=True)
        return
    log(f"generating workload {args.workload}")
    t = time.perf_counter()
    p = make_problem(args.workload, device=dev)
    log(f"  {p.name}: n={p.n} nnz={p.graph.nnz} K={p.K} ({time.perf_counter() - t:.1f} s)")
    g = p.graph
    order = torch.from_numpy(p.order).to(dev) if p.order is not None else None
    # image graphs: the grid layout (one-byte window-relative columns)
    grid = p.extra.get("grid") if not args.no_grid else None
    labels = torch.from_numpy(p.labels).to(dev)
    x0 = torch.from_numpy(np.random.default_rng(10_000 + p.seed).uniform(-1, 1, p.n)).to(
        dev, torch.float32)

    def run_variant(store_w, store_u, steps, warmup):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if grid is not None:
            op = gl.Operator(g.row_ptr, g.col, g.weight, store_w=store_w, layout="grid", grid=grid)
        else:
            op = gl.Operator(g.row_ptr, g.col, g.weight, store_w=store_w, order=order)
        torch.cuda.synchronize()
        t_create = time.perf_counter() - t0
        lam = 2.0
        t_power = 0.0
        if p.precond == "richardson":
            t0 = time.perf_counter()
            _, lam = op.power_max_eig(x0, 150)
            t_power = time.perf_counter() - t0
        U = torch.from_numpy(p.u0).to(dev, gl.TORCH_DTYPES[store_u]).contiguous()
        log(f"  {store_w}/{store_u}: operator {t_create * 1e3:.1f} ms, power method "
            f"{t_power * 1e3:.1f} ms, lambda_hat {lam:.6f}")
        U_first = U.clone()
        op.solve(labels, U_first, eps=p.eps, c=p.c, eta=p.eta, precond=p.precond,
                 outer=p.outer, sweeps=p.sweeps, delta0=p.delta0, lambda_max=lam,
                 step_k=p.step_k, stats=False)
        wall, ev_ms, stats = timed_solves(op, labels, U, p, lam, steps, warmup)
        Ut = torch.from_numpy(p.u0).to(dev, gl.TORCH_DTYPES[store_u]).contiguous()
        sweep_ms = gl.time_sweeps(op, labels, Ut, eps=p.eps, c=p.c, eta=p.eta,
                                  precond=p.precond, delta0=p.delta0, lambda_max=lam,
                                  step_k=p.step_k, reps=args.sweep_reps)
        info = op.info()
        B = sweep_bytes(info, p.n, p.K, store_u)
        Bm = method_bytes(info, p.n, p.K, store_w, store_u)
        res = {
            "solves_per_s": steps / wall,
            "ms_per_solve": wall / steps * 1e3,
            "ms_per_solve_events": ev_ms / steps,
            "sweep_kernel_ms": sweep_ms,
            "sweep_bytes": B,
            "sweep_bytes_method": Bm,
            "sweep_gbps": B / (sweep_ms * 1e-3) / 1e9,
            "operator_create_ms": t_create * 1e3,
            "power_method_ms": t_power * 1e3,
            "lambda_hat": lam,
            "layout": info["layout"],
            "stored_entries": info["stored_entries"],
            "halo_max": info["halo_max"],
            "halo_total": info["halo_total"],
        }
        labels_out = gl.assign_labels(U_first).cpu().numpy()
        op.close()
        return res, labels_out, U_first

    sw, su = p.store_w, p.store_u
    log(f"timing {sw}/{su}: {args.warmup} warmup + {args.steps} timed solves")
    main_res, lab_main, U_main = run_variant(sw, su, args.steps, args.warmup)
    fp32 = None
    if not args.no_fp32 and (sw, su) != ("f32", "f32"):
        log("timing f32/f32")
        fp32, lab32, _ = run_variant("f32", "f32", args.steps, args.warmup)
        fp32["label_agreement_with_main"] = float(np.mean(lab32 == lab_main))
        fp32 = {k: fp32[k] for k in ("solves_per_s", "ms_per_solve", "sweep_kernel_ms",
                                     "sweep_bytes", "sweep_gbps", "label_agreement_with_main",
                                     "power_method_ms", "layout")}
    acc = float(np.mean(lab_main == p.truth))

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import c_oracle
        rp, col, w = g.numpy()
        log("CPU oracle sample: whole solves of the same workload, about 10 s")
        lam_cpu = main_res["lambda_hat"]
        t0 = time.perf_counter()
        solves = 0
        while True:
            c_oracle.dca_solve(p.n, rp, col, w, p.labels, p.u0, eps=p.eps, c=p.c, eta=p.eta,
                               precond=p.precond, outer=p.outer, sweeps=p.sweeps,
                               delta0=p.delta0, lambda_max=lam_cpu, step_k=p.step_k,
                               record=True)
            solves += 1
            if time.perf_counter() - t0 >= 10.0 or solves >= 20:
                break
        t_cpu = time.perf_counter() - t0
        model = ""
        try:
            with open("/proc/cpuinfo") as fh:
                model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
        except OSError:
            pass
        # the numpy/scipy oracle on one thread: the time of 4 more sweeps
        # (runs of 1 and 5 sweeps in one DCA step, no energies)
        from threadpoolctl import threadpool_limits
        from oracle import gl_oracle
        kw1 = dict(eps=p.eps, c=p.c, eta=p.eta, precond=p.precond, delta0=p.delta0,
                   lambda_max=lam_cpu, step_k=p.step_k, record=False)
        log("CPU oracle sample, numpy/scipy on one thread: 1 and 5 sweeps")
        with threadpool_limits(1):
            ts = []
            for m in (1, 5):
                t1 = time.perf_counter()
                gl_oracle.dca_solve(p.n, rp, col, w, p.labels, p.u0, outer=1, sweeps=m, **kw1)
                ts.append(time.perf_counter() - t1)
        s1 = max(ts[1] - ts[0], 1e-9) / 4
        cpu = {"value": solves / t_cpu, "unit": "solves/s",
               "cores": c_oracle.num_threads(), "kind": "oracle",
               "sample": (f"{solves} whole solves ({p.outer} DCA steps x {p.sweeps} sweeps + "
                          f"energies, float64, C+OpenMP) on the full graph, {t_cpu:.1f} s"),
               "s_per_sweep": t_cpu / (solves * p.outer * p.sweeps),  # energies included
               "cpu_model": model, "host_cpus": os.cpu_count(),
               "scipy_1core": {"s_per_sweep": s1, "cores": 1,
                               "solves_per_s": 1.0 / (s1 * p.outer * p.sweeps),
                               "sample": (f"numpy/scipy float64 oracle, one thread: one DCA step "
                                          f"of 1 and of 5 sweeps on the full graph "
                                          f"({ts[0]:.1f} s, {ts[1]:.1f} s); per sweep = "
                                          f"difference / 4; solves/s excludes energies")}}

    log("unsupervised run (second eigenvector start)")
    unsup = unsupervised_bench(dev)
    log(f"  lambda2 {unsup['lambda2']:.4e} in {unsup['second_eigenpair_ms']:.1f} ms, solve "
        f"{unsup['solve_ms']:.1f} ms, accuracy {unsup['accuracy_vs_truth']:.4f}")

    window = None
    if not args.no_window:
        log("window graph (search window + patch weights, matrix-free operator)")
        window = window_bench(dev, args.steps, args.warmup, args.sweep_reps)
        log(f"  bf16 sweep {window['bf16']['sweep_kernel_ms'] * 1e3:.1f} us "
            f"({window['bf16']['sweep_gbps']:.0f} GB/s), f32 sweep "
            f"{window['f32']['sweep_kernel_ms'] * 1e3:.1f} us ({window['f32']['sweep_gbps']:.0f} GB/s)")

    log("kNN graph construction")
    kg = knn_graph_bench(dev)
    log(f"  {kg['points']} points: kNN {kg['knn_ms']:.1f} ms, graph {kg['graph_ms']:.1f} ms, "
        f"nnz {kg['nnz']}")

    pcmp = None
    if not args.no_precond:
        log("preconditioners, step sizes and L against L_s on the window graph")
        pcmp = precond_bench(dev)

    ceil = ceilings(dev)
    log(f"ceilings: read {ceil['read_gbps']:.0f} GB/s, copy {ceil['copy_gbps']:.0f} GB/s")
    hbm = None
    if not args.no_hbm_scale:
        log("grid sweep beyond the caches (4096 x 4096 image)")
        hbm = hbm_scale_bench(dev, args.sweep_reps)

    served = None
    if not args.no_served:
        served = served_bench(dev, args.served_count, args.served_rate, args.served_budget_gib,
                              args.served_slots)

    B = main_res["sweep_bytes"]
    achieved = main_res["sweep_gbps"]
    out = {
        "metric": METRIC,
        "value": main_res["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "storage": {"weights": sw, "field": su},
        "data": "synthetic",
        "config": {"workload": p.name, "n": p.n, "nnz": g.nnz, "K": p.K,
                   "outer_steps": p.outer, "sweeps": p.sweeps, "precond": p.precond,
                   "eps": p.eps, "c": p.c, "eta": p.eta,
                   "labelled_fraction": float(np.mean(p.labels >= 0))},
        "sweep_gbps": achieved,
        "sweep_kernel_ms": main_res["sweep_kernel_ms"],
        "per_graph_setup_ms": {"operator_create": main_res["operator_create_ms"],
                               "power_method_150": main_res["power_method_ms"]},
        "layout": {k: main_res[k] for k in ("layout", "stored_entries", "halo_max",
                                            "halo_total")},
        "accuracy_vs_ground_truth": acc,
        "fp32": fp32,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": recorded_traffic(p.name, f"{sw}/{su}"),
                     "kernel": {"tile": f"tile_sweep_kernel<{p.K}, {sw}, {su}>",
                                "grid": f"grid_sweep_kernel<{p.K}, {sw}, {su}>"}.get(
                                    main_res["layout"], "sweep_kernel"),
                     "bytes_per_launch": B,
                     "bytes_per_launch_method": main_res["sweep_bytes_method"],
                     "frac_method": main_res["sweep_bytes_method"]
                     / (main_res["sweep_kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                     "measured_ceiling_gbps": ceil["read_gbps"],
                     "frac_of_measured_ceiling": achieved / ceil["read_gbps"],
                     "timing": ("mean per launch of --sweep-reps plain sweeps (the kernel "
                                "named) back to back between one HIP event pair on their "
                                "stream; sweep 0 of each DCA step and the energy-only pass "
                                "run as grid_energy_sweep_kernel")},
        "ceilings": ceil,
        "hbm_scale": hbm,
        "precond_comparison": pcmp,
        "cpu_baseline": cpu,
        "served": served,
        "unsupervised": unsup,
        "window_graph": window,
        "knn_graph": kg,
    }
    print(json.dumps(out), flush=True)
    if args.calib_copy:
        calib_copy(dev)


if __name__ == "__main__":
    main()
