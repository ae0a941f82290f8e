"""Benchmark of the phase-field DUGKS step on one MI355X.

Default workload: the coupled (Allen-Cahn + hydrodynamics) stationary bubble,
128 x 128 periodic, R = 32, density ratio 1000, sigma = 1e-3, nu = 0.1,
M = 0.1, FP32 step (Sec. IV.A of arXiv:1810.07802). One benchmark step is one
DUGKS time step of the whole grid; `--steps` of them are timed after
`--warmup` untimed ones, replayed from a HIP graph on the stream that the
HIP events time. `value` is MLUPS = cells * steps / s / 1e6.

The same JSON line carries:
  roofline      HBM roofline of the step kernel at this workload (algorithmic
                bytes: 160 B per cell and step in FP32)
  large_grid    the same physics on 4096 x 4096 (R = 1024), where the working
                set (2.8 GB) is far larger than the 256 MB Infinity Cache, with
                the bandwidth a plain 16-byte copy of the same bytes reaches
                (copy_ceiling) and the step's fraction of it
  batched       the spinodal batch (64 cases of 64^2..512^2): one graph of
                batched launches vs one launch per case per step
  served        the served request stream through the continuous-batching
                pool: p50 / p99 time to solution at 80 % load, aggregate
                MLUPS, vs the plain sequential per-case loop
  upwind        the same bubble with the upwind, limited face reconstruction
                (two kernels per step, 516 algorithmic bytes per cell in
                FP32), 128^2 and 4096^2, launched step by step
  mesh          the 4096^2 bubble on a stretched mesh (widths 1 +- 0.3 sin),
                central and upwind, through the same two kernels
  cpu_baseline  the FP64 C oracle on the host cores, on a bounded sample
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
B_PER_CELL = {"fp32": 160.0, "fp64": 320.0}  # read + write of 18 populations + 2 history values
# upwind reconstruction / stretched mesh, coupled, FP32: stage 260 (21 state
# values in; tilde-plus and history, 20 values, out; 18 bar-plus + 6 face
# inputs out), faces and update 256 (18 bar-plus + 5 face inputs + 20 state
# values in, 21 values out) bytes per cell
B_UPWIND = {"fp32": 516.0, "fp64": 1032.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--large-steps", type=int, default=200)
    ap.add_argument("--large-seg", type=int, default=0,
                    help="tile (rows per segment) of the 4096x4096 leg; 0: the library's autotuner")
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--serve-requests", type=int, default=60,
                    help="requests of the served stream (0: skip the serving leg)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--skip-extra", action="store_true", help="only the default workload")
    ap.add_argument("--profile-batch", action="store_true",
                    help="run only the batched spinodal leg (one graph per chunk, "
                         "autotuned tiles): for kernel traces")
    ap.add_argument("--profile-kernel", action="store_true",
                    help="run only the timed default workload (for profilers)")
    ap.add_argument("--profile-large", action="store_true",
                    help="run only the timed 4096x4096 workload (for profilers)")
    ap.add_argument("--profile-upwind", action="store_true",
                    help="only the upwind leg on 4096^2 (for rocprofv3)")
    ap.add_argument("--profile-mesh", action="store_true",
                    help="only the stretched-mesh central leg on 4096^2 (for rocprofv3)")
    ap.add_argument("--upwind-steps", type=int, default=50)
    ap.add_argument("--profile-copy", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (calibrates the "
                         "HBM byte counters)")
    return ap.parse_args()


def copy_ceiling(torch, D, nbytes, reps=10):
    """HBM bandwidth of the library's plain copy (one 16-byte load and store per
    work item) over `nbytes` read and `nbytes` written, timed with HIP events on
    the stream it runs on: what a streaming kernel reaches on this device."""
    n = max(4, nbytes // 16 * 4)  # float32 elements, a multiple of 16 bytes
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    nb = 4 * n
    for _ in range(3):
        D.copy_probe(dst.data_ptr(), src.data_ptr(), nb, stream.cuda_stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        D.copy_probe(dst.data_ptr(), src.data_ptr(), nb, stream.cuda_stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return {"GBps": round(2 * nb / t / 1e9, 1), "bytes_read": nb, "bytes_written": nb,
            "us": round(t * 1e6, 1)}


def timed_graph(torch, D, solvers, steps, warmup, chunk=1000, autotune=False):
    """Replay `steps` steps of `solvers` (a batch) from HIP graphs of `chunk`
    launches on torch's current stream; returns seconds measured by HIP events
    on that stream. With `autotune`, the batch's tiles are picked by the
    library's autotuner first (outside the timed region)."""
    stream = torch.cuda.current_stream()
    b = D.Batch(solvers)
    b.set_stream(stream.cuda_stream)
    b.tiles = b.autotune(5) if autotune else None
    chunk = max(1, min(chunk, steps))
    w = warmup
    while w > 0:
        n = min(chunk, w)
        b.step(n, use_graph=True)
        w -= n
    # make sure every graph used in the timed region is already instantiated
    rest = steps % chunk
    if rest:
        b.step(rest, use_graph=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    left = steps
    while left > 0:
        n = min(chunk, left)
        b.step(n, use_graph=True)
        left -= n
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3, b


def timed_eager(torch, D, solvers, steps):
    """One launch per case per step (the plain per-case loop)."""
    stream = torch.cuda.current_stream()
    for s in solvers:
        s.set_stream(stream.cuda_stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for s in solvers:
        s.step(steps)  # `steps` launches of the step kernel for this case
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


def counter_traffic(workload):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's
    reading), or None when the kernel sources differ from the profiled ones."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_step_hbm_counters.txt")
    if workload is None or not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in ("dugks_kernels.hip", "dugks_impl.h"):
        with open(os.path.join(ROOT, "paper_1810_07802_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    sha, val = None, None
    for line in open(path):
        w = line.split()
        if len(w) >= 2 and w[0] == "kernel_source_sha256":
            sha = w[1]
        if len(w) >= 2 and w[0] == "workload" and w[1] == workload:
            val = float(w[w.index("bytes_per_launch") + 1])
    return val if sha == h.hexdigest() else None


def roofline(cells, steps, seconds, prec, workload=None):
    per_launch = B_PER_CELL[prec] * cells
    t_launch = seconds / steps
    achieved = per_launch / t_launch / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(workload),
            "bytes_per_launch": per_launch, "launch_us": round(t_launch * 1e6, 3)}


def timed_upwind(torch, D, c, steps, warmup, recon="upwind", mesh=None, chunk=100):
    """Two-kernel steps of case `c` (coupled FP32): the upwind
    reconstruction, or a stretched mesh `mesh` = (dx, dy) in either
    reconstruction, on torch's current stream in calls of `chunk` steps (the
    library replays each call from a HIP graph recorded on first use; the
    warm-up records every sequence length the timed region uses); seconds by
    HIP events on that stream."""
    stream = torch.cuda.current_stream()
    s = D.Solver(c["nx"], c["ny"], dict(c["params"], recon=recon), "coupled", "fp32")
    s.set_stream(stream.cuda_stream)
    if mesh is not None:
        s.set_mesh(*mesh)
    s.init(c["phi"])
    chunk = max(1, min(chunk, steps))
    s.step(max(warmup, chunk))
    if steps % chunk:
        s.step(steps % chunk)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    left = steps
    while left > 0:
        n = min(chunk, left)
        s.step(n)
        left -= n
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3
    d = s.diagnostics()
    cells = c["nx"] * c["ny"]
    ach = B_UPWIND["fp32"] * cells * steps / t / 1e9
    return {"mlups": round(cells * steps / t / 1e6, 1), "steps": steps,
            "us_per_step": round(t / steps * 1e6, 3), "bytes_per_cell": B_UPWIND["fp32"],
            "achieved_GBps": round(ach, 1), "frac_hbm": round(ach / HBM_PEAK_GBS, 4),
            "nonfinite": d["nonfinite"]}


def served_stream(torch, D, W, n_req):
    """The served request stream: closed-loop capacity, then Poisson arrivals
    at 80 % of it (p50 / p99 time to solution, aggregate MLUPS), then the
    plain sequential per-case loop on the same requests."""
    import numpy as np
    from paper_1810_07802_amd import serve
    cases = W.served_stream(n=n_req)
    lups = [c["nx"] * c["ny"] * c["steps"] for c in cases]
    mean_lups = float(np.mean(lups))

    def pool():
        p = D.Pool(8 << 30, max_cases=32, max_cells=1024 * 1024)
        p.set_stream(torch.cuda.current_stream().cuda_stream)
        return p

    warm = [serve.Request(0, W.bubble(L=64, steps=0), 200, 0.0)]
    serve.run(pool(), warm, chunk=100)
    # closed loop: everything queued at t = 0
    reqs = [serve.Request(k, c, c["steps"], 0.0) for k, c in enumerate(cases)]
    closed = serve.summary(serve.run(pool(), reqs, chunk=200))
    cap = closed["mlups"] * 1e6  # LUP/s
    rate = 0.8 * cap / mean_lups  # requests per second
    arr = np.cumsum(np.random.default_rng(7802).exponential(1.0 / rate, size=len(cases)))
    reqs = [serve.Request(k, c, c["steps"], float(arr[k])) for k, c in enumerate(cases)]
    opened = serve.summary(serve.run(pool(), reqs, chunk=200))
    # the plain sequential per-case loop: create, init, step, read out, one case at a time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in cases:
        s = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
        s.init(c["phi"], c.get("u"), c.get("v"), c.get("p"))
        s.step(c["steps"])
        s.macros()
        del s
    seq = time.perf_counter() - t0
    return {"workload": f"{len(cases)} requests: layered Poiseuille (mu ratio 100, nx 64, ny 64..1024) "
                        "and stationary bubbles (64^2..1024^2), 1k-20k steps each (seed 7802), FP32, "
                        "pool of 32 slots and an 8 GiB arena",
            "closed_loop_mlups": round(closed["mlups"], 1),
            "arrival_rate_per_s": round(rate, 3), "load": 0.8,
            "served_mlups": round(opened["mlups"], 1),
            "p50_s": round(opened["p50_s"], 4), "p99_s": round(opened["p99_s"], 4),
            "sequential_mlups": round(sum(lups) / seq / 1e6, 1)}


def cpu_baseline(budget_s):
    """The FP64 oracle on the host: the bubble 128^2 for about 3/4 of the
    budget on all OpenMP threads, then about 1/4 on one thread."""
    import ctypes
    import oracle
    import workloads as W
    c = W.bubble(L=128, R=32)
    s = oracle.Sim(c["nx"], c["ny"], c["params"], "coupled")
    s.init(c["phi"])
    s.step(5)

    def rate(seconds):
        n, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            s.step(10)
            n += 10
        dt = time.perf_counter() - t0
        return c["nx"] * c["ny"] * n / dt / 1e6, n, dt

    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    v, n, dt = rate(0.75 * budget_s)
    one = None
    try:  # the oracle library links the OpenMP runtime
        omp = ctypes.CDLL(oracle._LIB_PATH)
        omp.omp_set_num_threads(1)
        one = rate(0.25 * budget_s)[0]
        omp.omp_set_num_threads(cores)
    except (OSError, AttributeError):
        pass
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(v, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"bubble 128x128 coupled FP64, {n} steps ({dt:.1f} s) on {cores} threads",
            "single_thread_value": None if one is None else round(one, 3),
            "cpu_model": model}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1810_07802_amd as D
    import workloads as W

    torch.cuda.set_device(0)
    # a created stream (default priority) as torch's current stream: the library
    # captures its HIP graphs on the caller's stream, and the null stream that
    # torch uses by default cannot be captured
    torch.cuda.set_stream(torch.cuda.Stream())
    if args.profile_copy:
        n = 1 << 28  # float32 elements: 1 GiB read + 1 GiB written per copy
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3 / 5
        print(json.dumps({"workload": "device copy 1 GiB", "bytes_read": 4 * n, "bytes_written": 4 * n,
                          "copy_GBps": round(8 * n / t / 1e9, 1)}), flush=True)
        return
    if args.profile_large:
        cl = W.bubble(L=4096, R=1024, steps=0)
        sl = D.Solver(cl["nx"], cl["ny"], cl["params"], "coupled", "fp32", args.large_seg or None)
        sl.init(cl["phi"])
        seg = sl.seg_rows if args.large_seg else sl.autotune(10)[0]
        tl, _ = timed_graph(torch, D, [sl], args.large_steps, 5, chunk=args.large_steps)
        ncl = cl["nx"] * cl["ny"]
        print(json.dumps({"workload": "bubble 4096x4096 coupled FP32", "steps": args.large_steps,
                          "seg_rows": seg, "mlups": round(ncl * args.large_steps / tl / 1e6, 1),
                          "roofline": roofline(ncl, args.large_steps, tl, "fp32", "bubble4096")}), flush=True)
        return
    if args.profile_mesh:
        cl = W.bubble(L=4096, R=1024, steps=0)
        mesh = (W.stretched_widths(4096, 0.3), W.stretched_widths(4096, 0.3, phase=1.0))
        print(json.dumps({"workload": "bubble 4096x4096 coupled FP32, stretched mesh, central",
                          **timed_upwind(torch, D, cl, args.upwind_steps, 3, "central", mesh)}),
              flush=True)
        return
    if args.profile_batch:
        cases = W.spinodal_batch(steps=0)
        solvers = []
        for cc in cases:
            t = D.Solver(cc["nx"], cc["ny"], cc["params"], "coupled", "fp32")
            t.init(cc["phi"])
            solvers.append(t)
        bc = sum(cc["nx"] * cc["ny"] for cc in cases)
        tb, bt = timed_graph(torch, D, solvers, args.batch_steps, 20, chunk=100, autotune=True)
        print(json.dumps({"workload": "spinodal batch, 64 cases of 64^2..512^2 (seed 1810), coupled FP32",
                          "cells": bc, "steps": args.batch_steps, "tile_seg_rows": bt.tiles,
                          "batched_graph_mlups": round(bc * args.batch_steps / tb / 1e6, 1),
                          "roofline": roofline(bc, args.batch_steps, tb, "fp32")}), flush=True)
        return
    if args.profile_upwind:
        cl = W.bubble(L=4096, R=1024, steps=0)
        print(json.dumps({"workload": "bubble 4096x4096 coupled FP32, upwind reconstruction",
                          **timed_upwind(torch, D, cl, args.upwind_steps, 3)}), flush=True)
        return
    c = W.bubble(L=128, R=32)
    cells = c["nx"] * c["ny"]
    s = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
    s.init(c["phi"])
    secs, batch = timed_graph(torch, D, [s], args.steps, args.warmup)
    mlups = cells * args.steps / secs / 1e6
    rec = {
        "metric": "MLUPS (coupled AC+hydro step, FP32) + %HBM peak; batched vs plain; p50/p99 solve latency",
        "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(secs / args.steps * 1e3, 6),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "stationary bubble 128x128, R=32, W=5, rho 1000:1, sigma=1e-3, "
                               "nu=0.1, M=0.1, periodic, coupled FP32 step",
                   "nx": c["nx"], "ny": c["ny"], "seg_rows": s.seg_rows,
                   "launch": "HIP graph of 1000 step launches"},
        "roofline": roofline(cells, args.steps, secs, "fp32", "bubble128"),
    }
    diag = s.diagnostics()
    rec["check"] = {"nonfinite": diag["nonfinite"], "max_u": diag["max_u"]}
    if args.profile_kernel:
        print(json.dumps(rec), flush=True)
        return
    if not args.skip_extra:
        # the same step launched one kernel at a time from the host
        e_steps = min(args.steps, 2000)
        t_e = timed_eager(torch, D, [s], e_steps)
        rec["plain_launch_mlups"] = round(cells * e_steps / t_e / 1e6, 2)
        # FP64 on the same workload
        s64 = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp64")
        s64.init(c["phi"])
        t64, _ = timed_graph(torch, D, [s64], min(args.steps, 5000), 100)
        rec["fp64_mlups"] = round(cells * min(args.steps, 5000) / t64 / 1e6, 2)
        del s64
        # large grid: HBM-resident working set
        cl = W.bubble(L=4096, R=1024, steps=0)
        sl = D.Solver(cl["nx"], cl["ny"], cl["params"], "coupled", "fp32")
        sl.init(cl["phi"])
        auto_seg = sl.seg_rows
        if args.large_seg:
            sl.set_tile(args.large_seg)
        else:
            sl.autotune(10)  # tile chosen by the library's autotuner (outside the timed region)
        tl, _ = timed_graph(torch, D, [sl], args.large_steps, 20, chunk=100)
        ncl = cl["nx"] * cl["ny"]
        rec["large_grid"] = {"workload": "stationary bubble 4096x4096, R=1024, coupled FP32",
                             "mlups": round(ncl * args.large_steps / tl / 1e6, 1),
                             "steps": args.large_steps, "seg_rows": sl.seg_rows,
                             "auto_seg_rows": auto_seg,
                             "roofline": roofline(ncl, args.large_steps, tl, "fp32", "bubble4096")}
        del sl
        # the same bytes per launch through a plain copy: the practical ceiling
        cc_ = copy_ceiling(torch, D, int(B_PER_CELL["fp32"] / 2 * ncl))
        lg = rec["large_grid"]
        lg["copy_ceiling"] = cc_
        lg["frac_of_copy"] = round(lg["roofline"]["achieved"] / cc_["GBps"], 4)
        # batched spinodal workload vs the per-case loop
        cases = W.spinodal_batch(steps=0)
        solvers = []
        for cc in cases:
            t = D.Solver(cc["nx"], cc["ny"], cc["params"], "coupled", "fp32")
            t.init(cc["phi"])
            solvers.append(t)
        bc = sum(cc["nx"] * cc["ny"] for cc in cases)
        tb_auto, _ = timed_graph(torch, D, solvers, args.batch_steps, 20, chunk=100)
        tb, bt = timed_graph(torch, D, solvers, args.batch_steps, 20, chunk=100, autotune=True)
        tp = timed_eager(torch, D, solvers, args.batch_steps)
        rec["batched"] = {"workload": "spinodal decomposition, 64 cases of 64^2..512^2 "
                                      "(seed 1810), rho 1000:1, coupled FP32",
                          "cells": bc, "steps": args.batch_steps,
                          "batched_graph_mlups": round(bc * args.batch_steps / tb / 1e6, 1),
                          "batched_graph_auto_tile_mlups": round(bc * args.batch_steps / tb_auto / 1e6, 1),
                          "tile_seg_rows": bt.tiles,
                          "per_case_loop_mlups": round(bc * args.batch_steps / tp / 1e6, 1),
                          "roofline": roofline(bc, args.batch_steps, tb, "fp32")}
        del solvers
        # upwind, limited reconstruction on the same physics
        rec["upwind"] = {
            "workload": "stationary bubble, coupled FP32, upwind reconstruction, two "
                        "kernels per step, replayed from HIP graphs of up to 100 steps",
            "bubble128": timed_upwind(torch, D, c, min(args.steps, 5000), 100),
            "bubble4096": timed_upwind(torch, D, W.bubble(L=4096, R=1024, steps=0),
                                       args.upwind_steps, 5)}
        # stretched tensor-product mesh, both reconstructions
        cm = W.bubble(L=4096, R=1024, steps=0)
        mesh = (W.stretched_widths(4096, 0.3), W.stretched_widths(4096, 0.3, phase=1.0))
        rec["mesh"] = {
            "workload": "stationary bubble 4096x4096 on a stretched mesh (widths 1 + 0.3 sin, "
                        "both axes), coupled FP32, two kernels per step, replayed from HIP "
                        "graphs of up to 100 steps",
            "central": timed_upwind(torch, D, cm, args.upwind_steps, 5, "central", mesh),
            "upwind": timed_upwind(torch, D, cm, args.upwind_steps, 5, "upwind", mesh)}
        if args.serve_requests > 0:
            rec["served"] = served_stream(torch, D, W, args.serve_requests)
        rec["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
